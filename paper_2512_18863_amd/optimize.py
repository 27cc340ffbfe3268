"""Gradient-based plan optimisation with the dose engine as a differentiable layer.

The loop of §2.5 / §3.4 (gradient-based optimisation from closed apertures):
unconstrained leaf, jaw and MU variables are projected to machine-feasible
values (§2.2.1, `ProjectFunction`, straight-through gradient), mapped to dose by
the HIP engine (`DoseFunction`), scored by a dose objective, and updated by
Adam.  The objective of the synthetic prostate workload is quadratic:

    L = mean_PTV (D - 78)^2 + mean_rectum max(0, D - 70)^2 + max(0, mean_bladder D - 40)^2

(the paper's own study used a weighted L1 objective, §2.5; the quadratic form is
the workload's choice).  The objective and Adam run as ordinary torch ops on the
dose tensor, as a user of the engine would write them; every dose and gradient
evaluation runs in the HIP library.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import torch

from . import engine as E
from . import inputs


@dataclass
class Limits:
    leaf: float = 50.0       # leaf-pair centre travel, mm
    jaw_x: float = 50.0
    jaw_y: float = 50.0
    w_min: float = 1.0       # minimum opening, mm
    mu_min: float = 0.22     # Eq. 3 with 20 MU/min, 6 deg/s, 4 deg spacing

    def as_dict(self):
        return {"leaf": self.leaf, "jaw_x": self.jaw_x, "jaw_y": self.jaw_y, "w_min": self.w_min,
                "mu_min": self.mu_min}


def mu_floor(dose_rate_min_mu_per_min: float, gantry_speed_max_deg_per_s: float, spacing_deg: float) -> float:
    """Minimum MU per control point, Eq. 3: eps = Ddot_min * dphi / phidot_max."""
    return (dose_rate_min_mu_per_min / 60.0) * spacing_deg / gantry_speed_max_deg_per_s


def objective(dose: torch.Tensor, masks: dict, rx: float = 78.0, rect_max: float = 70.0,
              bladder_mean: float = 40.0) -> torch.Tensor:
    ptv = dose[masks["ptv"]]
    rect = dose[masks["rectum"]]
    blad = dose[masks["bladder"]]
    return (((ptv - rx) ** 2).mean() + (torch.clamp(rect - rect_max, min=0.0) ** 2).mean()
            + torch.clamp(blad.mean() - bladder_mean, min=0.0) ** 2)


def c3_case():
    """The optimisation workload: the two-arc 192 x 192 x 128 geometry at 2.5 mm,
    31 x 31 kernel, calib 0.01 Gy/MU, closed start."""
    case = inputs.config_c2()
    case.machine.calib = 0.01
    case.field_limit = (50.0, 50.0)
    n, L = case.n_cp, case.machine.n_leaf
    case.leaves = np.zeros((n, 2, L))
    case.jaws = inputs.jaws_square(n, 40.0, 40.0)
    case.mu = np.zeros(n)
    return case


class PlanOptimizer:
    def __init__(self, case, masks, limits: Limits = Limits(), lr_pos: float = 0.5, lr_mu: float = 1.0,
                 conv: str = "fp32"):
        self.case = case
        self.eng = E.DoseEngine(case, conv=conv)
        dev = self.eng.device
        self.masks = {k: torch.tensor(v, device=dev) for k, v in masks.items()}
        self.limits = limits.as_dict()
        self.leaves = torch.tensor(case.leaves, dtype=torch.float32, device=dev, requires_grad=True)
        self.jaws = torch.tensor(case.jaws, dtype=torch.float32, device=dev, requires_grad=True)
        self.mu = torch.tensor(case.mu, dtype=torch.float32, device=dev, requires_grad=True)
        self.opt = torch.optim.Adam([{"params": [self.leaves, self.jaws], "lr": lr_pos},
                                     {"params": [self.mu], "lr": lr_mu}])

    def projected(self):
        return E.ProjectFunction.apply(self.leaves, self.jaws, self.mu, self.limits, True)

    def step(self) -> float:
        self.opt.zero_grad(set_to_none=True)
        lv, jw, mu = self.projected()
        dose = self.eng(lv, jw, mu)
        loss = objective(dose, self.masks)
        loss.backward()
        self.opt.step()
        return loss

    def run(self, steps: int):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        losses = [float(self.step()) for _ in range(steps)]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return losses, dt / max(steps, 1)

    def final(self):
        with torch.no_grad():
            lv, jw, mu = E.project_params(self.leaves.detach(), self.jaws.detach(), self.mu.detach(), self.limits)
            dose = self.eng.forward(lv, jw, mu)
            return (lv.cpu().numpy().astype(np.float64), jw.cpu().numpy().astype(np.float64),
                    mu.cpu().numpy().astype(np.float64), dose)
