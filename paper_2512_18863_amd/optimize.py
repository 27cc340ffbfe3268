"""Gradient-based plan optimisation with the dose engine as a differentiable layer.

The loop of §2.5 (gradient-based optimisation from closed apertures):
unconstrained leaf, jaw and MU variables are projected to machine-feasible
values (§2.2.1, `ProjectFunction`, straight-through gradient), mapped to dose by
the HIP engine (`DoseFunction`), scored by a dose objective, and updated by
Adam.  Two objectives:

* "l1", the paper's weighted sum (§2.5):
      L = lambda_PTV |D_PTV - D_rx|_1 + sum_s lambda_s |D_s|_1,
  evaluated with its gradient by the library's `pdrt_l1_objective`
  (`plan_eval.L1Objective`); the weights are chosen by `weight_search`, which
  keeps the combination whose plan has the highest Dice coefficient between the
  100 % isodose volume and the PTV;
* "quadratic", the synthetic prostate workload's own objective
      L = mean_PTV (D - 78)^2 + mean_rectum max(0, D - 70)^2 + max(0, mean_bladder D - 40)^2.

Optimisation can run in stages of growing kernel size ("smaller kernel sizes
first", §4): each stage has its own engine, and with `cache` set each engine
keeps the plan's geometry cache (depths and (SAD/d)^2 DD(W) for every control
point), so its steps skip the ray march.  Every dose, gradient and objective
evaluation runs in the HIP library; Adam's update is torch's.
"""
from __future__ import annotations

import itertools
import time
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import engine as E
from . import inputs
from . import plan_eval


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


@dataclass
class Stage:
    """steps Adam steps with an engine of n_taps x n_taps kernels."""
    steps: int
    n_taps: Optional[int] = None          # None: the case's own kernel size
    conv: str = "fp32"
    cache: Optional[str] = "fp32"         # geometry cache kind, or None for the ray march


class PlanOptimizer:
    def __init__(self, case, masks, limits: Limits = Limits(), lr_pos: float = 0.5, lr_mu: float = 1.0,
                 conv: str = "fp32", objective: str = "quadratic", weights: Optional[Dict[str, float]] = None,
                 rx: float = 78.0, target: str = "ptv", cache: Optional[str] = None):
        self.case = case
        self.conv = conv
        self._engines = {}
        self.eng = self.engine(case.n_taps, conv, cache)
        dev = self.eng.device
        self.masks = {k: torch.tensor(v, device=dev) for k, v in masks.items()}
        self.limits = limits.as_dict()
        self.objective = objective
        self.rx = rx
        self.names = list(masks)
        self.evaluator = plan_eval.Evaluator([masks[n] for n in self.names], self.names, device=dev)
        self.target_index = self.names.index(target) if target in self.names else None
        if objective == "l1":
            w = weights if weights is not None else {target: 100.0}
            self.l1_weights = [float(w.get(n, 0.0)) for n in self.names]
            self.l1_targets = [rx if n == target else 0.0 for n in self.names]
        elif objective != "quadratic":
            raise ValueError("objective is 'l1' or 'quadratic'")
        self.leaves = torch.tensor(case.leaves, dtype=torch.float32, device=dev, requires_grad=True)
        self.jaws = torch.tensor(case.jaws, dtype=torch.float32, device=dev, requires_grad=True)
        self.mu = torch.tensor(case.mu, dtype=torch.float32, device=dev, requires_grad=True)
        self.opt = torch.optim.Adam([{"params": [self.leaves, self.jaws], "lr": lr_pos},
                                     {"params": [self.mu], "lr": lr_mu}])

    def engine(self, n_taps: Optional[int], conv: str, cache: Optional[str]) -> "E.DoseEngine":
        """The engine for one kernel size / precision (built once, cache built once)."""
        n = self.case.n_taps if n_taps is None else n_taps
        key = (n, conv, cache)
        if key not in self._engines:
            eng = E.DoseEngine(self.case, n_taps=n, conv=conv)
            if cache:
                eng.build_cache(cache)
            self._engines[key] = eng
        return self._engines[key]

    def projected(self):
        return E.ProjectFunction.apply(self.leaves, self.jaws, self.mu, self.limits, True)

    def loss_of(self, dose: torch.Tensor) -> torch.Tensor:
        if self.objective == "l1":
            return plan_eval.L1Objective.apply(dose, self.evaluator, self.l1_weights, self.l1_targets)
        return objective(dose, self.masks)

    def step(self) -> torch.Tensor:
        self.opt.zero_grad(set_to_none=True)
        lv, jw, mu = self.projected()
        dose = self.eng(lv, jw, mu)
        loss = self.loss_of(dose)
        loss.backward()
        self.opt.step()
        return loss

    def run(self, steps: int):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        losses = [float(self.step().detach()) for _ in range(steps)]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return losses, dt / max(steps, 1)

    def run_stages(self, stages: Sequence[Stage]):
        """Coarse-to-fine: each stage switches engine, keeping parameters and Adam state.
        Returns [(stage, losses, seconds per step)]."""
        out = []
        for st in stages:
            self.eng = self.engine(st.n_taps, st.conv, st.cache)
            losses, sec = self.run(st.steps)
            out.append((st, losses, sec))
        return out

    def final(self, engine: Optional["E.DoseEngine"] = None):
        eng = self.eng if engine is None else engine
        with torch.no_grad():
            lv, jw, mu = E.project_params(self.leaves.detach(), self.jaws.detach(), self.mu.detach(), self.limits)
            dose = eng.forward(lv, jw, mu)
            return (lv.cpu().numpy().astype(np.float64), jw.cpu().numpy().astype(np.float64),
                    mu.cpu().numpy().astype(np.float64), dose)

    def dice(self, dose: torch.Tensor) -> float:
        """Dice of the 100 % isodose volume {D >= rx} with the target structure."""
        return self.evaluator.dice(dose.contiguous(), self.target_index, self.rx)


def weight_search(case, masks, oars: Sequence[str], stages: Sequence[Stage], rx: float,
                  lambdas: Sequence[float] = (0.0, 0.1, 1.0, 10.0, 100.0), target: str = "ptv",
                  target_weight: float = 100.0, combos: Optional[List[Dict[str, float]]] = None, **kw):
    """The paper's weight selection (§2.5): lambda_PTV fixed, every combination of
    OAR weights from `lambdas` (or the given `combos`) optimised from the closed
    start, and the plan with the highest isodose / PTV Dice kept.
    Returns (best weights, best Dice, [(weights, Dice, final loss)])."""
    if combos is None:
        combos = [dict(zip(oars, c)) for c in itertools.product(lambdas, repeat=len(oars))]
    results = []
    for c in combos:
        w = dict(c)
        w[target] = target_weight
        opt = PlanOptimizer(case, masks, objective="l1", weights=w, rx=rx, target=target, **kw)
        runs = opt.run_stages(stages)
        dose = opt.final()[3]
        results.append((w, opt.dice(dose), runs[-1][1][-1]))
    best = max(results, key=lambda r: r[1])
    return best[0], best[1], results
