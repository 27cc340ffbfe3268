"""Automatic output calibration (§2.4, commissioning).

The engine's dose per MU is scaled so that a reference number of MU gives 1 Gy
at reference conditions: a 10 cm x 10 cm field, 10 cm depth in water, source-to-
surface distance 90 cm.  The dose is computed by the engine itself in a virtual
water phantom; the returned factor is the `calib` (dose per MU) that makes
D(reference point) = 1 Gy per `ref_mu` MU.
"""
from __future__ import annotations

import numpy as np

from . import inputs


def reference_dose(dose_zyx, ref) -> float:
    """Dose at the reference point from a [nz][ny][nx] array (linear in y)."""
    ix, j, iz, w = ref
    return float((1.0 - w) * dose_zyx[iz, j, ix] + w * dose_zyx[iz, j + 1, ix])


def central_axis_pdd(dose_zyx, case):
    """Depth (mm, from the entrance face) and dose along the central axis of a
    gantry-0 reference case, normalised to its maximum."""
    nz, ny, nx = dose_zyx.shape
    ix = int(round(-case.origin[0] / case.spacing[0]))
    iz = int(round(-case.origin[2] / case.spacing[2]))
    d = np.asarray(dose_zyx[iz, :, ix], dtype=np.float64)
    depth = (np.arange(ny) + 0.5) * case.spacing[1]
    return depth, d / d.max()


def lateral_profile(dose_zyx, case, depth_mm: float):
    """Off-axis position (mm) and dose along x at a depth below the entrance face,
    normalised to the central-axis value (linear interpolation in y)."""
    ny = dose_zyx.shape[1]
    iz = int(round(-case.origin[2] / case.spacing[2]))
    t = depth_mm / case.spacing[1] - 0.5           # voxel j's centre lies (j + 1/2) s below the face
    j = int(np.clip(np.floor(t), 0, ny - 2))
    w = t - j
    row = (1 - w) * np.asarray(dose_zyx[iz, j, :], np.float64) + w * np.asarray(dose_zyx[iz, j + 1, :], np.float64)
    x = case.origin[0] + np.arange(row.size) * case.spacing[0]
    ic = int(round(-case.origin[0] / case.spacing[0]))
    return x, row / row[ic]


def calibrate(machine: inputs.Machine, n_taps: int = 61, ref_mu: float = 1.0, spacing: float = 2.0,
              device="cuda") -> float:
    """Dose per MU such that ref_mu MU give 1 Gy at the reference point, from one
    forward pass of the HIP engine with unit calibration."""
    import dataclasses

    import torch

    from . import engine as E
    case, ref = inputs.reference_case(dataclasses.replace(machine, calib=1.0), n_taps, spacing)
    eng = E.DoseEngine(case, device=device, calib=1.0)
    t = lambda a: torch.tensor(a, dtype=torch.float32, device=eng.device)
    dose = eng.forward(t(case.leaves), t(case.jaws), t(case.mu)).cpu().numpy()
    return 1.0 / (ref_mu * reference_dose(dose, ref))
