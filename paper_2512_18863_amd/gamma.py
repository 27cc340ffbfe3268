"""Global 3-D gamma pass rate (the agreement metric of §2.5 / §3.2).

gamma(x_r) = min over x_e of sqrt(|x_e - x_r|^2 / dta^2 + (D_e(x_e) - D_r(x_r))^2 / (dd * max D_r)^2),
evaluated on reference voxels with D_r >= cutoff * max D_r.  A point farther than
dta already gives gamma > 1, so the search is exactly confined to the dta ball;
it is sampled on a lattice of step dta * step_frac with D_e trilinear and zero
outside the grid (the engine's own convention for samples past the CT), nearest
points first, stopping at the first point with gamma <= 1.  Runs on the host
(numpy / scipy): an evaluation tool, not part of the dose path.
"""
from __future__ import annotations

import numpy as np
import scipy.ndimage


def pass_rate(ref: np.ndarray, ev: np.ndarray, spacing, dose_pct: float = 1.0, dta_mm: float = 1.0,
              cutoff: float = 0.1, step_frac: float = 0.1, mask=None, chunk: int = 1 << 20) -> float:
    ref = np.asarray(ref, dtype=np.float64)
    ev = np.asarray(ev, dtype=np.float64)
    assert ref.shape == ev.shape
    sx, sy, sz = spacing                       # arrays are [z][y][x]
    dmax = ref.max()
    tol = dose_pct / 100.0 * dmax
    sel = ref >= cutoff * dmax
    if mask is not None:
        sel &= mask
    n_sel = int(sel.sum())
    if n_sel == 0:
        return 1.0
    idx = np.nonzero(sel)
    failing = np.abs(ev[idx] - ref[idx]) > tol
    zz, yy, xx = (a[failing].astype(np.float64) for a in idx)
    rr = ref[idx][failing]
    if zz.size == 0:
        return 1.0
    st = dta_mm * step_frac
    n = int(np.floor(1.0 / step_frac + 1e-9))
    g = np.arange(-n, n + 1) * st
    oz, oy, ox = np.meshgrid(g, g, g, indexing="ij")
    r2 = (ox ** 2 + oy ** 2 + oz ** 2) / dta_mm ** 2
    keep = (r2 <= 1.0 + 1e-12) & (r2 > 0)
    order = np.argsort(r2[keep], kind="stable")
    offs = np.stack([oz[keep][order], oy[keep][order], ox[keep][order]], axis=1)
    rad = r2[keep][order]
    for (dz, dy, dx), d2 in zip(offs, rad):
        if zz.size == 0:
            break
        still = np.ones(zz.size, dtype=bool)
        for a in range(0, zz.size, chunk):
            b = min(zz.size, a + chunk)
            coords = np.stack([zz[a:b] + dz / sz, yy[a:b] + dy / sy, xx[a:b] + dx / sx])
            val = scipy.ndimage.map_coordinates(ev, coords, order=1, mode="grid-constant", cval=0.0)
            still[a:b] = d2 + ((val - rr[a:b]) / tol) ** 2 > 1.0
        zz, yy, xx, rr = zz[still], yy[still], xx[still], rr[still]
    return 1.0 - zz.size / n_sel
