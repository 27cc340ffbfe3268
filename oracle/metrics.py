"""Plan-evaluation oracle: the weighted L1 objective of the optimisation study,
dose-volume histograms and their metrics, and the isodose Dice coefficient
(arXiv:2512.18863 §2.5 objective and plan assessment; §3 DVH tables).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, never by the product
path.  Plain numpy in double precision, written from the definitions; nothing
here is shared with the HIP library.

Readings (where the paper leaves a choice open):
  * |.|_1 is the sum of absolute values over the structure's voxels (not a mean);
    its derivative at a kink (D exactly on the target) is taken as 0.
  * Structures may overlap; a voxel contributes once per structure it is in.
  * D_x% is the smallest dose received by the hottest x % of the structure:
    sorting its N doses in decreasing order, the value at position ceil(x N / 100)
    (1-based), ceil taken in integer arithmetic; D_{V cc} is the same with
    ceil(V / voxel volume) voxels.
  * V_d is the fraction of the structure receiving at least d.
  * The 100 % isodose volume is {D >= D_prescribed}; Dice = 2 |A n B| / (|A| + |B|).
"""
from __future__ import annotations

import math

import numpy as np


def _masks(masks) -> list:
    return [np.asarray(m, dtype=bool).ravel() for m in masks]


def l1_objective(dose, masks, weights, targets):
    """L = sum_s w_s sum_{v in s} |D_v - t_s| and dL/dD_v = sum_{s: v in s} w_s sign(D_v - t_s)."""
    d = np.asarray(dose, dtype=np.float64).ravel()
    loss = 0.0
    grad = np.zeros_like(d)
    for m, w, t in zip(_masks(masks), weights, targets):
        diff = d[m] - float(t)
        loss += float(w) * float(np.abs(diff).sum())
        grad[m] += float(w) * np.sign(diff)
    return loss, grad.reshape(np.shape(dose))


def dose_bins(dose, n_bins: int, bin_width: float) -> np.ndarray:
    """Bin index of each voxel: floor(D / width) in double precision, clamped to [0, n_bins - 1]."""
    d = np.asarray(dose, dtype=np.float64).ravel()
    b = np.floor(d / float(bin_width))
    return np.clip(b, 0, n_bins - 1).astype(np.int64)


def dose_histogram(dose, masks, n_bins: int, bin_width: float):
    """Differential DVH counts [S][n_bins] and per-structure (count, sum of dose, max dose);
    the maximum of an empty structure is 0 (doses are non-negative)."""
    b = dose_bins(dose, n_bins, bin_width)
    d = np.asarray(dose, dtype=np.float64).ravel()
    ms = _masks(masks)
    hist = np.zeros((len(ms), n_bins), dtype=np.int64)
    stats = np.zeros((len(ms), 3))
    for s, m in enumerate(ms):
        hist[s] = np.bincount(b[m], minlength=n_bins)
        stats[s, 0] = m.sum()
        stats[s, 1] = d[m].sum()
        stats[s, 2] = d[m].max() if m.any() else 0.0
    return hist, stats


def threshold_counts(dose, masks, threshold: float) -> np.ndarray:
    """[S + 1]: voxels of each structure with D >= threshold, then over the whole grid."""
    d = np.asarray(dose, dtype=np.float64).ravel()
    hot = d >= float(threshold)
    out = [int((hot & m).sum()) for m in _masks(masks)]
    out.append(int(hot.sum()))
    return np.asarray(out, dtype=np.int64)


def d_at_volume(values, n_hot: int) -> float:
    """Smallest dose among the n_hot hottest voxels (n_hot clamped to [1, N])."""
    v = np.sort(np.asarray(values, dtype=np.float64))[::-1]
    n_hot = min(max(int(n_hot), 1), len(v))
    return float(v[n_hot - 1])


def dvh_metrics(dose, mask, voxel_cc: float, rx: float) -> dict:
    """D98 %, D50 %, D2 %, Dmean, Dmax, D2cc and V50 % (of rx) of one structure."""
    v = np.asarray(dose, dtype=np.float64).ravel()[np.asarray(mask, dtype=bool).ravel()]
    n = len(v)
    return {
        "D98": d_at_volume(v, (98 * n + 99) // 100),
        "D50": d_at_volume(v, (50 * n + 99) // 100),
        "D2": d_at_volume(v, (2 * n + 99) // 100),
        "Dmean": float(v.mean()),
        "Dmax": float(v.max()),
        "D2cc": d_at_volume(v, math.ceil(2.0 / voxel_cc)),
        "V50": float((v >= 0.5 * rx).mean()),
    }


def dice(a, b) -> float:
    a = np.asarray(a, dtype=bool)
    b = np.asarray(b, dtype=bool)
    den = int(a.sum()) + int(b.sum())
    return 2.0 * int((a & b).sum()) / den if den else 1.0


def isodose_dice(dose, ptv, rx: float) -> float:
    return dice(np.asarray(dose, dtype=np.float64) >= float(rx), ptv)
