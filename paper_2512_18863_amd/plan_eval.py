"""Plan assessment through the HIP library: the weighted L1 objective of the
gradient-based optimisation study (arXiv:2512.18863 §2.5), dose-volume histograms
and the DVH parameters reported in §3 (D98 %, D50 %, D2 %, Dmean, Dmax, D2cc,
V50 %), and the Dice coefficient of the prescription isodose volume with the PTV
used to pick the objective weights (§2.5).

Structures travel as one uint32 label per voxel (bit s = structure s).  The
per-voxel work (objective, gradient, histogram, threshold counts, per-structure
sums) runs in the library's kernels; what is read back is a few hundred numbers,
from which the DVH parameters follow on the host.

DVH parameters from a histogram are exact to one bin: D_x% is reported as the
lower edge of the bin holding the ceil(x N / 100)-th hottest voxel, so the exact
value lies in [D, D + bin width).  Dmean and Dmax are exact; V_d and the Dice
coefficient come from exact counts.
"""
from __future__ import annotations

import ctypes
from typing import Dict, Iterable, List, Optional, Sequence

import numpy as np
import torch

from . import engine as E

MAX_STRUCTS = 32


def _lib():
    lib = E.lib()
    if not getattr(lib, "_eval_sigs", False):
        V = ctypes.c_void_p
        I32, I64 = ctypes.c_int32, ctypes.c_int64
        PD = ctypes.POINTER(ctypes.c_double)
        sigs = {
            "pdrt_eval_ws_bytes": (ctypes.c_size_t, [I32]),
            "pdrt_l1_objective": (ctypes.c_int, [I64, V, V, I32, PD, PD, V, V, V, ctypes.c_size_t, V]),
            "pdrt_dose_histogram": (ctypes.c_int, [I64, V, V, I32, I32, ctypes.c_double, V, V, V, ctypes.c_size_t,
                                                   V]),
            "pdrt_threshold_counts": (ctypes.c_int, [I64, V, V, I32, ctypes.c_double, V, V]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        lib._eval_sigs = True
    return lib


def labels_from_masks(masks: Sequence, device="cuda") -> torch.Tensor:
    """uint32 labels (stored as int32) with bit s set where masks[s] is true."""
    if not 1 <= len(masks) <= MAX_STRUCTS:
        raise ValueError("1 to %d structures" % MAX_STRUCTS)
    lab = np.zeros(np.shape(masks[0]), dtype=np.uint32)
    for s, m in enumerate(masks):
        m = m.cpu().numpy() if isinstance(m, torch.Tensor) else np.asarray(m)
        if m.shape != lab.shape:
            raise ValueError("all masks need the dose grid's shape")
        lab |= (m.astype(bool).astype(np.uint32) << np.uint32(s))
    return torch.from_numpy(lab.view(np.int32)).to(device)


def _check_pair(dose: torch.Tensor, labels: torch.Tensor):
    if not (dose.is_cuda and dose.dtype == torch.float32 and dose.is_contiguous()):
        raise ValueError("dose must be a contiguous float32 CUDA tensor")
    if not (labels.is_cuda and labels.dtype == torch.int32 and labels.is_contiguous()):
        raise ValueError("labels must be a contiguous int32 CUDA tensor (uint32 bits)")
    if labels.shape != dose.shape or labels.device != dose.device:
        raise ValueError("labels and dose must have the same shape and device")


class Evaluator:
    """Objective and plan metrics for one dose grid and one set of structures."""

    def __init__(self, masks: Sequence, names: Optional[Sequence[str]] = None, device="cuda"):
        self.n_struct = len(masks)
        self.names = list(names) if names is not None else ["s%d" % i for i in range(self.n_struct)]
        self.labels = labels_from_masks(masks, device)
        self.device = self.labels.device
        self.n_vox = int(self.labels.numel())
        nbytes = _lib().pdrt_eval_ws_bytes(self.n_struct)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.loss = torch.zeros(1, dtype=torch.float64, device=self.device)

    def _stream(self):
        return E._stream_ptr(self.device)

    # ---------------------------------------------------------------- objective
    def l1(self, dose: torch.Tensor, weights: Sequence[float], targets: Sequence[float], want_grad: bool = True):
        """(loss device tensor [1] float64, gradient dL/d dose or None)."""
        _check_pair(dose, self.labels)
        if len(weights) != self.n_struct or len(targets) != self.n_struct:
            raise ValueError("one weight and one target per structure")
        w = np.ascontiguousarray(weights, dtype=np.float64)
        t = np.ascontiguousarray(targets, dtype=np.float64)
        grad = torch.empty_like(dose) if want_grad else None
        PD = ctypes.POINTER(ctypes.c_double)
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        E._check(_lib().pdrt_l1_objective(self.n_vox, dose.data_ptr(), self.labels.data_ptr(), self.n_struct,
                                          w.ctypes.data_as(PD), t.ctypes.data_as(PD), loss.data_ptr(),
                                          grad.data_ptr() if grad is not None else None, self.ws.data_ptr(),
                                          self.ws.numel(), self._stream()), "pdrt_l1_objective")
        return loss, grad

    # ---------------------------------------------------------------- DVH
    def histogram(self, dose: torch.Tensor, n_bins: int, bin_width: float):
        """(hist [S][n_bins] int64, stats [S][3] = count, sum, max) on the host."""
        _check_pair(dose, self.labels)
        hist = torch.empty((self.n_struct, n_bins), dtype=torch.int32, device=self.device)
        stats = torch.empty((self.n_struct, 3), dtype=torch.float64, device=self.device)
        E._check(_lib().pdrt_dose_histogram(self.n_vox, dose.data_ptr(), self.labels.data_ptr(), self.n_struct,
                                            int(n_bins), float(bin_width), hist.data_ptr(), stats.data_ptr(),
                                            self.ws.data_ptr(), self.ws.numel(), self._stream()),
                 "pdrt_dose_histogram")
        h = hist.cpu().numpy().view(np.uint32).astype(np.int64)
        return h, stats.cpu().numpy()

    def counts_at_or_above(self, dose: torch.Tensor, threshold: float) -> np.ndarray:
        """[S + 1] voxel counts with dose >= threshold (per structure, then the whole grid)."""
        _check_pair(dose, self.labels)
        c = torch.empty(self.n_struct + 1, dtype=torch.int64, device=self.device)
        E._check(_lib().pdrt_threshold_counts(self.n_vox, dose.data_ptr(), self.labels.data_ptr(), self.n_struct,
                                              float(threshold), c.data_ptr(), self._stream()),
                 "pdrt_threshold_counts")
        return c.cpu().numpy()

    def dice(self, dose: torch.Tensor, s: int, rx: float, sizes: Optional[np.ndarray] = None) -> float:
        """Dice coefficient of {dose >= rx} with structure s."""
        c = self.counts_at_or_above(dose, rx)
        if sizes is None:
            sizes = self.counts_at_or_above(dose, -np.inf)[:-1]
        den = int(c[-1]) + int(sizes[s])
        return 2.0 * int(c[s]) / den if den else 1.0

    def report(self, dose: torch.Tensor, rx: float, voxel_cc: float, bin_width: float = 0.01,
               max_dose: Optional[float] = None) -> Dict[str, dict]:
        """DVH parameters of every structure (§3 tables) at the histogram's resolution."""
        if max_dose is None:  # the structures' maximum dose, from a one-bin pass
            _, st = self.histogram(dose, 1, 1.0)
            max_dose = float(st[:, 2].max())
        n_bins = int(min(16384, max(1, np.floor(max_dose / bin_width) + 2)))
        hist, stats = self.histogram(dose, n_bins, bin_width)
        v50 = self.counts_at_or_above(dose, 0.5 * rx)
        out = {}
        for s in range(self.n_struct):
            out[self.names[s]] = dvh_parameters(hist[s], stats[s], bin_width, voxel_cc, int(v50[s]))
        return out


def d_from_histogram(hist_row: np.ndarray, bin_width: float, n_hot: int) -> float:
    """Lower edge of the bin that holds the n_hot-th hottest voxel."""
    n = int(hist_row.sum())
    if n == 0:
        return 0.0
    n_hot = min(max(int(n_hot), 1), n)
    above = np.cumsum(hist_row[::-1])[::-1]     # above[b] = voxels in bins >= b
    b = int(np.nonzero(above >= n_hot)[0].max())
    return b * bin_width


def dvh_parameters(hist_row, stats_row, bin_width: float, voxel_cc: float, n_at_half_rx: int) -> dict:
    n = int(stats_row[0])
    if n == 0:
        return {"N": 0}
    return {
        "N": n,
        "D98": d_from_histogram(hist_row, bin_width, (98 * n + 99) // 100),
        "D50": d_from_histogram(hist_row, bin_width, (50 * n + 99) // 100),
        "D2": d_from_histogram(hist_row, bin_width, (2 * n + 99) // 100),
        "Dmean": float(stats_row[1]) / n,
        "Dmax": float(stats_row[2]),
        "D2cc": d_from_histogram(hist_row, bin_width, int(np.ceil(2.0 / voxel_cc))),
        "V50": n_at_half_rx / n,
    }


class L1Objective(torch.autograd.Function):
    """loss = weighted L1 objective of dose (float64 scalar) with the kernel's gradient."""

    @staticmethod
    def forward(ctx, dose, evaluator: Evaluator, weights, targets):
        loss, grad = evaluator.l1(dose.detach().contiguous(), weights, targets, want_grad=dose.requires_grad)
        ctx.save_for_backward(grad if grad is not None else torch.empty(0, device=dose.device))
        return loss[0]

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return (grad * g.to(torch.float32), None, None, None)
