"""GPU plan assessment against the plan-evaluation oracle (weighted L1 objective,
DVH counts and parameters, isodose Dice; arXiv:2512.18863 §2.5 and §3).

Inputs are seeded synthetic dose fields and structure masks (never a dose from
the HIP path).  Counts and the objective's gradient are compared exactly; the
double-precision sums to rounding; DVH parameters read from a histogram to one
bin width of the exact sorted-dose values.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle import metrics as M
from tests.test_gpu_parity import _say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_18863_amd import plan_eval  # noqa: F401


def _field(shape, seed, n_struct=5, rx=60.0):
    """A smooth dose blob around a target, noise, exact ties at rx and at bin edges,
    and overlapping ellipsoid / random structures."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    Z, Y, X = np.meshgrid(np.linspace(-1, 1, nz), np.linspace(-1, 1, ny), np.linspace(-1, 1, nx), indexing="ij")
    r2 = X ** 2 + Y ** 2 + Z ** 2
    dose = (rx * 1.1 * np.exp(-r2 / 0.3) + rng.normal(0.0, 0.5, size=shape)).clip(0.0, None)
    dose = dose.astype(np.float32)
    flat = dose.ravel()
    idx = rng.choice(flat.size, size=min(500, flat.size), replace=False)
    flat[idx[:250]] = np.float32(rx)                 # on the PTV target
    flat[idx[250:]] = np.float32(0.5) * rng.integers(0, 100, size=len(idx) - 250)  # on bin edges of 0.5
    masks = [r2 <= 0.15, (r2 > 0.1) & (r2 < 0.5), X > 0.3]
    while len(masks) < n_struct:
        masks.append(rng.uniform(size=shape) < rng.uniform(0.05, 0.6))
    return dose, masks[:n_struct]


def _gpu(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


@pytest.mark.parametrize("shape,n_struct", [((17, 23, 29), 5), ((64, 70, 50), 3), ((40, 41, 42), 32)])
def test_l1_objective_matches_oracle(shape, n_struct):
    from paper_2512_18863_amd.plan_eval import Evaluator
    _say("L1 objective %s, %d structures" % (shape, n_struct))
    dose, masks = _field(shape, seed=sum(shape) + n_struct, n_struct=n_struct)
    rng = np.random.default_rng(5)
    weights = [100.0] + list(rng.choice([0.0, 0.1, 1.0, 10.0, 100.0], size=n_struct - 1))
    targets = [60.0] + [0.0] * (n_struct - 1)
    ev = Evaluator(masks)
    loss, grad = ev.l1(_gpu(dose), weights, targets)
    L, G = M.l1_objective(dose, masks, weights, targets)
    got = float(loss.cpu()[0])
    _say("loss GPU %.12e oracle %.12e" % (got, L))
    assert got == pytest.approx(L, rel=1e-12)
    assert np.array_equal(grad.cpu().numpy(), G.astype(np.float32))


def test_histogram_and_stats_match_oracle():
    from paper_2512_18863_amd.plan_eval import Evaluator
    _say("DVH histogram, 96 x 80 x 72, 6 structures, 0.5 Gy bins")
    dose, masks = _field((96, 80, 72), seed=11, n_struct=6)
    ev = Evaluator(masks)
    for n_bins, w in ((160, 0.5), (40, 0.5), (3000, 0.025), (1, 7.0)):   # clamped top bin, one bin
        hist, stats = ev.histogram(_gpu(dose), n_bins, w)
        h_ref, s_ref = M.dose_histogram(dose, masks, n_bins, w)
        assert np.array_equal(hist, h_ref), (n_bins, w)
        assert np.array_equal(stats[:, 0], s_ref[:, 0]) and np.array_equal(stats[:, 2], s_ref[:, 2])
        np.testing.assert_allclose(stats[:, 1], s_ref[:, 1], rtol=1e-12)


def test_histogram_32_structures_in_two_passes():
    from paper_2512_18863_amd.plan_eval import Evaluator
    _say("DVH histogram with 32 structures x 1000 bins (two LDS passes)")
    dose, masks = _field((30, 33, 31), seed=12, n_struct=32)
    ev = Evaluator(masks)
    hist, stats = ev.histogram(_gpu(dose), 1000, 0.1)
    h_ref, s_ref = M.dose_histogram(dose, masks, 1000, 0.1)
    assert np.array_equal(hist, h_ref)
    assert np.array_equal(stats[:, 0], s_ref[:, 0])


def test_threshold_counts_and_dice_match_oracle():
    from paper_2512_18863_amd.plan_eval import Evaluator
    _say("threshold counts / isodose Dice")
    dose, masks = _field((50, 61, 47), seed=13, n_struct=4)
    ev = Evaluator(masks)
    for thr in (60.0, 30.0, 0.0, 1e9):
        c = ev.counts_at_or_above(_gpu(dose), thr)
        assert np.array_equal(c, M.threshold_counts(dose, masks, thr)), thr
    d = ev.dice(_gpu(dose), 0, 60.0)
    assert d == M.isodose_dice(dose, masks[0], 60.0)


def test_dvh_parameters_within_one_bin_of_exact():
    from paper_2512_18863_amd.plan_eval import Evaluator
    _say("DVH parameters from the histogram vs sorted doses, 128^3")
    dose, masks = _field((128, 128, 128), seed=14, n_struct=3)
    ev = Evaluator(masks, names=["ptv", "ring", "side"])
    w, vox_cc = 0.01, 0.027
    rep = ev.report(_gpu(dose), rx=60.0, voxel_cc=vox_cc, bin_width=w)
    for s, name in enumerate(["ptv", "ring", "side"]):
        ex = M.dvh_metrics(dose, masks[s], vox_cc, 60.0)
        got = rep[name]
        for k in ("D98", "D50", "D2", "D2cc"):
            # the bin index is floor(D / w) of a rounded quotient: allow 1e-9 Gy at the edges
            assert -1e-9 <= ex[k] - got[k] < w + 1e-9, (name, k, ex[k], got[k])
        assert got["Dmax"] == ex["Dmax"]
        assert got["Dmean"] == pytest.approx(ex["Dmean"], rel=1e-12)
        assert got["V50"] == ex["V50"]


def test_empty_grid_and_autograd_hook():
    from paper_2512_18863_amd import plan_eval as PE
    from paper_2512_18863_amd import engine as E
    _say("n_vox = 0 through the C ABI; L1Objective autograd")
    lib = PE._lib()
    ws = torch.empty(lib.pdrt_eval_ws_bytes(2), dtype=torch.uint8, device="cuda")
    loss = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    d0 = torch.empty(1, device="cuda")
    l0 = torch.empty(1, dtype=torch.int32, device="cuda")
    w = (ctypes.c_double * 2)(1.0, 2.0)
    st = lib.pdrt_l1_objective(0, d0.data_ptr(), l0.data_ptr(), 2, w, w, loss.data_ptr(), None, ws.data_ptr(),
                               ws.numel(), E._stream_ptr(loss.device))
    assert st == 0 and float(loss.cpu()[0]) == 0.0
    hist = torch.full((2, 4), 9, dtype=torch.int32, device="cuda")
    stats = torch.full((2, 3), 9.0, dtype=torch.float64, device="cuda")
    st = lib.pdrt_dose_histogram(0, d0.data_ptr(), l0.data_ptr(), 2, 4, 1.0, hist.data_ptr(), stats.data_ptr(),
                                 ws.data_ptr(), ws.numel(), E._stream_ptr(loss.device))
    assert st == 0 and not hist.any() and not stats.any()
    assert lib.pdrt_dose_histogram(5, d0.data_ptr(), l0.data_ptr(), 33, 4, 1.0, hist.data_ptr(), stats.data_ptr(),
                                   ws.data_ptr(), ws.numel(), None) == -1
    dose, masks = _field((12, 13, 14), seed=15, n_struct=2)
    ev = PE.Evaluator(masks)
    x = _gpu(dose).requires_grad_(True)
    L = PE.L1Objective.apply(x, ev, [100.0, 1.0], [60.0, 0.0])
    L.backward()
    _, G = M.l1_objective(dose, masks, [100.0, 1.0], [60.0, 0.0])
    assert np.array_equal(x.grad.cpu().numpy(), G.astype(np.float32))
