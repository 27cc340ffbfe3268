"""Pins of the plan-evaluation oracle (weighted L1 objective of the optimisation
study, DVH counts and metrics, isodose Dice; arXiv:2512.18863 §2.5 and §3).

Each check is tied to something other than the oracle's own vectorised code:
pure-Python loops over tiny inputs, closed forms on ramps and constant doses,
finite differences of the objective, and set identities of the Dice coefficient.
"""
import math

import numpy as np
import pytest

from oracle import metrics as M


def _tiny(seed, n=37, n_struct=3):
    rng = np.random.default_rng(seed)
    dose = rng.uniform(0.0, 80.0, size=n)
    dose[::7] = 40.0                      # voxels exactly on a target
    masks = [rng.uniform(size=n) < 0.5 for _ in range(n_struct)]
    return dose, masks


def test_l1_objective_brute_force_loops():
    """§2.5 objective: L = lambda_PTV |D_PTV - D_rx|_1 + sum_s lambda_s |D_s|_1, written as loops."""
    dose, masks = _tiny(1)
    weights, targets = [100.0, 1.0, 10.0], [40.0, 0.0, 0.0]
    loss, grad = M.l1_objective(dose, masks, weights, targets)
    L = 0.0
    G = [0.0] * len(dose)
    for s in range(3):
        for v in range(len(dose)):
            if masks[s][v]:
                x = dose[v] - targets[s]
                L += weights[s] * abs(x)
                G[v] += weights[s] * (1.0 if x > 0 else (-1.0 if x < 0 else 0.0))
    assert loss == pytest.approx(L, rel=1e-14)
    assert np.array_equal(grad, np.asarray(G))


def test_l1_objective_finite_differences():
    """The gradient is the derivative of L wherever no voxel sits on a kink."""
    rng = np.random.default_rng(2)
    dose = rng.uniform(1.0, 80.0, size=50)
    masks = [rng.uniform(size=50) < 0.6 for _ in range(2)]
    w, t = [3.0, 0.5], [42.0, 0.0]
    _, g = M.l1_objective(dose, masks, w, t)
    h = 1e-6
    for v in (0, 7, 19, 33, 49):
        if abs(dose[v] - 42.0) < 1e-3:
            continue
        dp, dm = dose.copy(), dose.copy()
        dp[v] += h
        dm[v] -= h
        fd = (M.l1_objective(dp, masks, w, t)[0] - M.l1_objective(dm, masks, w, t)[0]) / (2 * h)
        assert fd == pytest.approx(g[v], abs=1e-6)


def test_l1_objective_closed_forms():
    """An OAR term with target 0 is lambda times the structure's total dose; a PTV at
    exactly the prescription costs nothing and has zero gradient."""
    dose = np.linspace(0.0, 10.0, 11)
    oar = np.ones(11, dtype=bool)
    loss, grad = M.l1_objective(dose, [oar], [2.5], [0.0])
    assert loss == pytest.approx(2.5 * 55.0)
    assert np.array_equal(grad, np.r_[0.0, np.full(10, 2.5)])
    flat = np.full(11, 60.0)
    loss, grad = M.l1_objective(flat, [oar], [100.0], [60.0])
    assert loss == 0.0 and not grad.any()


def test_histogram_brute_force_loops():
    """Differential DVH: each voxel of a structure counted once in bin floor(D / w), clamped."""
    dose, masks = _tiny(3, n=101)
    dose[3] = 250.0                       # beyond the last bin
    dose[5] = 0.0
    n_bins, w = 30, 2.5
    hist, stats = M.dose_histogram(dose, masks, n_bins, w)
    for s, m in enumerate(masks):
        ref = [0] * n_bins
        tot, mx, cnt = 0.0, 0.0, 0
        for v in range(len(dose)):
            if m[v]:
                b = min(int(math.floor(dose[v] / w)), n_bins - 1)
                ref[b] += 1
                tot += dose[v]
                mx = max(mx, dose[v])
                cnt += 1
        assert hist[s].tolist() == ref
        assert stats[s, 0] == cnt and stats[s, 2] == mx
        assert stats[s, 1] == pytest.approx(tot, rel=1e-14)


def test_histogram_bin_edges_exact():
    """A dose exactly on a bin edge falls in the bin above it."""
    dose = np.array([0.0, 2.0, 4.0, 3.999999, 5.0])
    hist, _ = M.dose_histogram(dose, [np.ones(5, dtype=bool)], 4, 2.0)
    assert hist[0].tolist() == [1, 2, 2, 0]


def test_threshold_counts_brute_force():
    dose, masks = _tiny(4, n=64)
    c = M.threshold_counts(dose, masks, 40.0)
    for s, m in enumerate(masks):
        assert c[s] == sum(1 for v in range(64) if m[v] and dose[v] >= 40.0)
    assert c[-1] == sum(1 for v in range(64) if dose[v] >= 40.0)


def test_dvh_metrics_on_a_ramp():
    """Doses 1, 2, ..., 200 (one voxel each): D_x% is the ceil(2 x)-th largest value,
    i.e. 201 - ceil(2 x); Dmean = 100.5; V50% of rx = 100 counts doses >= 50."""
    dose = np.arange(1.0, 201.0)
    mask = np.ones(200, dtype=bool)
    m = M.dvh_metrics(dose, mask, voxel_cc=0.5, rx=100.0)
    assert m["D98"] == 201 - 196
    assert m["D50"] == 201 - 100
    assert m["D2"] == 201 - 4
    assert m["Dmax"] == 200.0 and m["Dmean"] == pytest.approx(100.5)
    assert m["D2cc"] == 201 - 4          # 2 cc = 4 voxels of 0.5 cc
    assert m["V50"] == pytest.approx(151 / 200)


def test_dvh_metrics_constant_dose():
    dose = np.full(37, 42.7)
    m = M.dvh_metrics(dose, np.ones(37, dtype=bool), voxel_cc=0.027, rx=42.7)
    for k in ("D98", "D50", "D2", "Dmean", "Dmax", "D2cc"):
        assert m[k] == pytest.approx(42.7, rel=1e-15)
    assert m["V50"] == 1.0


def test_dice_identities():
    """Dice = 1 for equal sets, 0 for disjoint ones, 2/3 for a set and its half."""
    a = np.zeros(20, dtype=bool)
    a[:10] = True
    b = np.zeros(20, dtype=bool)
    b[10:] = True
    h = np.zeros(20, dtype=bool)
    h[:5] = True
    assert M.dice(a, a) == 1.0 and M.dice(a, b) == 0.0
    assert M.dice(a, h) == pytest.approx(2 * 5 / 15)
    dose = np.where(a, 70.0, 10.0)
    assert M.isodose_dice(dose, a, 60.0) == 1.0
    assert M.isodose_dice(dose, h, 60.0) == pytest.approx(2 * 5 / 15)
