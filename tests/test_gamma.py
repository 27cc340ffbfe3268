"""Gamma tool self-tests (special cases with known answers)."""
import numpy as np

from paper_2512_18863_amd import gamma


def _blob(n=24, s=3.0):
    z, y, x = np.meshgrid(*(np.arange(n) - n / 2 + 0.5,) * 3, indexing="ij")
    r2 = (x ** 2 + y ** 2 + z ** 2) * s * s
    return np.exp(-r2 / (2 * 20.0 ** 2)), (s, s, s)


def test_self_comparison_passes_everywhere():
    d, sp = _blob()
    assert gamma.pass_rate(d, d, sp) == 1.0


def test_scaled_within_dose_criterion_passes():
    d, sp = _blob()
    assert gamma.pass_rate(d, 1.0099 * d, sp, 1.0, 1.0) == 1.0


def test_offset_beyond_criterion_fails_in_flat_region():
    n = 20
    d = np.ones((n, n, n))
    d[:, :, : n // 2] = 0.5         # a flat plateau and a step
    ev = d + 0.011 * d.max()
    # away from the grid's faces (where the evaluated dose falls towards the zero
    # outside) only the high-side plane next to the step sees the shifted dose fall
    # back to its own value within 1 mm; on the low side the evaluated dose only rises
    inner = np.zeros_like(d, dtype=bool)
    inner[1:-1, 1:-1, 1:-1] = True
    assert abs(gamma.pass_rate(d, ev, (3.0, 3.0, 3.0), 1.0, 1.0, mask=inner) - 1.0 / (n - 2)) < 1e-12
    flat = inner.copy()
    flat[:, :, n // 2] = False
    assert gamma.pass_rate(d, ev, (3.0, 3.0, 3.0), 1.0, 1.0, mask=flat) == 0.0


def test_shift_within_dta_passes():
    """A linear ramp shifted by 0.5 mm in x passes at 1 mm even though the dose
    difference at the same point exceeds 1 %."""
    n = 16
    x = np.arange(n) * 3.0
    d = np.broadcast_to(0.5 + 0.2 * x[None, None, :], (n, n, n)).copy()
    ev = np.broadcast_to(0.5 + 0.2 * (x[None, None, :] - 0.5), (n, n, n)).copy()
    d = d[:, :, 1:-1]
    ev = ev[:, :, 1:-1]
    assert np.abs(ev - d).max() > 0.01 * d.max()
    interior = np.ones_like(d, dtype=bool)
    interior[:, :, -1] = False       # the matching point of the last plane lies beyond the grid
    assert gamma.pass_rate(d, ev, (3.0, 3.0, 3.0), 1.0, 1.0, mask=interior) == 1.0


def test_evaluated_dose_is_zero_outside_the_grid():
    """D_e is trilinear with zero outside the grid.  A ramp 0.3 ... 2.1 along x whose
    evaluated edge plane reads 0.35 instead of 0.3 (more than 1 % of max): inward the
    evaluated dose only rises, but 0.43 mm outward it has fallen to 0.3 towards the
    zero outside, so the edge plane passes at 1 %/1 mm; an edge-extended D_e (the
    value 0.35 continued outward) would fail it."""
    n = 10
    x = np.arange(n, dtype=np.float64)
    d = np.broadcast_to(0.3 + 0.2 * x[None, None, :], (n, n, n)).copy()
    ev = d.copy()
    ev[:, :, 0] = 0.35
    assert np.abs(ev - d).max() > 0.01 * d.max()
    assert gamma.pass_rate(d, ev, (3.0, 3.0, 3.0), 1.0, 1.0) == 1.0
