"""Pins of the oracle's fluence corrections (§2.2.2 list: source penumbra, head
scatter, off-axis factor), each against a library routine, a hand-computed value
or an invariant.  The corrections act on the aperture fluence map, so the maps
here come from the oracle's raster of random apertures."""
import dataclasses
import math

import numpy as np
import pytest
import scipy.ndimage

import oracle
from paper_2512_18863_amd import inputs

FWHM = 2.0 * math.sqrt(2.0 * math.log(2.0))


def _case(machine_kw, field=60.0, spacing=3.0, n_taps=5, seed=3):
    c = inputs.tiny_case(seed=seed, n_cp=1, n_taps=n_taps, shape=(6, 6, 6), spacing=spacing, field=field,
                         n_leaf=20, leaf_width=6.0)
    c.machine = dataclasses.replace(c.machine, fcorr=True, **machine_kw)
    return c


def _scipy_blur(F, sigma_mm, D, axis):
    """scipy's sampled, unit-sum Gaussian with the radius ceil(3 sigma / D)."""
    sd = sigma_mm / D
    R = math.ceil(3.0 * sd - 1e-9)
    return scipy.ndimage.gaussian_filter1d(F, sd, axis=axis, mode="constant", cval=0.0, truncate=(R - 0.25) / sd)


def test_penumbra_is_two_directional_gaussians():
    c = _case(dict(pen_fwhm_u=4.0, pen_fwhm_v=7.0))
    m = oracle.Model(c)
    F = oracle.raster(m, c.leaves[0], c.jaws[0])
    got = oracle.fluence_correct(m, F)
    D = c.lat_step
    # maps are [Nv][Nu]: u runs along axis 1
    ref = _scipy_blur(_scipy_blur(F, 4.0 / FWHM, D, axis=1), 7.0 / FWHM, D, axis=0)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)


def test_head_scatter_adds_an_isotropic_gaussian():
    c = _case(dict(hs_amp=0.07, hs_sigma=9.0))
    m = oracle.Model(c)
    F = oracle.raster(m, c.leaves[0], c.jaws[0])
    got = oracle.fluence_correct(m, F)
    D = c.lat_step
    blur = _scipy_blur(_scipy_blur(F, 9.0, D, axis=1), 9.0, D, axis=0)
    np.testing.assert_allclose(got, F + 0.07 * blur, rtol=0, atol=1e-14)


def test_off_axis_factor_at_a_3_4_5_pixel():
    c = _case(dict(oar=(1e-3, 2e-5)))
    m = oracle.Model(c)
    F = np.ones((m.Nv, m.Nu))
    got = oracle.fluence_correct(m, F)
    D = c.lat_step
    cu, cv = (m.Nu - 1) // 2, (m.Nv - 1) // 2          # odd grids: the centre is a pixel
    r = 5.0 * D                                          # pixel (cu + 3, cv + 4)
    assert got[cv + 4, cu + 3] == pytest.approx(1.0 + 1e-3 * r + 2e-5 * r * r, rel=1e-14)
    assert got[cv, cu] == 1.0


def test_corrections_adjoint_dot_product():
    c = _case(dict(pen_fwhm_u=3.5, pen_fwhm_v=4.5, hs_amp=0.04, hs_sigma=12.0, oar=(0.0, 4e-6)))
    m = oracle.Model(c)
    rng = np.random.default_rng(7)
    x = rng.normal(size=(m.Nv, m.Nu))
    y = rng.normal(size=(m.Nv, m.Nu))
    lhs = np.vdot(oracle.fluence_correct(m, x), y)
    rhs = np.vdot(x, oracle.fluence_correct(m, y, transpose=True))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def test_uniform_field_centre_gains_exactly_the_head_scatter():
    """Far inside a wide uniform field the normalised blurs leave the fluence at one,
    so without an off-axis factor the central dose grows by exactly 1 + hs_amp."""
    m0 = inputs.Machine()
    case, (ix, j, iz, w) = inputs.reference_case(m0, 7, 5.0, field_mm=260.0)
    mc = dataclasses.replace(inputs.with_fluence_corrections(m0), oar=(0.0, 0.0))
    case_c, _ = inputs.reference_case(mc, 7, 5.0, field_mm=260.0)
    d = []
    for cs in (case, case_c):
        m = oracle.Model(cs)
        rho = oracle.density(m)
        d.append(oracle.forward(m, rho, cs.gantry, cs.leaves, cs.jaws, cs.mu)[iz, j, ix])
    assert d[1] / d[0] == pytest.approx(1.0 + mc.hs_amp, rel=1e-12)


def test_gradients_with_corrections_match_central_differences():
    """With the corrections on, the dose is still piecewise linear in every leaf and
    jaw, so central differences away from pixel edges are exact up to rounding."""
    c = inputs.tiny_case(seed=21, n_cp=2, n_taps=3, shape=(6, 7, 6), field=30.0)
    c.machine = inputs.with_fluence_corrections(c.machine)
    m = oracle.Model(c)
    rho = oracle.density(m)
    w = np.random.default_rng(5).uniform(size=m.vol_shape)
    gl, gj, gm = oracle.backward(m, rho, c.gantry, c.leaves, c.jaws, c.mu, w)
    D = c.lat_step
    boundaries = (np.arange(m.Nu + 1) - m.Nu / 2) * D
    h = 1e-3

    def loss(lv, jw, mu):
        return np.vdot(w, oracle.forward(m, rho, c.gantry, lv, jw, mu))
    checked = 0
    for b in range(c.n_cp):
        for side in (0, 1):
            for l in range(c.machine.n_leaf):
                x = c.leaves[b, side, l]
                if np.min(np.abs(x - boundaries)) < 10 * h:
                    continue
                lp, lm = c.leaves.copy(), c.leaves.copy()
                lp[b, side, l] += h
                lm[b, side, l] -= h
                fd = (loss(lp, c.jaws, c.mu) - loss(lm, c.jaws, c.mu)) / (2 * h)
                assert abs(fd - gl[b, side, l]) < 1e-7 * max(1.0, abs(fd))
                checked += 1
        for q in range(4):
            x = c.jaws[b, q]
            if np.min(np.abs(x - boundaries)) < 10 * h:
                continue
            jp, jm = c.jaws.copy(), c.jaws.copy()
            jp[b, q] += h
            jm[b, q] -= h
            fd = (loss(c.leaves, jp, c.mu) - loss(c.leaves, jm, c.mu)) / (2 * h)
            assert abs(fd - gj[b, q]) < 1e-7 * max(1.0, abs(fd))
            checked += 1
    assert checked >= 10
    # and the MU identity MU_b dL/dMU_b = <g, calib MU_b D_b>
    for b in range(c.n_cp):
        Db = oracle.forward(m, rho, c.gantry[b:b + 1], c.leaves[b:b + 1], c.jaws[b:b + 1], c.mu[b:b + 1])
        assert abs(c.mu[b] * gm[b] - np.vdot(w, Db)) < 1e-11 * max(1.0, abs(np.vdot(w, Db)))
