"""GPU collimator rotation (arXiv:2512.18863 §2.2.2, last paragraph: the fluence
map is turned in the beam's-eye view about the central axis before the rays are
traced) against the FP64 oracle, through the C ABI.

Bars as for the unrotated path: forward <= 1e-5 of max dose, gradients <= 1e-4
of max |g| per group, the beam-frame fluence map within 2e-6 of the oracle's
(bilinear weights of FP32 coordinates), FP64 central differences within 1e-6 of
the oracle gradient, and the FP32 geometry cache equal to the uncached path bit
for bit.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2512_18863_amd import inputs
from tests.test_gpu_parity import TOL_FWD, _rel_err, _say, _t, gpu_dose, oracle_dose, subset

pytestmark = pytest.mark.gpu

TOL_GRAD = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rotated(case, angles):
    c = inputs.Case(**{k: getattr(case, k) for k in case.__dataclass_fields__})
    c.collimator = np.asarray(angles, dtype=np.float64)
    return c


def _check_grad(name, got, ref):
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max() / scale if scale > 0 else np.abs(got).max()
    _say("%s: max|dg|/max|g| = %.3e" % (name, err))
    assert err <= TOL_GRAD, name


def _grads(case, w, **kw):
    from paper_2512_18863_amd.engine import DoseEngine
    eng = DoseEngine(case, **kw)
    gl, gj, gm = eng.backward(_t(case.leaves), _t(case.jaws), _t(case.mu), _t(w))
    torch.cuda.synchronize()
    m = oracle.Model(case)
    rho = oracle.density(m)
    ref = oracle.backward(m, rho, case.gantry, case.leaves, case.jaws, case.mu, w, coll=case.collimator)
    return (gl.cpu().numpy(), gj.cpu().numpy(), gm.cpu().numpy()), ref, eng


ANGLES = [[0.0, 90.0, 180.0], [30.0, -17.0, 123.4], [45.0, 271.0, 359.5], [7.5, 200.0, -90.0]]


@pytest.mark.parametrize("k", range(len(ANGLES)))
def test_tiny_forward_and_map(k):
    ang = ANGLES[k]
    _say("collimator tiny forward, angles %s" % ang)
    c = _rotated(inputs.tiny_case(seed=40 + k, n_cp=3, n_taps=5 + 4 * k, shape=(7, 8, 6), spacing=6.0,
                                  field=30.0), ang)
    ref, m, rho = oracle_dose(c)
    got, eng = gpu_dose(c)
    err = _rel_err(got, ref)
    _say("max|dD|/maxD = %.3e" % err)
    assert err <= TOL_FWD
    # beam-frame fluence of the last batch against the oracle's intermediate
    Nk, Nu, Nv = eng.fan_shape()
    assert (Nu, Nv) == (m.Nu, m.Nv) and Nu == Nv
    Fb = eng.ws_view("rot", (c.n_cp, Nu, Nv), with_backward=0).cpu().numpy()
    for b in range(c.n_cp):
        r = oracle.forward_cp(m, rho, c.gantry[b], c.leaves[b], c.jaws[b], coll=c.collimator[b])
        np.testing.assert_allclose(Fb[b].T, r["F"], rtol=0, atol=2e-6)


@pytest.mark.parametrize("fcorr", [False, True])
def test_tiny_gradients(fcorr):
    _say("collimator tiny gradients, fluence corrections %s" % fcorr)
    c = _rotated(inputs.tiny_case(seed=51, n_cp=4, n_taps=9, shape=(7, 8, 6), spacing=6.0, field=30.0),
                 [12.0, 90.0, -33.3, 150.0])
    if fcorr:
        c.machine = inputs.with_fluence_corrections(c.machine)
    w = np.random.default_rng(51).uniform(size=c.shape)
    (gl, gj, gm), (rl, rj, rm), _ = _grads(c, w)
    _check_grad("leaves", gl, rl)
    _check_grad("jaws", gj, rj)
    _check_grad("mu", gm, rm)


def _c1_rotated(n):
    c = subset(inputs.config_c1(), np.arange(0, 90, 90 // n)[:n])
    ang = np.random.default_rng(77).uniform(-90.0, 90.0, size=c.n_cp)
    return _rotated(c, ang)


def test_c1_shape_forward_and_backward():
    """C1 geometry (128 x 128 x 96 pelvis, n = 15) with random collimator angles on
    10 control points: the MFMA/VALU convolutions on the square grid, with the
    aperture rectangle turned into the beam frame."""
    c = _c1_rotated(10)
    _say("C1 shape, 10 CPs, collimator angles %s" % np.round(c.collimator, 1))
    ref, m, _ = oracle_dose(c)
    got, eng = gpu_dose(c)
    err = _rel_err(got, ref)
    _say("C1 rotated max|dD|/maxD = %.3e (grid %d x %d)" % (err, eng.Nu, eng.Nv))
    assert err <= TOL_FWD
    w = np.random.default_rng(5).uniform(size=c.shape)
    (gl, gj, gm), (rl, rj, rm), _ = _grads(c, w)
    _check_grad("C1 leaves", gl, rl)
    _check_grad("C1 jaws", gj, rj)
    _check_grad("C1 mu", gm, rm)


def test_c4bench_shape_n61_forward_and_backward():
    """The 128^3 benchmark geometry with the 61 x 61 kernel and collimator angles on
    3 control points (the FP32 matrix-core convolutions on a rotated aperture)."""
    c = _rotated(subset(inputs.config_c4_plan(2000, bench=True), np.array([5, 80, 140])), [20.0, -45.0, 90.0])
    _say("C4-bench shape, 3 CPs, n=61, collimator 20/-45/90")
    ref, _, _ = oracle_dose(c)
    got, _ = gpu_dose(c)
    err = _rel_err(got, ref)
    _say("max|dD|/maxD = %.3e" % err)
    assert err <= TOL_FWD
    w = np.random.default_rng(6).uniform(size=c.shape)
    (gl, gj, gm), (rl, rj, rm), _ = _grads(c, w)
    _check_grad("leaves", gl, rl)
    _check_grad("jaws", gj, rj)
    _check_grad("mu", gm, rm)


def test_bf16_and_cache_with_rotation():
    """BF16 convolution with rotation against the oracle (2^-8 of max dose, the BF16
    bar), and the FP32 geometry cache against the uncached path (bit for bit)."""
    c = _c1_rotated(6)
    ref, _, _ = oracle_dose(c)
    d16, _ = gpu_dose(c, conv="bf16")
    e16 = _rel_err(d16, ref)
    _say("bf16 rotated: max|dD|/maxD = %.3e" % e16)
    assert e16 <= 2.0 ** -8
    from paper_2512_18863_amd.engine import DoseEngine
    eng = DoseEngine(c)
    lv, jw, mu = _t(c.leaves), _t(c.jaws), _t(c.mu)
    w = _t(np.random.default_rng(8).uniform(size=c.shape))
    d0 = eng.forward(lv, jw, mu).clone()
    g0 = [x.clone() for x in eng.backward(lv, jw, mu, w)]
    eng.build_cache("fp32")
    d1 = eng.forward(lv, jw, mu)
    g1 = eng.backward(lv, jw, mu, w)
    torch.cuda.synchronize()
    assert torch.equal(d0, d1)
    for a, b in zip(g0, g1):
        assert torch.equal(a, b)


def test_fd_fp64_vs_oracle_gradient():
    """GPU FP64 central differences (h = 0.01 mm) of L = sum w D on 12 leaf edges and
    the four jaws of a rotated plan against the oracle gradient (the map is piecewise
    linear in every edge, so central differences are exact away from kinks)."""
    from paper_2512_18863_amd.engine import DoseEngine
    from tests.test_gpu_grad import _fd_edges
    c = _rotated(inputs.tiny_case(seed=61, n_cp=2, n_taps=7, shape=(7, 8, 6), spacing=6.0, field=30.0),
                 [25.0, -70.0])
    c.jaws = c.jaws + np.array([-1.3, 1.1, -0.7, 0.9])   # off the pixel boundaries (kinks)
    w = np.random.default_rng(61).uniform(size=c.shape)
    m = oracle.Model(c)
    rho = oracle.density(m)
    rl, rj, _ = oracle.backward(m, rho, c.gantry, c.leaves, c.jaws, c.mu, w, coll=c.collimator)
    eng = DoseEngine(c, with_f64=True)
    eng.set_density_f64(torch.tensor(rho, dtype=torch.float64))
    wt = torch.tensor(w, dtype=torch.float64, device="cuda")
    h = 0.01

    def loss(lv, jw):
        d = eng.forward_f64(_t(lv, torch.float64), _t(jw, torch.float64), _t(c.mu, torch.float64))
        return float((d * wt).sum())

    errs = []
    scale = max(np.abs(rl).max(), np.abs(rj).max())
    picks = _fd_edges(c, 12, 62, h)
    assert len(picks) >= 6
    for (b, s, l) in picks:
        lp, lm = c.leaves.copy(), c.leaves.copy()
        lp[b, s, l] += h
        lm[b, s, l] -= h
        fd = (loss(lp, c.jaws) - loss(lm, c.jaws)) / (2 * h)
        errs.append(abs(fd - rl[b, s, l]) / scale)
    for b in range(c.n_cp):
        for q in range(4):
            jp, jm = c.jaws.copy(), c.jaws.copy()
            jp[b, q] += h
            jm[b, q] -= h
            fd = (loss(c.leaves, jp) - loss(c.leaves, jm)) / (2 * h)
            errs.append(abs(fd - rj[b, q]) / scale)
    _say("FD fp64 vs oracle gradient (rotated): max = %.3e" % max(errs))
    assert max(errs) <= 1e-6
