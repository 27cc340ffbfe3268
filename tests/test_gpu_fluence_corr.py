"""GPU parity of the fluence corrections (source penumbra, head scatter, off-axis
factor; §2.2.2 list) against the FP64 oracle: the corrected fluence map, the
forward dose (FP32 bar 1e-5 of max dose; FP64 path 1e-12), the FP32 adjoint
(1e-4 of max |grad| per group) and FP64 central differences of the GPU's own
forward against the oracle gradient."""
import numpy as np
import pytest
import torch

import oracle
from paper_2512_18863_amd import inputs
from tests.test_gpu_grad import TOL_GRAD, _check, _grads_gpu, _grads_oracle
from tests.test_gpu_parity import TOL_FWD, _rel_err, _say, _t, gpu_dose, oracle_dose, subset

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _corr(case):
    case.machine = inputs.with_fluence_corrections(case.machine)
    return case


def test_corrected_fluence_map():
    _say("corrected fluence maps (C1, 4 CPs) vs oracle")
    c = _corr(subset(inputs.config_c1(), np.array([0, 20, 45, 70])))
    m = oracle.Model(c)
    _, eng = gpu_dose(c)
    Nk, Nu, Nv = eng.fan_shape()
    F = eng.ws_view("fluence", (c.n_cp, Nu, Nv)).cpu().numpy()
    for b in range(c.n_cp):
        ref = oracle.fluence_correct(m, oracle.raster(m, c.leaves[b], c.jaws[b]))
        err = np.abs(F[b].T - ref).max()
        _say("cp %d: max|dF| = %.3e (max F %.3f)" % (b, err, ref.max()))
        assert err <= 2e-6


@pytest.mark.parametrize("name,mk,idx", [
    ("tiny", lambda: inputs.tiny_case(seed=41, n_cp=3, n_taps=9, shape=(8, 9, 7), spacing=4.0, field=40.0,
                                      n_leaf=12, leaf_width=8.0), np.arange(3)),
    ("C1", inputs.config_c1, np.arange(0, 90, 9)),
    ("C4-bench", lambda: inputs.config_c4_plan(2000, bench=True), np.array([3, 91, 170])),
])
def test_forward_parity_with_corrections(name, mk, idx):
    c = _corr(subset(mk(), idx))
    ref, _, _ = oracle_dose(c)
    got, _ = gpu_dose(c)
    err = _rel_err(got, ref)
    _say("%s with fluence corrections (%d CPs): max|dD|/maxD = %.3e" % (name, len(idx), err))
    assert err <= TOL_FWD


def test_forward_f64_with_corrections():
    from paper_2512_18863_amd.engine import DoseEngine
    c = _corr(inputs.tiny_case(seed=42, n_cp=2, n_taps=7, shape=(7, 8, 6), spacing=5.0, field=35.0,
                               n_leaf=10, leaf_width=8.0))
    ref, _, rho = oracle_dose(c)
    eng = DoseEngine(c, with_f64=True)
    eng.set_density_f64(_t(rho, torch.float64))
    got = eng.forward_f64(_t(c.leaves, torch.float64), _t(c.jaws, torch.float64),
                          _t(c.mu, torch.float64)).cpu().numpy()
    err = _rel_err(got, ref)
    _say("FP64 path with fluence corrections: max|dD|/maxD = %.3e" % err)
    assert err <= 1e-12


@pytest.mark.parametrize("name,mk,idx", [
    ("tiny", lambda: inputs.tiny_case(seed=43, n_cp=3, n_taps=5, shape=(6, 7, 6), spacing=6.0, field=30.0,
                                      n_leaf=10, leaf_width=6.0), np.arange(3)),
    ("C1", inputs.config_c1, np.arange(0, 90, 15)),
])
def test_gradient_parity_with_corrections(name, mk, idx):
    _say("%s gradients with fluence corrections" % name)
    c = _corr(subset(mk(), idx))
    w = np.random.default_rng(44).uniform(size=c.shape)
    gl, gj, gm, _ = _grads_gpu(c, w)
    rl, rj, rm = _grads_oracle(c, w)
    _check("leaves", gl, rl)
    _check("jaws", gj, rj)
    _check("mu", gm, rm)
