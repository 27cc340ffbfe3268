"""The segmented-scan form of the ray march (spec.march_scan = 1: the depth
integral of Eq. 7 split over the wavefronts of a workgroup, each scanning its
segment of planes and adding the sums of the segments before it) against the
FP64 oracle, with the bars of the default form: forward <= 1e-5 of max dose,
gradients <= 1e-4 of max |g|, the FP64 path <= 1e-12, and the FP32 geometry cache
built in the same form equal to the uncached path bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from paper_2512_18863_amd import inputs
from tests.test_gpu_parity import TOL_FWD, _rel_err, _say, _t, oracle_dose, subset

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _engine(case, **kw):
    from paper_2512_18863_amd.engine import DoseEngine
    return DoseEngine(case, march_scan=True, **kw)


def _check_grads(case, eng, w):
    m = oracle.Model(case)
    rho = oracle.density(m)
    ref = oracle.backward(m, rho, case.gantry, case.leaves, case.jaws, case.mu, w)
    got = [t.cpu().numpy() for t in eng.backward(_t(case.leaves), _t(case.jaws), _t(case.mu), _t(w))]
    for name, a, r in zip(("leaves", "jaws", "mu"), got, ref):
        e = np.abs(a - r).max() / np.abs(r).max()
        _say("scan march %s: max|dg|/max|g| = %.3e" % (name, e))
        assert e <= 1e-4, name


CASES = [
    dict(seed=71, n_taps=3, shape=(5, 6, 5), spacing=10.0, field=25.0),
    dict(seed=72, n_taps=15, shape=(9, 8, 10), spacing=6.0, field=40.0),                       # MFMA path
    dict(seed=73, n_taps=5, shape=(6, 7, 6), spacing=8.0, field=30.0, wepl_mode=inputs.WEPL_CENTRAL_AXIS),
    # a long ray: more planes than eight 32-plane segments, so each wavefront makes several passes
    dict(seed=74, n_taps=9, shape=(3, 200, 200), spacing=2.5, field=25.0),
]


@pytest.mark.parametrize("kw", CASES, ids=[str(i) for i in range(len(CASES))])
def test_scan_march_forward_and_gradients(kw):
    c = inputs.tiny_case(n_cp=3, **kw)
    _say("scan march, tiny %s" % kw)
    eng = _engine(c)
    got = eng.forward(_t(c.leaves), _t(c.jaws), _t(c.mu)).cpu().numpy().astype(np.float64)
    ref, m, _ = oracle_dose(c)
    err = _rel_err(got, ref)
    _say("scan march forward: Nk = %d, max|dD|/maxD = %.3e" % (m.Nk, err))
    assert err <= TOL_FWD
    _check_grads(c, eng, np.random.default_rng(kw["seed"]).uniform(size=c.shape))


def test_scan_march_c4bench_subset_and_fp64():
    c = subset(inputs.config_c4_plan(2000, bench=True), np.array([7, 88, 151]))
    _say("scan march, 128^3 n=61, 3 CPs")
    eng = _engine(c, with_f64=True)
    got = eng.forward(_t(c.leaves), _t(c.jaws), _t(c.mu)).cpu().numpy().astype(np.float64)
    ref, m, rho = oracle_dose(c)
    assert _rel_err(got, ref) <= TOL_FWD
    _check_grads(c, eng, np.random.default_rng(77).uniform(size=c.shape))
    eng.set_density_f64(_t(rho, torch.float64))
    d64 = eng.forward_f64(_t(c.leaves, torch.float64), _t(c.jaws, torch.float64),
                          _t(c.mu, torch.float64)).cpu().numpy()
    e64 = _rel_err(d64, ref)
    _say("scan march FP64 path: %.3e" % e64)
    assert e64 <= 1e-12


def test_scan_march_geometry_cache_bitwise():
    c = subset(inputs.config_c1(), np.arange(0, 90, 15))
    eng = _engine(c)
    lv, jw, mu = _t(c.leaves), _t(c.jaws), _t(c.mu)
    w = _t(np.random.default_rng(5).uniform(size=c.shape))
    d0 = eng.forward(lv, jw, mu).clone()
    g0 = [x.clone() for x in eng.backward(lv, jw, mu, w)]
    eng.build_cache("fp32")
    d1 = eng.forward(lv, jw, mu)
    g1 = eng.backward(lv, jw, mu, w)
    torch.cuda.synchronize()
    assert torch.equal(d0, d1)
    for a, b in zip(g0, g1):
        assert torch.equal(a, b)
