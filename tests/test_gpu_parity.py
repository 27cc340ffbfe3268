"""GPU forward parity: the HIP path through the C ABI against the FP64 oracle.

Bar (FP32 path): max |D_gpu - D_oracle| <= 1e-5 * max D_oracle, element by
element on the same seeded inputs.  Intermediates are compared kernel by
kernel on small problems.  Invariants that hold exactly in any precision are
checked bit for bit.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2512_18863_amd import inputs

pytestmark = pytest.mark.gpu

TOL_FWD = 1e-5          # of max dose, FP32 path vs FP64 oracle


def _say(msg):
    print("[gpu-test] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_18863_amd import engine  # noqa: F401  (raises if the library is missing)


def _t(a, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def gpu_dose(case, conv="fp32", n_taps=None, wepl_mode=None, max_cp_batch=0, leaves=None, jaws=None, mu=None):
    from paper_2512_18863_amd.engine import DoseEngine
    eng = DoseEngine(case, conv=conv, n_taps=n_taps, wepl_mode=wepl_mode, max_cp_batch=max_cp_batch)
    lv = case.leaves if leaves is None else leaves
    jw = case.jaws if jaws is None else jaws
    m = case.mu if mu is None else mu
    d = eng.forward(_t(lv), _t(jw), _t(m))
    torch.cuda.synchronize()
    return d.cpu().numpy().astype(np.float64), eng


def oracle_dose(case, n_taps=None, wepl_mode=None):
    m = oracle.Model(case, n_taps=n_taps, wepl_mode=wepl_mode)
    rho = oracle.density(m)
    return oracle.forward(m, rho, case.gantry, case.leaves, case.jaws, case.mu,
                          coll=getattr(case, "collimator", None)), m, rho


def _rel_err(a, ref):
    return float(np.abs(a - ref).max() / np.abs(ref).max())


def subset(case, idx):
    """The same problem restricted to the control points idx."""
    import copy
    c = copy.copy(case)
    c.gantry = case.gantry[idx]
    c.leaves = case.leaves[idx]
    c.jaws = case.jaws[idx]
    c.mu = case.mu[idx]
    if getattr(case, "collimator", None) is not None:
        c.collimator = case.collimator[idx]
    return c


# ------------------------------------------------------------------ forward


def test_c0_forward_parity():
    _say("C0 forward fp32 (32^3 water, n=7, 1 CP)")
    c = inputs.config_c0()
    ref, _, _ = oracle_dose(c)
    got, _ = gpu_dose(c)
    err = _rel_err(got, ref)
    _say("C0 max|dD|/maxD = %.3e" % err)
    assert err <= TOL_FWD


def test_c0_intermediates():
    _say("C0 intermediates F, z, P, Dfan")
    c = inputs.config_c0()
    m = oracle.Model(c)
    rho = oracle.density(m)
    r = oracle.forward_cp(m, rho, c.gantry[0], c.leaves[0], c.jaws[0])
    _, eng = gpu_dose(c)
    Nk, Nu, Nv = eng.fan_shape()
    assert (Nu, Nv, Nk) == (m.Nu, m.Nv, m.Nk)
    F = eng.ws_view("fluence", (1, Nu, Nv)).cpu().numpy()[0].T            # -> [Nv][Nu]
    z = eng.ws_view("depth", (1, Nk)).cpu().numpy()[0]
    Dfan = eng.ws_view("vol1", (1, Nk, Nu, Nv)).cpu().numpy()[0].transpose(0, 2, 1)
    P = eng.ws_view("vol0", (1, Nk, Nu, Nv)).cpu().numpy()[0].transpose(0, 2, 1)
    # leaf positions enter as FP32 (|l| <= 50 mm: rounding <= 4e-6 mm, i.e. <= 8e-7 of a 5 mm pixel)
    np.testing.assert_allclose(F, r["F"], rtol=0, atol=1e-6)
    np.testing.assert_allclose(z, r["z"], rtol=2e-6, atol=1e-4)
    assert np.abs(P - r["P"]).max() <= 2e-6 * np.abs(r["P"]).max()
    assert np.abs(Dfan - r["Dfan"]).max() <= 5e-6 * np.abs(r["Dfan"]).max()


def test_c0_exact_invariants():
    _say("C0 invariants: closed jaws / zero MU give 0, MU x2 bitwise, x-mirror")
    c = inputs.config_c0()
    d, eng = gpu_dose(c)
    cj = inputs.config_c0("jaws_closed")
    z1 = eng.forward(_t(cj.leaves), _t(cj.jaws), _t(cj.mu)).cpu().numpy()
    z2 = eng.forward(_t(c.leaves), _t(c.jaws), _t(np.zeros(1))).cpu().numpy()
    assert np.all(z1 == 0.0) and np.all(z2 == 0.0)
    d2 = eng.forward(_t(c.leaves), _t(c.jaws), _t(2 * c.mu)).cpu().numpy().astype(np.float64)
    assert np.array_equal(d2, 2.0 * d)
    cm = inputs.config_c0("mirror")
    jm = c.jaws[:, [1, 0, 2, 3]] * np.array([-1, -1, 1, 1])
    dm = eng.forward(_t(cm.leaves), _t(jm), _t(cm.mu)).cpu().numpy()
    assert np.abs(dm - d[:, :, ::-1]).max() <= 1e-6 * d.max()
    cl = inputs.config_c0("leaves_closed")
    d0, _ = gpu_dose(cl)
    assert np.all(d0 == 0.0)


TINY = [
    dict(seed=7, n_taps=3),
    dict(seed=8, n_taps=5, gantry=[0.0, 90.0]),
    dict(seed=9, n_taps=3, wepl_mode=inputs.WEPL_CENTRAL_AXIS),
    dict(seed=11, n_taps=1),
    dict(seed=12, n_taps=9, shape=(7, 9, 8), spacing=7.0, field=35.0),
    dict(seed=13, n_taps=15, shape=(9, 8, 10), spacing=6.0, field=40.0),      # MFMA path, ragged tiles
    dict(seed=14, n_taps=31, shape=(8, 8, 8), spacing=5.0, field=30.0, n_cp=3),
    dict(seed=15, n_taps=13, shape=(1, 5, 4), spacing=8.0, field=20.0),      # a single slice
    # a 115 x 115 beam-frame plane: several convolution regions in both directions
    dict(seed=16, n_taps=15, shape=(10, 12, 11), spacing=3.0, field=150.0, n_leaf=30, leaf_width=10.0),
    # small kernels on a 107 x 107 plane: the vector-ALU convolution splits it into two row bands
    dict(seed=17, n_taps=9, shape=(10, 12, 11), spacing=3.0, field=150.0, n_leaf=30, leaf_width=10.0),
    dict(seed=18, n_taps=11, shape=(7, 6, 8), spacing=6.0, field=40.0),
    dict(seed=19, n_taps=7, shape=(6, 7, 5), spacing=7.0, field=30.0, n_cp=3),
]


@pytest.mark.parametrize("kw", TINY, ids=[str(i) for i in range(len(TINY))])
def test_tiny_forward_parity(kw):
    _say("tiny forward %s" % kw)
    kw = dict(kw)
    kw.setdefault("shape", (5, 6, 5))
    kw.setdefault("spacing", 10.0)
    kw.setdefault("field", 25.0)
    c = inputs.tiny_case(**kw)
    ref, _, _ = oracle_dose(c)
    got, _ = gpu_dose(c)
    err = _rel_err(got, ref)
    _say("max|dD|/maxD = %.3e" % err)
    assert err <= TOL_FWD


def test_batched_equals_whole_plan():
    _say("C1 12 CPs: CP batches of 5 vs whole plan")
    c = subset(inputs.config_c1(), np.arange(0, 90, 7)[:12])
    a, _ = gpu_dose(c)
    b, _ = gpu_dose(c, max_cp_batch=5)
    assert np.abs(a - b).max() <= 1e-6 * a.max()


def test_c1_forward_parity():
    _say("C1 forward fp32 (128x128x96 pelvis, 90 CPs, n=15)")
    c = inputs.config_c1()
    ref, _, _ = oracle_dose(c)
    got, _ = gpu_dose(c)
    err = _rel_err(got, ref)
    _say("C1 max|dD|/maxD = %.3e" % err)
    assert err <= TOL_FWD


def test_c1_central_axis_mode_parity():
    _say("C1 central-axis depth mode, 10 CPs")
    c = subset(inputs.config_c1(), np.arange(0, 90, 9))
    ref, _, _ = oracle_dose(c, wepl_mode=inputs.WEPL_CENTRAL_AXIS)
    got, _ = gpu_dose(c, wepl_mode=inputs.WEPL_CENTRAL_AXIS)
    assert _rel_err(got, ref) <= TOL_FWD


def test_c2_forward_parity_subset():
    _say("C2 forward fp32 (192x192x128 at 2.5 mm, n=31), 20 of 180 CPs")
    c = subset(inputs.config_c2(), np.arange(0, 180, 9))
    ref, _, _ = oracle_dose(c)
    got, _ = gpu_dose(c)
    err = _rel_err(got, ref)
    _say("C2 max|dD|/maxD = %.3e" % err)
    assert err <= TOL_FWD


def test_c4bench_forward_parity_subset():
    _say("C4-bench forward fp32 (128^3 at 3 mm, n=61), 4 of 180 CPs")
    c = subset(inputs.config_c4_plan(2000, bench=True), np.array([0, 45, 97, 170]))
    ref, _, _ = oracle_dose(c)
    got, _ = gpu_dose(c)
    err = _rel_err(got, ref)
    _say("C4-bench max|dD|/maxD = %.3e" % err)
    assert err <= TOL_FWD


def test_full_plan_c4bench_sampled_voxels():
    """Full 180-CP C4-bench plan in the launch configuration the benchmark times;
    the oracle recomputes a sample of voxels from the control points that reach them
    (dose is linear over control points, so a voxel sample of a CP subset is exact)."""
    _say("C4-bench full plan fp32, 180 CPs; oracle on 6 CPs for sampled comparison")
    c = inputs.config_c4_plan(2000, bench=True)
    got, eng = gpu_dose(c)
    assert np.isfinite(got).all() and got.max() > 0
    idx = np.array([3, 60, 91, 122, 150, 177])
    mu0 = np.zeros_like(c.mu)
    mu0[idx] = c.mu[idx]
    part = eng.forward(_t(c.leaves), _t(c.jaws), _t(mu0)).cpu().numpy().astype(np.float64)
    ref, _, _ = oracle_dose(subset(c, idx))
    assert _rel_err(part, ref) <= TOL_FWD
