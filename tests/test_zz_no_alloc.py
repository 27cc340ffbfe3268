"""The allocation-free forward (pdrt_dose_forward_noalloc, static device scratch)
against pdrt_dose_forward on the same inputs, through the C ABI.

Bar: max |D_noalloc - D_forward| <= 1e-5 * max D (the FP32 parity bar); the two
differ only in how the control points are grouped into batches, and the
compensated sum is carried across batches, so equality is expected.  Three calls
in a row, each smaller than the one before, so a later call must not see what
an earlier one left in the shared scratch.
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_2512_18863_amd import inputs
from tests.test_gpu_parity import _say, _t

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _both(case, **kw):
    from paper_2512_18863_amd import engine as E
    eng = E.DoseEngine(case, **kw)
    lv, jw, mu = _t(case.leaves), _t(case.jaws), _t(case.mu)
    ref = eng.forward(lv, jw, mu)
    out = torch.full(eng.vol_shape, float("nan"), dtype=torch.float32, device=eng.device)
    eng.forward_noalloc(lv, jw, mu, out)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy(), eng


def _compare(name, ref, got):
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max() / scale
    _say("%s: max|dD|/maxD = %.3e, bitwise equal: %s" % (name, err, np.array_equal(got, ref)))
    assert np.isfinite(got).all(), name
    assert scale > 0 and err <= TOL, name


def test_noalloc_forward_matches_forward_on_successively_smaller_plans():
    # 1: the 128^3 benchmark plan (180 control points, n = 61): about nine control
    #    points per scratch batch, so about twenty batches
    c1 = inputs.config_c4_plan(2000, bench=True)
    _say("noalloc call 1: 128^3, %d CPs, n=%d" % (c1.n_cp, c1.n_taps))
    ref, got, _ = _both(c1)
    _compare("128^3 benchmark plan", ref, got)
    # 2: smaller CT, fewer control points, smaller kernel (C1 shape)
    c2 = inputs.config_c1(n_cp=40)
    _say("noalloc call 2: %s, %d CPs, n=%d" % (c2.shape, c2.n_cp, c2.n_taps))
    ref, got, _ = _both(c2)
    _compare("C1 shape, 40 CPs", ref, got)
    # 3: tiny, BF16 convolution, with a caller batch cap of 2
    c3 = inputs.tiny_case(seed=91, n_cp=5, n_taps=15, shape=(9, 10, 11), spacing=6.0, field=30.0)
    _say("noalloc call 3: tiny %s, %d CPs, batch cap 2, bf16" % (c3.shape, c3.n_cp))
    ref, got, _ = _both(c3, conv="bf16", max_cp_batch=2)
    _compare("tiny, bf16, batch cap 2", ref, got)
