"""Plan optimisation workload on the GPU: 200 Adam steps from closed apertures on
the two-arc 192 x 192 x 128 geometry; the final objective is recomputed from the
FP64 oracle's dose of the final (projected) parameters.  Also checks the
projection layer against the oracle's projection and its Jacobian against
finite differences."""
import numpy as np
import pytest
import torch

import oracle
from paper_2512_18863_amd import inputs
from tests.test_gpu_parity import _say, _t

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_projection_matches_oracle_and_jacobian():
    _say("projection layer vs oracle; Jacobian vs central differences")
    from paper_2512_18863_amd import engine as E
    rng = np.random.default_rng(8)
    lv = rng.uniform(-70, 70, size=(5, 2, 12))
    jw = rng.uniform(-70, 70, size=(5, 4))
    mu = rng.uniform(-1, 3, size=5)
    lim = {"leaf": 50.0, "jaw_x": 45.0, "jaw_y": 40.0, "w_min": 1.0, "mu_min": 0.22}
    got = [t.cpu().numpy() for t in E.project_params(_t(lv), _t(jw), _t(mu), lim)]
    ref = oracle.project(lv, jw, mu, 50.0, 45.0, 40.0, 1.0, 0.22)
    for a, b in zip(got, ref):
        np.testing.assert_allclose(a, b, rtol=0, atol=2e-5)
    g = [rng.normal(size=x.shape) for x in (lv, jw, mu)]
    ste = [t.cpu().numpy() for t in E.project_params_backward(_t(lv), _t(jw), _t(mu), lim, *map(_t, g), True)]
    for a, b in zip(ste, g):
        np.testing.assert_allclose(a, b, rtol=1e-6)
    jac = [t.cpu().numpy() for t in E.project_params_backward(_t(lv), _t(jw), _t(mu), lim, *map(_t, g), False)]

    def lin(l_, j_, m_):
        out = oracle.project(l_, j_, m_, 50.0, 45.0, 40.0, 1.0, 0.22)
        return sum(float(np.vdot(o, gg)) for o, gg in zip(out, g))
    h = 1e-4
    for (arr, idx, jg) in [(lv, (1, 0, 3), jac[0]), (lv, (2, 1, 7), jac[0]), (jw, (3, 2), jac[1]), (mu, (4,), jac[2])]:
        ap, am = [x.copy() for x in (lv, jw, mu)], [x.copy() for x in (lv, jw, mu)]
        which = 0 if arr is lv else (1 if arr is jw else 2)
        ap[which][idx] += h
        am[which][idx] -= h
        fd = (lin(*ap) - lin(*am)) / (2 * h)
        assert abs(fd - jg[idx]) < 1e-3 * max(1.0, abs(fd)), (idx, fd, jg[idx])


def test_c3_optimisation_200_steps():
    from paper_2512_18863_amd import optimize
    case = optimize.c3_case()
    masks = inputs.structures_c3(case)
    _say("C3 optimisation: %d CPs, grid %s, 200 Adam steps" % (case.n_cp, case.shape))
    opt = optimize.PlanOptimizer(case, masks)
    losses, sec_per_step = opt.run(200)
    lv, jw, mu, dose = opt.final()
    L_gpu = float(optimize.objective(dose, opt.masks))
    _say("C3: %.2f ms/step, L: %.3f -> %.3f (final eval %.4f)" % (1e3 * sec_per_step, losses[0], losses[-1], L_gpu))
    assert losses[-1] < 0.25 * losses[0]
    # oracle recomputation of the final dose and objective
    import copy
    c = copy.copy(case)
    c.leaves, c.jaws, c.mu = lv, jw, mu
    m = oracle.Model(c)
    rho = oracle.density(m)
    ref = oracle.forward(m, rho, c.gantry, lv, jw, mu)
    assert np.abs(dose.cpu().numpy() - ref).max() <= 1e-5 * ref.max()
    L_ref = float(optimize.objective(torch.tensor(ref), {k: torch.tensor(v) for k, v in masks.items()}))
    _say("C3 objective: GPU %.6f vs oracle %.6f" % (L_gpu, L_ref))
    assert abs(L_gpu - L_ref) <= 1e-4 * max(1.0, L_ref)
