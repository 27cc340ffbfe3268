"""Plan optimisation workload on the GPU: Adam from closed apertures on the
two-arc 192 x 192 x 128 geometry with the workload's quadratic objective and with
the paper's weighted L1 objective (coarse-to-fine kernel sizes on geometry
caches, weight selection by isodose Dice).  Also checks the projection layer
against the oracle's projection (seeded inputs) and its Jacobian against finite
differences.  The optimised plans are checked by properties (objective decrease,
feasibility, Dice), and the 200-step plan's final dose and objective against the
oracle's recomputation from the same projected parameters."""
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
    from paper_2512_18863_amd import engine as E
    from paper_2512_18863_amd import optimize
    case = optimize.c3_case()
    masks = inputs.structures_c3(case)
    _say("C3 optimisation: %d CPs, grid %s, 200 Adam steps" % (case.n_cp, case.shape))
    opt = optimize.PlanOptimizer(case, masks)
    losses, sec_per_step = opt.run(200)
    lv, jw, mu, dose = opt.final()
    L_end = float(optimize.objective(dose, opt.masks))
    _say("C3: %.2f ms/step, L: %.3f -> %.3f (final eval %.4f)" % (1e3 * sec_per_step, losses[0], losses[-1], L_end))
    assert losses[-1] < 0.25 * losses[0]
    assert L_end < 0.25 * losses[0]
    # the final parameters are feasible: projecting them again moves nothing beyond
    # FP32 rounding of the centre / width round trip (values up to 50 mm)
    again = E.project_params(_t(lv), _t(jw), _t(mu), opt.limits)
    for a, b in zip(again, (lv, jw, mu)):
        np.testing.assert_allclose(a.cpu().numpy(), b, rtol=0, atol=2e-5)
    assert (lv[:, 1] - lv[:, 0] >= opt.limits["w_min"] - 1e-4).all() and (mu >= opt.limits["mu_min"] - 1e-6).all()
    # the final plan's dose and objective recomputed by the oracle from the projected
    # parameters (plain inputs to both paths: the oracle takes nothing else from the
    # GPU).  Dose bar: 1e-5 of max dose.  Objective: with delta = max|D_gpu - D_oracle|
    # each of the three terms T (a mean of squares) moves by at most 2 delta sqrt(T) +
    # delta^2, so |dL| <= 2 delta sqrt(3 L) + 3 delta^2 (Cauchy-Schwarz over the terms).
    _say("C3: oracle recomputes the final dose of all %d control points" % case.n_cp)
    m = oracle.Model(case)
    ref = oracle.forward(m, oracle.density(m), case.gantry, lv, jw, mu)
    got = dose.cpu().numpy().astype(np.float64)
    delta = float(np.abs(got - ref).max())
    L_ref = float(optimize.objective(torch.tensor(ref), {k: torch.tensor(v) for k, v in masks.items()}))
    bound = 2.0 * delta * np.sqrt(3.0 * L_ref) + 3.0 * delta ** 2 + 1e-6 * L_ref
    _say("C3 final: max|dD|/maxD = %.3e, L(gpu) = %.6f, L(oracle dose) = %.6f, |dL| = %.2e (bound %.2e)"
         % (delta / ref.max(), L_end, L_ref, abs(L_end - L_ref), bound))
    assert delta <= 1e-5 * ref.max()
    assert abs(L_end - L_ref) <= bound


def test_c3_l1_objective_coarse_to_fine_with_cache():
    """The paper's weighted L1 objective (§2.5) from the closed start: 100 steps with
    9 x 9 kernels, then 40 with the workload's 31 x 31, both on geometry caches."""
    from paper_2512_18863_amd import optimize
    case = optimize.c3_case()
    masks = inputs.structures_c3(case)
    w = {"ptv": 100.0, "rectum": 1.0, "bladder": 1.0, "femur_l": 0.1, "femur_r": 0.1, "external": 0.1}
    _say("C3 L1 objective, stages n=9 (100 steps) -> n=31 (40 steps), FP32 geometry caches")
    opt = optimize.PlanOptimizer(case, masks, objective="l1", weights=w, rx=78.0, cache="fp32")
    runs = opt.run_stages([optimize.Stage(100, n_taps=9), optimize.Stage(40, n_taps=31)])
    (_, l9, s9), (_, l31, s31) = runs
    dose = opt.final()[3]
    dice = opt.dice(dose)
    _say("L1: %.4g -> %.4g (n=9, %.1f ms/step) -> %.4g (n=31, %.1f ms/step); Dice(100%% isodose, PTV) = %.3f"
         % (l9[0], l9[-1], 1e3 * s9, l31[-1], 1e3 * s31, dice))
    rep = opt.evaluator.report(dose, rx=78.0, voxel_cc=2.5 ** 3 / 1000.0, bin_width=0.01)
    _say("PTV D98 %.2f D50 %.2f D2 %.2f Gy; rectum Dmean %.2f, bladder Dmean %.2f Gy"
         % (rep["ptv"]["D98"], rep["ptv"]["D50"], rep["ptv"]["D2"], rep["rectum"]["Dmean"], rep["bladder"]["Dmean"]))
    assert l9[-1] < 0.3 * l9[0] and l31[-1] < 0.3 * l9[0]
    assert dice > 0.3


def test_weight_search_keeps_the_best_dice():
    from paper_2512_18863_amd import optimize
    case = optimize.c3_case()
    masks = inputs.structures_c3(case)
    _say("weight search over two OAR weight combinations (100 steps each, n=9, cached)")
    combos = [{"rectum": 0.0, "bladder": 0.0}, {"rectum": 100.0, "bladder": 100.0}]
    best, dice, res = optimize.weight_search(case, masks, ["rectum", "bladder"], [optimize.Stage(100, n_taps=9)],
                                             rx=78.0, combos=combos)
    _say("results (rectum/bladder weight, Dice): %s" % [(r[0]["rectum"], round(r[1], 3)) for r in res])
    assert dice == max(r[1] for r in res) and best in [r[0] for r in res]
    assert dice > 0.3
