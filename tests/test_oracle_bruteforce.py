"""Oracle vs the pure-Python brute force on tiny heterogeneous grids (1e-12)."""
import numpy as np
import pytest

import oracle
from paper_2512_18863_amd import inputs
from tests.bruteforce import BruteForce


@pytest.mark.parametrize("seed,n_taps,mode,gantry", [
    (7, 3, inputs.WEPL_PER_RAY, None),
    (8, 5, inputs.WEPL_PER_RAY, [0.0, 90.0]),
    (9, 3, inputs.WEPL_CENTRAL_AXIS, None),
])
def test_forward_matches_bruteforce(seed, n_taps, mode, gantry):
    c = inputs.tiny_case(seed=seed, n_cp=2, n_taps=n_taps, shape=(5, 6, 5), spacing=10.0, field=25.0,
                         wepl_mode=mode, gantry=gantry)
    m = oracle.Model(c)
    rho = oracle.density(m)
    dose = oracle.forward(m, rho, c.gantry, c.leaves, c.jaws, c.mu)
    bf = BruteForce(c, rho)
    assert (bf.Nu, bf.Nv, bf.Nk) == (m.Nu, m.Nv, m.Nk)
    ref = bf.dose()
    assert ref.max() > 0
    np.testing.assert_allclose(dose, ref, rtol=0, atol=1e-12 * ref.max())


def test_intermediates_match_bruteforce():
    c = inputs.tiny_case(seed=10, n_cp=1, n_taps=3, shape=(5, 5, 6), spacing=10.0, field=25.0)
    m = oracle.Model(c)
    rho = oracle.density(m)
    r = oracle.forward_cp(m, rho, c.gantry[0], c.leaves[0], c.jaws[0])
    bf = BruteForce(c, rho)
    for (k, j, i) in [(3, 4, 4), (7, 2, 5), (m.Nk - 1, 0, 0), (5, m.Nv - 1, 3)]:
        assert abs(r["W"][k, j, i] - bf.wepl_node(0, k, j, i)) < 1e-12
        assert abs(r["P"][k, j, i] - bf.primary(0, k, j, i)) < 1e-12
        assert abs(r["Dfan"][k, j, i] - bf.beam_dose_node(0, k, j, i)) < 1e-12
    for j in range(m.Nv):
        for i in range(m.Nu):
            assert abs(r["F"][j, i] - bf.fluence(0, j, i)) < 1e-15
