"""Pins of the step-size theory (Sec. 3.5-3.6), CPU only.

  * Thm. 3's closed form (eq. (opt:cond), eq. (eta_opt)) against brute-force
    minimisation of theta = max(phi, psi) on a fine eta grid;
  * the admissible interval of the Proposition in Sec. 3.5;
  * the Remark of Sec. 3.4: identical operators with uniform p give
    L = Lbar_p = n|C| and Lbar = sqrt(n)|C|;
  * the power method against dense eigenvalues.
"""
import numpy as np
import pytest

import oracle
from oracle import steps


@pytest.mark.parametrize("seed", range(6))
def test_eta_opt_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    L2 = rng.uniform(0.5, 50)
    lb = rng.uniform(0.05, 1.0) * L2
    lp = rng.uniform(1.0, 3.0) * lb
    pmin = rng.uniform(0.05, 0.5)
    cb = steps.cbar(L2, lp)
    for c in cb * np.array([0.05, 0.3, 0.7, 0.95]):
        for rho in (0.1, 0.5, 0.9):
            eta, th = steps.eta_opt(c, rho, L2, lb, lp, pmin)
            grid = np.linspace(0.0, c, 1_000_001)
            tg = steps.theta(grid, c, rho, L2, lb, lp, pmin)
            q = int(np.argmin(tg))
            # refine around the coarse minimiser: theta has a kink at eta*
            fine = np.linspace(grid[max(q - 1, 0)], grid[min(q + 1, len(grid) - 1)], 200_001)
            tf = steps.theta(fine, c, rho, L2, lb, lp, pmin)
            qf = int(np.argmin(tf))
            assert th <= tf[qf] + 1e-13
            assert abs(tf[qf] - th) < 1e-10
            assert abs(fine[qf] - eta) < 2e-6 * c


def test_both_regimes_of_thm3_occur():
    # large pmin and tiny c: eta* = c (first case); small pmin: interior root
    L2, lb, lp = 5.0, 1.0, 5.0
    c = steps.cbar(L2, lp) * 0.01
    eta, th = steps.eta_opt(c, 0.5, L2, lb, lp, 0.9)
    assert eta == c and th == pytest.approx(1 - 0.5 * c)
    eta2, th2 = steps.eta_opt(steps.cbar(L2, lp) * 0.9, 0.5, L2, lb, lp, 0.01)
    assert 0 < eta2 < steps.cbar(L2, lp) * 0.9
    assert th2 == pytest.approx(steps.psi(eta2, steps.cbar(L2, lp) * 0.9, 0.5, L2, lb, lp, 0.01))


def test_admissible_interval():
    L2, lb, lp, pmin = 6.0, 2.0, 6.0, 1 / 3
    c = steps.cbar(L2, lp) * 0.6
    rho = 0.4
    lo, hi = steps.admissible(c, rho, L2, lb, lp, pmin)
    for eta in np.linspace(lo, hi, 50)[1:-1]:
        assert steps.theta(eta, c, rho, L2, lb, lp, pmin) < 1
    assert steps.theta(hi * 1.001, c, rho, L2, lb, lp, pmin) >= 1
    assert steps.theta(lo * 0.999, c, rho, L2, lb, lp, pmin) >= 1


def test_remark_identical_operators():
    rng = np.random.default_rng(3)
    K = rng.standard_normal((30, 20))
    n, mu = 4, 1.0
    L2, lb, lp = steps.constants_dense([K] * n, [1 / n] * n, mu)
    nc = np.linalg.norm(K / n, 2)  # C = A_i = p_i K
    assert np.sqrt(L2) == pytest.approx(n * nc, rel=1e-12)
    assert np.sqrt(lp) == pytest.approx(n * nc, rel=1e-12)
    assert np.sqrt(lb) == pytest.approx(np.sqrt(n) * nc, rel=1e-12)


def test_power_method_matches_dense():
    g = oracle.Geometry(8, 12, 12)
    lv = oracle.Levels([0, 1, 2], [0.5, 0.3, 0.2], oracle.MODE_PAPER)
    Ks = [oracle.dense_matrix(lambda e, k=k: oracle.sketch_fwd(g, lv, k, e), (8, 8), 144) for k in range(3)]
    dense = steps.constants_dense(Ks, lv.p, 0.1)
    pw = steps.constants_power(lambda k, x: oracle.sketch_fwd(g, lv, k, x),
                               lambda k, y: oracle.sketch_adj(g, lv, k, y),
                               lv.p, 0.1, (8, 8), (12, 12), iters=2000)
    np.testing.assert_allclose(pw, dense, rtol=1e-8)


def test_sigma_thm3_is_admissible_and_better_than_neighbours():
    L2, lb, lp, pmin = 6.0, 2.0, 6.0, 1 / 3
    sigma, th, c, rho = steps.sigma_thm3(L2, lb, lp, pmin, 80, 80)
    assert 0 < sigma and th < 1
    for dc in (0.9, 1.1):
        cc = min(c * dc, steps.cbar(L2, lp) * 0.999)
        assert steps.eta_opt(cc, rho, L2, lb, lp, pmin)[1] >= th - 1e-12
