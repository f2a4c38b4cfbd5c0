"""Pins of the oracle's ImaSk-Seq variant (Sec. 5), CPU only.

  * A single level (r = 1) is the primal-dual hybrid gradient method of
    Chambolle and Pock (dual step first, extrapolation theta), written here
    from its textbook form with dense matrices, for theta = 0 and 1.
  * Tikhonov: the iterates converge to the dense minimiser of
    1/2|Kbar x - b|^2 + lam/2 |x|^2 (Cholesky) in both sketch modes.
  * Fixed point: started at the saddle point with consistent tables and
    xbar = x, the iteration does not move.
  * Resuming from a saved state (including xbar) is bitwise identical.
"""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle
import synth

G16 = oracle.Geometry(16, 24, 24)


def _dense_sketches(g, lv):
    return [oracle.dense_matrix(lambda e, k=k: oracle.sketch_fwd(g, lv, k, e), (g.n, g.n),
                                g.n_angles * g.n_det) for k in range(lv.r)]


@pytest.mark.parametrize("theta", [0.0, 1.0])
def test_single_level_is_chambolle_pock(theta):
    """Chambolle-Pock for min_x F(Kx) + G(x) with F(z) = 1/2|z - b|^2 and
    G = lam/2 |.|^2: y+ = prox_{s F*}(y + s K xbar), x+ = prox_{t G}(x - t K^T y+),
    xbar+ = x+ + theta (x+ - x), with s = sigma and t = sigma / lam."""
    lv = oracle.Levels([0], [1.0])
    _, b = synth.ct_problem(16, 24, 24, 1e4, 1010, 2010)
    K = oracle.dense_matrix(lambda e: oracle.project(G16, 0, e), (16, 16), 24 * 24)
    lam, s = 0.5, 0.04
    t = s / lam
    bb = b.ravel()
    # prox of s F*, F*(y) = 1/2|y|^2 + <b, y>: argmin 1/2|u - v|^2 + s F*(u)
    prox_fstar = lambda v: (v - s * bb) / (1.0 + s)  # noqa: E731
    prox_g = lambda v: v / (1.0 + t * lam)  # noqa: E731
    x = np.zeros(256)
    xb = np.zeros(256)
    y = np.zeros(576)
    for _ in range(50):
        y = prox_fstar(y + s * (K @ xb))
        xn = prox_g(x - t * (K.T @ y))
        xb = xn + theta * (xn - x)
        x = xn
    st = oracle.imask_seq_run(G16, lv, oracle.Reg(lam=lam), s, theta, 1, 0, b, 50)
    np.testing.assert_allclose(st.x.ravel(), x, rtol=0, atol=1e-12 * np.abs(x).max())
    np.testing.assert_allclose(st.y.ravel(), y, rtol=0, atol=1e-12 * np.abs(y).max())
    np.testing.assert_allclose(st.xbar.ravel(), xb, rtol=0, atol=1e-12 * np.abs(xb).max())
    assert st.epochs == 50.0


@pytest.mark.parametrize("mode", [oracle.MODE_PAPER, oracle.MODE_UNBIASED])
def test_seq_tikhonov_converges_to_dense_minimiser(mode):
    lv = oracle.Levels([0, 1, 2], [1 / 3] * 3, mode)
    Ks = _dense_sketches(G16, lv)
    Kb = sum(p * K for p, K in zip(lv.p, Ks))
    _, b = synth.ct_problem(16, 24, 24, 1e4, 1011, 2011)
    lam = 1.0
    H = Kb.T @ Kb + lam * np.eye(256)
    xs = sl.cho_solve(sl.cho_factor(H), Kb.T @ b.ravel())
    # a twentieth of the single-level stability limit sigma^2 |K|^2 / lam < 1
    sigma = 0.05 * np.sqrt(lam) / max(np.linalg.norm(K, 2) for K in Ks)
    st = None
    errs = []
    for _ in range(20):
        st = oracle.imask_seq_run(G16, lv, oracle.Reg(lam=lam), sigma, 1.0, 42, 0, b, 100, st)
        errs.append(np.linalg.norm(st.x.ravel() - xs) / np.linalg.norm(xs))
    assert errs[0] > 1e-2 and errs[-1] < 1e-13
    assert all(e1 < e0 for e0, e1 in zip(errs[:12], errs[1:13]))


@pytest.mark.parametrize("mode", [oracle.MODE_PAPER, oracle.MODE_UNBIASED])
def test_seq_fixed_point(mode):
    lv = oracle.Levels([0, 1, 2], [0.5, 0.25, 0.25], mode)
    Ks = _dense_sketches(G16, lv)
    Kb = sum(p * K for p, K in zip(lv.p, Ks))
    _, b = synth.ct_problem(16, 24, 24, 1e4, 1012, 2012)
    lam = 0.1
    H = Kb.T @ Kb + lam * np.eye(256)
    xs = sl.cho_solve(sl.cho_factor(H), Kb.T @ b.ravel())
    ys = Kb @ xs - b.ravel()
    st = oracle.State(xs.reshape(16, 16).copy(), ys.reshape(24, 24).copy(),
                      np.stack([(K.T @ ys).reshape(16, 16) for K in Ks]),
                      np.stack([(K @ xs).reshape(24, 24) for K in Ks]), xbar=xs.reshape(16, 16).copy())
    out = oracle.imask_seq_run(G16, lv, oracle.Reg(lam=lam), 0.05, 1.0, 42, 0, b, 40, st)
    assert len(set(out.draws)) == 3
    np.testing.assert_allclose(out.x, st.x, rtol=0, atol=1e-11 * np.abs(xs).max())
    np.testing.assert_allclose(out.xbar, st.x, rtol=0, atol=1e-11 * np.abs(xs).max())
    np.testing.assert_allclose(out.y, st.y, rtol=0, atol=1e-11 * np.abs(ys).max())


def test_seq_resume_is_bitwise():
    lv = oracle.Levels([0, 1, 2], [1 / 3] * 3)
    _, b = synth.ct_problem(16, 24, 24, 1e4, 1013, 2013)
    reg = oracle.Reg(oracle.REG_SMOOTH_TV, lam=0.1, tv_weight=0.02, tv_eps=0.05, tv_inner=5)
    whole = oracle.imask_seq_run(G16, lv, reg, 0.03, 1.0, 42, 2, b, 30)
    half = oracle.imask_seq_run(G16, lv, reg, 0.03, 1.0, 42, 2, b, 15)
    rest = oracle.imask_seq_run(G16, lv, reg, 0.03, 1.0, 42, 2, b, 15, half)
    assert np.array_equal(whole.x, rest.x) and np.array_equal(whole.y, rest.y)
    assert np.array_equal(whole.xbar, rest.xbar)
    assert np.array_equal(whole.phi, rest.phi) and np.array_equal(whole.psi, rest.psi)
    assert whole.draws == rest.draws and whole.epochs == rest.epochs


def test_seq_differs_from_parallel():
    """Same draws and step: the two schedules give different iterates."""
    lv = oracle.Levels([0, 1, 2], [1 / 3] * 3)
    _, b = synth.ct_problem(16, 24, 24, 1e4, 1014, 2014)
    par = oracle.imask_run(G16, lv, oracle.Reg(lam=0.5), 0.02, 42, 0, b, 10)
    seq = oracle.imask_seq_run(G16, lv, oracle.Reg(lam=0.5), 0.02, 0.0, 42, 0, b, 10)
    assert par.draws == seq.draws
    assert np.linalg.norm(par.x - seq.x) > 1e-3 * np.linalg.norm(par.x)
