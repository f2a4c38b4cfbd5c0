"""Pins of the oracle's Algorithm 1 (ImaSk) and its proximal maps, CPU only.

  * Tikhonov: the iterates converge linearly to the dense minimiser of
    1/2|Kbar x - b|^2 + lam/2 |x|^2 (Cholesky), and the mean squared error
    over independent draw streams stays under Thm. 1's bound theta^K C/mu.
  * Fixed point: started at the saddle point with consistent gradient
    tables, the iteration does not move (pins signs, the sigma/mu placement
    and the use of the old table averages).
  * r = 1 reduces to the deterministic primal-dual recursion.
  * Smoothed TV: closed-form TV value of a step edge, gradient against
    finite differences, prox against an independent L-BFGS solve, and the
    fixed point of the TV problem (minimiser from torch autograd + L-BFGS).
  * Resuming from a saved state is bitwise identical to an unbroken run.
"""
import numpy as np
import pytest
import scipy.linalg as sl
import scipy.optimize as so

import oracle
import synth
from oracle import steps

G16 = oracle.Geometry(16, 24, 24)


def _dense_sketches(g, lv):
    return [oracle.dense_matrix(lambda e, k=k: oracle.sketch_fwd(g, lv, k, e), (g.n, g.n),
                                g.n_angles * g.n_det) for k in range(lv.r)]


def _tikhonov_minimiser(Kb, b, lam):
    H = Kb.T @ Kb + lam * np.eye(Kb.shape[1])
    return sl.cho_solve(sl.cho_factor(H), Kb.T @ b.ravel())


@pytest.mark.parametrize("mode", [oracle.MODE_PAPER, oracle.MODE_UNBIASED])
def test_tikhonov_converges_to_dense_minimiser(mode):
    lv = oracle.Levels([0, 1, 2], [1 / 3] * 3, mode)
    Ks = _dense_sketches(G16, lv)
    Kb = sum(p * K for p, K in zip(lv.p, Ks))
    _, b = synth.ct_problem(16, 24, 24, 1e4, 1000, 2000)
    lam = 1.0
    xs = _tikhonov_minimiser(Kb, b, lam)
    L2, lb, lp = steps.constants_dense(Ks, lv.p, lam)
    sigma, _, _, _ = steps.sigma_thm3(L2, lb, lp, min(lv.p), 60, 60)
    st = None
    errs = []
    for _ in range(30):
        st = oracle.imask_run(G16, lv, oracle.Reg(lam=lam), sigma, 42, 0, b, 100, st)
        errs.append(np.linalg.norm(st.x.ravel() - xs) / np.linalg.norm(xs))
    errs = np.array(errs)
    assert errs[-1] < 1e-12
    # linear rate: log-error is close to a straight line while above rounding
    live = errs > 1e-13
    kk = np.arange(1, len(errs) + 1)[live]
    slope, icpt = np.polyfit(kk, np.log(errs[live]), 1)
    resid = np.log(errs[live]) - (slope * kk + icpt)
    r2 = 1 - np.sum(resid ** 2) / np.sum((np.log(errs[live]) - np.log(errs[live]).mean()) ** 2)
    assert slope < 0 and r2 > 0.95


def test_thm1_bound_in_expectation():
    lv = oracle.Levels([0, 1, 2], [1 / 3] * 3, oracle.MODE_UNBIASED)
    Ks = _dense_sketches(G16, lv)
    Kb = sum(p * K for p, K in zip(lv.p, Ks))
    _, b = synth.ct_problem(16, 24, 24, 1e4, 1001, 2001)
    lam = 1.0
    xs = _tikhonov_minimiser(Kb, b, lam)
    ys = Kb @ xs - b.ravel()
    L2, lb, lp = steps.constants_dense(Ks, lv.p, lam)
    sigma, th, c, rho = steps.sigma_thm3(L2, lb, lp, min(lv.p), 60, 60)
    bb = rho * c / lb
    # C = |z0 - z*|^2 + b sum_i p_i^{-1} |B_i z*|^2 in normalised variables
    C = lam * xs @ xs + ys @ ys
    C += bb * sum(p * (np.sum((K.T @ ys) ** 2) / lam + np.sum((K @ xs) ** 2)) for p, K in zip(lv.p, Ks))
    for K in (50, 150):
        sq = [np.sum((oracle.imask_run(G16, lv, oracle.Reg(lam=lam), sigma, 42, s, b, K).x.ravel() - xs) ** 2)
              for s in range(16)]
        assert np.mean(sq) <= th ** K * C / lam


@pytest.mark.parametrize("mode", [oracle.MODE_PAPER, oracle.MODE_UNBIASED])
def test_fixed_point_tikhonov(mode):
    lv = oracle.Levels([0, 1, 2], [0.5, 0.25, 0.25], mode)
    Ks = _dense_sketches(G16, lv)
    Kb = sum(p * K for p, K in zip(lv.p, Ks))
    _, b = synth.ct_problem(16, 24, 24, 1e4, 1002, 2002)
    lam = 0.1
    xs = _tikhonov_minimiser(Kb, b, lam)
    ys = Kb @ xs - b.ravel()
    st = oracle.State(xs.reshape(16, 16).copy(), ys.reshape(24, 24).copy(),
                      np.stack([(K.T @ ys).reshape(16, 16) for K in Ks]),
                      np.stack([(K @ xs).reshape(24, 24) for K in Ks]))
    out = oracle.imask_run(G16, lv, oracle.Reg(lam=lam), 0.05, 42, 0, b, 40, st)
    assert len(set(out.draws)) == 3
    np.testing.assert_allclose(out.x, st.x, rtol=0, atol=1e-11 * np.abs(xs).max())
    np.testing.assert_allclose(out.y, st.y, rtol=0, atol=1e-11 * np.abs(ys).max())


def test_single_level_is_deterministic_primal_dual():
    lv = oracle.Levels([0], [1.0])
    _, b = synth.ct_problem(16, 24, 24, 1e4, 1003, 2003)
    K = oracle.dense_matrix(lambda e: oracle.project(G16, 0, e), (16, 16), 24 * 24)
    lam, sigma = 0.5, 0.04
    x = np.zeros(256)
    y = np.zeros(576)
    for _ in range(50):
        x, y = (x - (sigma / lam) * (K.T @ y)) / (1 + sigma), (y + sigma * (K @ x) - sigma * b.ravel()) / (1 + sigma)
    st = oracle.imask_run(G16, lv, oracle.Reg(lam=lam), sigma, 1, 0, b, 50)
    np.testing.assert_allclose(st.x.ravel(), x, rtol=0, atol=1e-12 * np.abs(x).max())
    np.testing.assert_allclose(st.y.ravel(), y, rtol=0, atol=1e-12 * np.abs(y).max())
    assert st.epochs == 50.0


def test_resume_is_bitwise():
    lv = oracle.Levels([0, 1, 2], [1 / 3] * 3)
    _, b = synth.ct_problem(16, 24, 24, 1e4, 1004, 2004)
    reg = oracle.Reg(oracle.REG_SMOOTH_TV, lam=0.1, tv_weight=0.02, tv_eps=0.05, tv_inner=5)
    whole = oracle.imask_run(G16, lv, reg, 0.03, 42, 2, b, 30)
    half = oracle.imask_run(G16, lv, reg, 0.03, 42, 2, b, 15)
    rest = oracle.imask_run(G16, lv, reg, 0.03, 42, 2, b, 15, half)
    assert np.array_equal(whole.x, rest.x) and np.array_equal(whole.y, rest.y)
    assert np.array_equal(whole.phi, rest.phi) and np.array_equal(whole.psi, rest.psi)
    assert whole.draws == rest.draws and whole.epochs == rest.epochs


# ------------------------------------------------------------ smoothed TV

def test_tv_value_of_step_edge():
    n, eps = 16, 1e-3
    u = np.zeros((n, n))
    u[:, n // 2:] = 1.0
    expect = n * np.sqrt(1 + eps ** 2) + (n * n - n) * eps
    assert abs(oracle.tv_value(u, eps) - expect) < 1e-12


def test_tv_gradient_matches_finite_differences():
    n, eps = 8, 0.05
    u = synth.random_image(n, 9)
    g = oracle.tv_gradient(u, eps)
    h = 1e-6
    rng = np.random.default_rng(0)
    for _ in range(20):
        i, j = rng.integers(0, n, size=2)
        up, um = u.copy(), u.copy()
        up[i, j] += h
        um[i, j] -= h
        fd = (oracle.tv_value(up, eps) - oracle.tv_value(um, eps)) / (2 * h)
        assert abs(fd - g[i, j]) < 1e-6


def _torch_objective(Kb, b, lam, w, eps, n):
    import torch

    Kt = torch.from_numpy(Kb)
    bt = torch.from_numpy(b.ravel())

    def f(xv):
        x = torch.tensor(xv, dtype=torch.float64, requires_grad=True)
        u = x.view(n, n)
        g1 = torch.zeros_like(u)
        g2 = torch.zeros_like(u)
        g1[:-1, :] = u[1:, :] - u[:-1, :]
        g2[:, :-1] = u[:, 1:] - u[:, :-1]
        val = 0.5 * torch.sum((Kt @ x - bt) ** 2) + w * torch.sum(torch.sqrt(g1 ** 2 + g2 ** 2 + eps ** 2)) \
            + 0.5 * lam * torch.sum(x ** 2)
        val.backward()
        return val.item(), x.grad.numpy().copy()

    return f


def test_tv_prox_matches_lbfgs():
    n, eps, w, tau, lam = 8, 0.1, 0.3, 0.7, 0.2
    v = synth.random_image(n, 10)
    ref = so.minimize(_torch_objective(np.eye(n * n), v, tau * lam, tau * w, eps, n), np.zeros(n * n),
                      jac=True, method="L-BFGS-B", options={"gtol": 1e-13, "ftol": 1e-15, "maxiter": 20000})
    out = oracle.tv_prox(v, v, tau, lam, w, eps, 4000)
    np.testing.assert_allclose(out.ravel(), ref.x, rtol=0, atol=2e-7)


def test_tv_prox_constant_and_exact_start():
    n, tau, lam = 8, 0.5, 0.4
    v = np.full((n, n), 0.8)
    exact = v / (1 + tau * lam)
    np.testing.assert_allclose(oracle.tv_prox(v, exact, tau, lam, 1.0, 1e-3, 10), exact, rtol=0, atol=1e-15)
    # without TV the inner problem is a scalar quadratic solved in one step
    np.testing.assert_allclose(oracle.tv_prox(v, v, tau, lam, 0.0, 1e-3, 1), exact, rtol=0, atol=1e-15)


def test_fixed_point_smooth_tv():
    n = 8
    g = oracle.Geometry(n, 12, 12)
    lv = oracle.Levels([0, 1, 2], [1 / 3] * 3, oracle.MODE_UNBIASED)
    Ks = _dense_sketches(g, lv)
    Kb = sum(p * K for p, K in zip(lv.p, Ks))
    _, b = synth.ct_problem(n, 12, 12, 1e4, 1005, 2005)
    lam, w, eps = 0.1, 0.05, 0.05
    res = so.minimize(_torch_objective(Kb, b, lam, w, eps, n), np.zeros(n * n), jac=True, method="L-BFGS-B",
                      options={"gtol": 1e-13, "ftol": 1e-16, "maxiter": 50000})
    xs = res.x
    ys = Kb @ xs - b.ravel()
    st = oracle.State(xs.reshape(n, n).copy(), ys.reshape(12, 12).copy(),
                      np.stack([(K.T @ ys).reshape(n, n) for K in Ks]),
                      np.stack([(K @ xs).reshape(12, 12) for K in Ks]))
    reg = oracle.Reg(oracle.REG_SMOOTH_TV, lam=lam, tv_weight=w, tv_eps=eps, tv_inner=10)
    out = oracle.imask_run(g, lv, reg, 0.05, 42, 0, b, 20, st)
    assert np.abs(out.x - st.x).max() < 1e-6 * np.abs(xs).max()
    # ... whereas a wrong-signed TV term would move it away
    bad = oracle.Reg(oracle.REG_SMOOTH_TV, lam=lam, tv_weight=-w, tv_eps=eps, tv_inner=10)
    out_bad = oracle.imask_run(g, lv, bad, 0.05, 42, 0, b, 20, st)
    assert np.abs(out_bad.x - st.x).max() > 1e-3 * np.abs(xs).max()
