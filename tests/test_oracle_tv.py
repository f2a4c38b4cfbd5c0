"""Pins of the oracle's TV + nonnegativity prior (Sec. 4.5: mu_g |grad x|_{1,2}
+ chi_{>=0}), CPU only.

  * The prox (dual fast gradient projection) on an image that is constant
    along its columns reduces to 1-D TV denoising of a step, whose solution
    has a closed form: the two plateaus move towards each other by
    gamma/m and gamma/(n-m).
  * Constant inputs: a positive constant is a fixed point, a negative one
    is projected to zero.
  * The prox agrees with an independent solver (Chambolle-Pock on the ROF
    problem with the constraint, written here with its own difference
    operators).
  * ImaSk with this prior converges to the minimiser of the full problem
    computed independently by Chambolle-Pock on the stacked operator
    [Kbar; grad] with dense matrices.
"""
import numpy as np
import pytest

import oracle
import synth


def _grad(u):
    g1 = np.zeros_like(u)
    g2 = np.zeros_like(u)
    g1[:-1, :] = u[1:, :] - u[:-1, :]
    g2[:, :-1] = u[:, 1:] - u[:, :-1]
    return g1, g2


def _grad_t(g1, g2):
    """Adjoint of _grad (checked below by a dot-product test)."""
    out = np.zeros_like(g1)
    out[1:, :] += g1[:-1, :]
    out[:-1, :] -= g1[:-1, :]
    out[:, 1:] += g2[:, :-1]
    out[:, :-1] -= g2[:, :-1]
    return out


def test_difference_operators_are_adjoint():
    rng = np.random.default_rng(0)
    u = rng.standard_normal((7, 7))
    g1, g2 = rng.standard_normal((7, 7)), rng.standard_normal((7, 7))
    a1, a2 = _grad(u)
    assert abs(np.vdot(a1, g1) + np.vdot(a2, g2) - np.vdot(u, _grad_t(g1, g2))) < 1e-12


@pytest.mark.parametrize("m,a,gamma", [(5, 1.0, 0.5), (8, 2.0, 1.5), (3, 0.7, 0.2)])
def test_fgp_step_closed_form(m, a, gamma):
    n = 12
    b = np.zeros((n, n))
    b[:, m:] = a
    u, _ = oracle.tv_fgp(b, gamma, 6000)
    expect = np.zeros((n, n))
    expect[:, :m] = gamma / m
    expect[:, m:] = a - gamma / (n - m)
    np.testing.assert_allclose(u, expect, rtol=0, atol=2e-6)


def test_fgp_constants_and_nonnegativity():
    n = 8
    u, p = oracle.tv_fgp(np.full((n, n), 0.7), 0.3, 50)
    np.testing.assert_allclose(u, 0.7, rtol=0, atol=1e-14)
    assert np.abs(p).max() < 1e-14
    u, _ = oracle.tv_fgp(np.full((n, n), -0.4), 0.3, 50)
    assert np.array_equal(u, np.zeros((n, n)))
    # nonnegativity with a mixed-sign input
    u, _ = oracle.tv_fgp(synth.random_image(n, 3), 0.05, 200)
    assert u.min() >= 0.0


def _rof_chambolle_pock(b, gamma, iters, quad=0.0):
    """min_u 1/2|u - b|^2 + gamma |grad u|_{1,2} + chi_{>=0}(u) + quad/2 |u|^2."""
    u = np.zeros_like(b)
    ub = u.copy()
    y1 = np.zeros_like(b)
    y2 = np.zeros_like(b)
    L = np.sqrt(8.0)
    s = t = 1.0 / L
    for _ in range(iters):
        g1, g2 = _grad(ub)
        y1, y2 = y1 + s * g1, y2 + s * g2
        nrm = np.maximum(1.0, np.sqrt(y1 ** 2 + y2 ** 2) / gamma)
        y1, y2 = y1 / nrm, y2 / nrm
        un = np.maximum(0.0, (u - t * _grad_t(y1, y2) + t * b) / (1.0 + t * (1.0 + quad)))
        ub = 2 * un - u
        u = un
    return u


def test_fgp_matches_chambolle_pock():
    n = 10
    b = synth.random_image(n, 4) * 0.5 + 0.3
    gamma = 0.15
    u, _ = oracle.tv_fgp(b, gamma, 8000)
    ref = _rof_chambolle_pock(b, gamma, 40000)
    np.testing.assert_allclose(u, ref, rtol=0, atol=1e-5)


@pytest.mark.parametrize("lam", [0.5, 1e-8])
def test_tv_prior_prox_with_lambda(lam):
    """The prior with strong convexity lam (R = w TV + chi_{>=0} + lam/2 |x|^2,
    mu = lam) inside Alg. 1: one step of one level from x^0 = v, y^0 = 0 and
    zero tables has xi = 0, so x^1 = prox_{tau R}(v) with tau = sigma / lam.
    Against Chambolle-Pock on that prox problem written out (no folding of
    the quadratic into the data term); at lam = 1e-8 the quadratic is
    negligible and x^1 is the prox of the paper's prior alone."""
    n = 10
    g = oracle.Geometry(n, 8, 14)
    lv = oracle.Levels([0], [1.0])
    tau, w = 0.2, 0.5
    v = synth.random_image(n, 6) * 0.5 + 0.2
    st = oracle.State.zeros(g, lv)
    st.x = v.copy()
    reg = oracle.Reg(oracle.REG_TV, lam=lam, tv_weight=w, tv_inner=8000)
    out = oracle.imask_run(g, lv, reg, tau * lam, 42, 0, np.zeros((8, 14)), 1, st)
    ref = _rof_chambolle_pock(v, tau * w, 40000, quad=tau * lam)
    np.testing.assert_allclose(out.x, ref, rtol=0, atol=1e-5)
    if lam < 1e-6:
        np.testing.assert_allclose(out.x, _rof_chambolle_pock(v, tau * w, 40000), rtol=0, atol=1e-5)


def _tv_minimiser(Kb, b, w, lam, n, iters):
    """min_x 1/2|Kb x - b|^2 + w |grad x|_{1,2} + lam/2 |x|^2 + chi_{>=0}(x)
    by Chambolle-Pock on A = [Kb; grad] with dense matrices."""
    bb = b.ravel()
    nrmK = np.linalg.norm(Kb, 2)
    L = np.sqrt(nrmK ** 2 + 8.0)
    s = t = 0.99 / L
    x = np.zeros(n * n)
    xb = x.copy()
    z = np.zeros_like(bb)
    y1 = np.zeros((n, n))
    y2 = np.zeros((n, n))
    for _ in range(iters):
        # prox of s F1*, F1(z) = 1/2|z - b|^2
        z = (z + s * (Kb @ xb) - s * bb) / (1.0 + s)
        g1, g2 = _grad(xb.reshape(n, n))
        y1, y2 = y1 + s * g1, y2 + s * g2
        nrm = np.maximum(1.0, np.sqrt(y1 ** 2 + y2 ** 2) / w)
        y1, y2 = y1 / nrm, y2 / nrm
        v = x - t * (Kb.T @ z + _grad_t(y1, y2).ravel())
        xn = np.maximum(0.0, v / (1.0 + t * lam))
        xb = 2 * xn - x
        x = xn
    return x


def test_imask_tv_converges_to_minimiser():
    n = 8
    g = oracle.Geometry(n, 12, 12)
    lv = oracle.Levels([0, 1, 2], [1 / 3] * 3, oracle.MODE_UNBIASED)
    Ks = [oracle.dense_matrix(lambda e, k=k: oracle.sketch_fwd(g, lv, k, e), (n, n), 144) for k in range(3)]
    Kb = sum(p * K for p, K in zip(lv.p, Ks))
    _, b = synth.ct_problem(n, 12, 12, 1e4, 1015, 2015)
    w, lam = 0.05, 0.1
    xs = _tv_minimiser(Kb, b, w, lam, n, 60000)
    reg = oracle.Reg(oracle.REG_TV, lam=lam, tv_weight=w, tv_inner=10)
    st = None
    errs = []
    for _ in range(12):
        st = oracle.imask_run(g, lv, reg, 0.02, 42, 0, b, 250, st)
        errs.append(np.linalg.norm(st.x.ravel() - xs) / np.linalg.norm(xs))
    assert st.x.min() >= 0.0
    assert errs[-1] < 1e-6 and errs[-1] < 1e-3 * errs[0]
