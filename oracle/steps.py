"""Step-size theory of ImaSk (Sec. 3.4-3.6 of the paper), FP64, test oracle.

Normalised constants for ImaSk with A_i = p_i K_i, mu_f* = 1, mu_g = mu:
  L^2     = |sum_i p_i K_i|^2 / mu                        (Lemma on B: L = |A~|)
  Lbar^2  = max(lmax(sum p_i^2 K_i^T K_i), lmax(sum p_i^2 K_i K_i^T)) / mu
  Lbarp^2 = max(lmax(sum p_i   K_i^T K_i), lmax(sum p_i   K_i K_i^T)) / mu
(the operator norms of Bbar and Bbar_p of Sec. 3.4 for the skew operator B).

With eta = sigma/(1+sigma) the rate is theta = max(phi, psi) (eq. (theta),
eq. (phi_psi)); under b = rho c / Lbar^2 (Sec. 3.5):
  phi(eta) = (eta - c)^2 / c + 1 - (1 - rho) c
  psi(eta) = alpha^{-1} eta^2 + 1 - min p,
  alpha^{-1} from eq. (alpha).
Thm. 3 (eq. (opt:cond), eq. (eta_opt)) gives the optimal eta for a (c, rho).
"""
from __future__ import annotations

import numpy as np


def constants_dense(Ks, p, mu: float):
    """(L^2, Lbar^2, Lbarp^2) from explicit matrices K_i (m x d)."""
    p = np.asarray(p, dtype=np.float64)
    Kbar = sum(pi * K for pi, K in zip(p, Ks))
    L2 = np.linalg.norm(Kbar, 2) ** 2 / mu

    def lmax(S):
        return float(np.linalg.eigvalsh(S)[-1])

    lb = max(lmax(sum(pi ** 2 * K.T @ K for pi, K in zip(p, Ks))),
             lmax(sum(pi ** 2 * K @ K.T for pi, K in zip(p, Ks)))) / mu
    lp = max(lmax(sum(pi * K.T @ K for pi, K in zip(p, Ks))),
             lmax(sum(pi * K @ K.T for pi, K in zip(p, Ks)))) / mu
    return L2, lb, lp


def power_lmax(apply, shape, iters: int = 200, seed: int = 0) -> float:
    """Largest eigenvalue of a symmetric PSD operator by the power method."""
    v = np.random.default_rng(seed).standard_normal(shape)
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = apply(v)
        lam = float(np.vdot(v, w))
        nrm = np.linalg.norm(w)
        if nrm == 0.0:
            return 0.0
        v = w / nrm
    return lam


def constants_power(fwd, adj, p, mu: float, x_shape, y_shape, iters: int = 200):
    """(L^2, Lbar^2, Lbarp^2) by the power method on operator callbacks
    fwd(k, x) = K_k x and adj(k, y) = K_k^T y."""
    p = np.asarray(p, dtype=np.float64)
    r = len(p)

    def kbar(x):
        return sum(p[k] * fwd(k, x) for k in range(r))

    def kbar_t(y):
        return sum(p[k] * adj(k, y) for k in range(r))

    L2 = power_lmax(lambda x: kbar_t(kbar(x)), x_shape, iters) / mu

    def gram_x(w):
        return lambda x: sum(w[k] * adj(k, fwd(k, x)) for k in range(r))

    def gram_y(w):
        return lambda y: sum(w[k] * fwd(k, adj(k, y)) for k in range(r))

    lb = max(power_lmax(gram_x(p ** 2), x_shape, iters), power_lmax(gram_y(p ** 2), y_shape, iters)) / mu
    lp = max(power_lmax(gram_x(p), x_shape, iters), power_lmax(gram_y(p), y_shape, iters)) / mu
    return L2, lb, lp


def cbar(L2: float, lp: float) -> float:
    return 1.0 / (1.0 + L2 + lp)


def alpha_inv(c: float, rho: float, L2: float, lb: float, lp: float) -> float:
    return (lb / (rho * c)) * (1.0 - (1.0 + L2) * c) / (1.0 - (1.0 + L2 + lp) * c)


def phi(eta, c, rho):
    return (eta - c) ** 2 / c + 1.0 - (1.0 - rho) * c


def psi(eta, c, rho, L2, lb, lp, pmin):
    return alpha_inv(c, rho, L2, lb, lp) * eta ** 2 + 1.0 - pmin


def theta(eta, c, rho, L2, lb, lp, pmin):
    return np.maximum(phi(eta, c, rho), psi(eta, c, rho, L2, lb, lp, pmin))


def eta_opt(c: float, rho: float, L2: float, lb: float, lp: float, pmin: float):
    """Optimal eta and theta for fixed (c, rho), Thm. 3."""
    ai = alpha_inv(c, rho, L2, lb, lp)
    if pmin > ai * c * c + (1.0 - rho) * c:  # eq. (opt:cond)
        return c, 1.0 - (1.0 - rho) * c
    q = ai - 1.0 / c
    if abs(q) < 1e-300:
        eta = (pmin + rho * c) / 2.0
    else:
        eta = (np.sqrt(1.0 + q * (pmin + rho * c)) - 1.0) / q  # eq. (eta_opt)
    return eta, float(phi(eta, c, rho))


def admissible(c: float, rho: float, L2: float, lb: float, lp: float, pmin: float):
    """Open eta interval on which theta < 1 (Prop. in Sec. 3.5)."""
    lo = c - c * np.sqrt(1.0 - rho)
    hi = min(c + c * np.sqrt(1.0 - rho), np.sqrt(pmin / alpha_inv(c, rho, L2, lb, lp)))
    return lo, hi


def sigma_thm3(L2: float, lb: float, lp: float, pmin: float, n_c: int = 400, n_rho: int = 400):
    """Minimise theta(eta*(c, rho)) over a (c, rho) grid; returns
    (sigma, theta, c, rho) with sigma = eta/(1-eta)."""
    cb = cbar(L2, lp)
    best = (np.inf, None, None, None)
    for c in cb * (np.arange(1, n_c + 1) / (n_c + 1)):
        for rho in np.arange(1, n_rho + 1) / (n_rho + 1):
            eta, th = eta_opt(c, rho, L2, lb, lp, pmin)
            if th < best[0]:
                best = (th, eta, c, rho)
    th, eta, c, rho = best
    return eta / (1.0 - eta), th, c, rho


def sigma_balamurugan(L2: float, lb: float) -> float:
    """sigma_B = 1/(L^2 + 3 Lbar^2), the rule of Balamurugan & Bach (Sec. 3.6)."""
    return 1.0 / (L2 + 3.0 * lb)
