"""Textbook Kalman filter, RTS smoother and joint Gaussian conditioning (oracle, FP64).

These dense references pin the computation-aware recursions on tiny problems:

* kalman_filter  - predict/update moments of Sec. 2.1 (Thm. A.1), plus the
                   prediction-error log-likelihood log N(y_k; H m_k^-, G_k).
* rts_smoother   - the RTS recursion of Sec. 2.1 (Thm. A.3).
* joint_posterior - brute-force conditioning of the joint Gaussian of all states and
                   all (projected) observations; independent of any recursion.

The LGSSM is the one the paper's separable spatiotemporal prior induces with an
Ornstein-Uhlenbeck temporal factor (Lemma C.1 with A^t = a, Q^t = 1 - a^2):
u_0 ~ N(0, Sigma), u_k = a u_{k-1} + q_k, q_k ~ N(0, (1 - a^2) Sigma),
y_k = H_k u_k + eps_k, eps_k ~ N(0, R_k).

Test infrastructure only; not part of the product path.
"""
from __future__ import annotations

import numpy as np


def _logpdf_zero_mean(r: np.ndarray, G: np.ndarray) -> float:
    L = np.linalg.cholesky(G)
    z = np.linalg.solve(L, r)
    return float(-0.5 * (r.size * np.log(2.0 * np.pi) + 2.0 * np.sum(np.log(np.diag(L)))
                         + z @ z))


def kalman_filter(Sigma: np.ndarray, a: float, obs):
    """obs[k-1] = (H_k, R_k, y_k) or None for k = 1..T.

    Returns a list of dicts with m_pred, P_pred, m, P, loglik for k = 1..T; the
    initial state (k = 0) has mean 0 and covariance Sigma."""
    n = Sigma.shape[0]
    m = np.zeros(n)
    P = Sigma.copy()
    out = []
    for item in obs:
        m_pred = a * m
        P_pred = a * a * P + (1.0 - a * a) * Sigma
        if item is None:
            m, P, ll = m_pred, P_pred, 0.0
        else:
            H, R, y = item
            r = y - H @ m_pred
            G = H @ P_pred @ H.T + R
            Kg = np.linalg.solve(G, H @ P_pred).T          # P_pred H^T G^{-1}
            m = m_pred + Kg @ r
            P = P_pred - Kg @ G @ Kg.T
            ll = _logpdf_zero_mean(r, G)
        out.append(dict(m_pred=m_pred, P_pred=P_pred, m=m, P=P, loglik=ll))
    return out


def rts_smoother(a: float, filt):
    """RTS recursion over the output of kalman_filter (k = T..1)."""
    T = len(filt)
    ms = [None] * T
    Ps = [None] * T
    ms[T - 1] = filt[T - 1]["m"]
    Ps[T - 1] = filt[T - 1]["P"]
    for k in range(T - 2, -1, -1):
        P = filt[k]["P"]
        Pp = filt[k + 1]["P_pred"]
        Gk = np.linalg.solve(Pp, a * P).T                   # P A^T (P_pred)^{-1}
        ms[k] = filt[k]["m"] + Gk @ (ms[k + 1] - filt[k + 1]["m_pred"])
        Ps[k] = P + Gk @ (Ps[k + 1] - Pp) @ Gk.T
    return ms, Ps


def state_covariance(Sigma: np.ndarray, a: float, T: int) -> np.ndarray:
    """Joint prior covariance of (u_1, ..., u_T): Cov(u_j, u_k) = a^|j-k| Sigma."""
    n = Sigma.shape[0]
    C = np.empty((T * n, T * n))
    for j in range(T):
        for k in range(T):
            C[j * n:(j + 1) * n, k * n:(k + 1) * n] = a ** abs(j - k) * Sigma
    return C


def joint_posterior(Sigma: np.ndarray, a: float, obs, upto=None):
    """Condition the joint Gaussian of (u_1..u_T) on the observations of steps 1..upto.

    Returns (mean, cov) of the stacked states and the log marginal likelihood of the
    used observations.  Brute force: builds the full joint and solves densely."""
    n = Sigma.shape[0]
    T = len(obs)
    upto = T if upto is None else upto
    C = state_covariance(Sigma, a, T)
    rows, ys, Rs = [], [], []
    for k, item in enumerate(obs[:upto]):
        if item is None:
            continue
        H, R, y = item
        Hk = np.zeros((H.shape[0], T * n))
        Hk[:, k * n:(k + 1) * n] = H
        rows.append(Hk)
        ys.append(y)
        Rs.append(R)
    if not rows:
        return np.zeros(T * n), C, 0.0
    Hall = np.vstack(rows)
    y = np.concatenate(ys)
    R = np.zeros((y.size, y.size))
    o = 0
    for Rk in Rs:
        R[o:o + Rk.shape[0], o:o + Rk.shape[0]] = Rk
        o += Rk.shape[0]
    G = Hall @ C @ Hall.T + R
    CHt = C @ Hall.T
    mean = CHt @ np.linalg.solve(G, y)
    cov = C - CHt @ np.linalg.solve(G, CHt.T)
    return mean, cov, _logpdf_zero_mean(y, G)


def row_selector(idx, n: int) -> np.ndarray:
    """Observation matrix H that picks the entries idx of an n-vector."""
    H = np.zeros((len(idx), n))
    H[np.arange(len(idx)), np.asarray(idx)] = 1.0
    return H
