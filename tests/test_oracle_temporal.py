"""Pins of the Matérn-3/2 temporal state-space model (oracle.temporal) and of the filter
on it, against the spatiotemporal Gaussian process it represents, written from the
kernel's closed form k_t(tau) = (1 + lam |tau|) exp(-lam |tau|) (no state space):

* the transition reproduces the kernel and its time derivative:
  [(A^t)^k]_00 = k_t(k dt), [(A^t)^k]_10 = k_t'(k dt) / lam;
* the stationary covariance is preserved: A^t A^t^T + Q^t = I with Q^t PSD;
* full actions, no truncation: the filter's value means and covariances are the GP
  posterior of f(t_k, X) given the data up to step k (brute-force conditioning);
* partial given actions: the same with the data projected by S_k;
* CG actions with truncation: the value variances never fall below the exact ones
  (conservative, Sec. 3.2).
"""
import math

import numpy as np
import pytest

from oracle import matern
from oracle.cakf import run_filter
from oracle.temporal import Matern32TimeModel


def k_t(tau, lam):
    lt = lam * np.abs(tau)
    return (1.0 + lt) * np.exp(-lt)


def dk_t(tau, lam):
    """d/dtau k_t(tau) for tau >= 0."""
    return -lam * lam * tau * np.exp(-lam * tau)


def _problem(seed, n=10, T=4, m=6, a=0.7, missing=()):
    rng = np.random.default_rng(seed)
    X = rng.random((n, 2))
    model = Matern32TimeModel(X, 3, 0.4, 1.3, a, 0.05)
    steps = []
    for k in range(1, T + 1):
        if k in missing:
            steps.append(None)
            continue
        idx = rng.choice(n, m, replace=False)
        steps.append((idx, rng.standard_normal(m)))
    return model, steps


def _gp_posterior(model, steps, upto, actions=None):
    """Posterior of the values f(t_k, X) (k = upto) given the (projected) data of steps
    1..upto under k_t(t - t') Sigma(x, x'), steps at t_k = k (dt = 1)."""
    lam = model.s                      # lam dt with dt = 1
    p = model.points
    Ks = matern.gram(model.X, model.X, model.nu2, model.ell, model.sigma_f2)
    T = len(steps)
    times = np.arange(1, T + 1, dtype=np.float64)
    C = np.kron(k_t(np.subtract.outer(times, times), lam), Ks)
    rows, ys, Rs = [], [], []
    for k in range(upto):
        if steps[k] is None:
            continue
        idx, y = steps[k]
        S = np.eye(len(idx)) if actions is None else actions[k]
        H = np.zeros((S.shape[1], T * p))
        H[:, k * p + np.asarray(idx)] = S.T
        rows.append(H)
        ys.append(S.T @ y)
        Rs.append(model.noise_var * S.T @ S)
    sl = slice((upto - 1) * p, upto * p)
    if not rows:
        return np.zeros(p), C[sl, sl]
    Hall = np.vstack(rows)
    yall = np.concatenate(ys)
    R = np.zeros((yall.size, yall.size))
    o = 0
    for Rk in Rs:
        R[o:o + Rk.shape[0], o:o + Rk.shape[0]] = Rk
        o += Rk.shape[0]
    G = Hall @ C @ Hall.T + R
    CH = C[sl] @ Hall.T
    return CH @ np.linalg.solve(G, yall), C[sl, sl] - CH @ np.linalg.solve(G, CH.T)


def test_transition_reproduces_the_kernel():
    model, _ = _problem(0, a=0.6)
    At = model.At()
    lam = model.s
    P = np.eye(2)
    for k in range(1, 7):
        P = At @ P
        assert abs(P[0, 0] - k_t(k, lam)) < 1e-12
        assert abs(P[1, 0] - dk_t(k, lam) / lam) < 1e-12
    Q = np.eye(2) - At @ At.T
    assert np.linalg.eigvalsh(Q).min() > 0


@pytest.mark.parametrize("partial", [False, True])
def test_filter_is_the_gp_posterior(partial):
    model, steps = _problem(1, missing=(3,))
    rng = np.random.default_rng(2)
    actions = None
    if partial:
        actions = [None if s is None else rng.standard_normal((6, 3)) for s in steps]
        recs = run_filter(model, steps, 3, 1000, policy="given", actions=actions)
    else:
        recs = run_filter(model, steps, 6, 1000, policy="given",
                          actions=[None if s is None else np.eye(6) for s in steps])
    p = model.points
    for k in range(1, len(steps) + 1):
        mean, cov = _gp_posterior(model, steps, k, actions)
        rec = recs[k - 1]
        np.testing.assert_allclose(rec.m[:p], mean, atol=1e-9)
        P = model.cov() - rec.M @ rec.M.T
        np.testing.assert_allclose(P[:p, :p], cov, atol=1e-9)


def test_truncated_cg_filter_is_conservative():
    model, steps = _problem(3, n=14, T=5, m=8)
    recs = run_filter(model, steps, 3, 5, policy="cg")
    p = model.points
    for k in range(1, len(steps) + 1):
        _, cov = _gp_posterior(model, steps, k)
        var = model.sigma_f2 - np.sum(recs[k - 1].M_plus[:p] ** 2, axis=1)
        assert np.min(var - np.diag(cov)) > -1e-10
