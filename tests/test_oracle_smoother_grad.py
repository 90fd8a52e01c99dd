"""Pins of the oracle's smoother (Alg. 3) and likelihood derivative.

* full actions, no truncation: the computation-aware smoother is the RTS smoother
  (Prop. A.4 and Thm. A.3);
* partial given actions, no truncation: it is exact inference on the projected data of
  all steps (iteratively approximated batch GP with block-diagonal actions, Prop. C.5);
* the finite-difference derivative of the replayed projected log-likelihood equals the
  textbook GP evidence gradient 1/2 tr((alpha alpha^T - C^{-1}) dC) of the projected
  spatiotemporal Gram matrix.
"""
import math

import numpy as np
import pytest

from oracle import kalman, matern
from oracle.cakf import Model, run_filter
from oracle.caks import run_smoother
from oracle.grad import fd_gradient, model_at, replay_loglik
from tiny import dense_obs, tiny_problem


def test_full_action_smoother_is_rts():
    model, steps = tiny_problem(seed=30, T=4, m=8, missing_steps=(2,))
    recs = run_filter(model, steps, 8, 1000, policy="given",
                      actions=[None if s is None else np.eye(8) for s in steps])
    sm = run_smoother(model, recs, 1000)
    kf = kalman.kalman_filter(model.cov(), model.a, dense_obs(model, steps))
    ms, Ps = kalman.rts_smoother(model.a, kf)
    for k in range(len(steps)):
        np.testing.assert_allclose(sm[k].m, ms[k], atol=1e-9)
        np.testing.assert_allclose(model.cov() - sm[k].M @ sm[k].M.T, Ps[k], atol=1e-9)


def test_partial_action_smoother_is_projected_batch_posterior():
    model, steps = tiny_problem(seed=31, T=4, m=9)
    rng = np.random.default_rng(32)
    actions = [rng.standard_normal((9, 3)) for _ in steps]
    recs = run_filter(model, steps, 3, 1000, policy="given", actions=actions)
    sm = run_smoother(model, recs, 1000)
    mean, cov, _ = kalman.joint_posterior(model.cov(), model.a,
                                          dense_obs(model, steps, actions))
    n = model.n
    for k in range(len(steps)):
        sl = slice(k * n, (k + 1) * n)
        np.testing.assert_allclose(sm[k].m, mean[sl], atol=1e-9)
        np.testing.assert_allclose(model.cov() - sm[k].M @ sm[k].M.T, cov[sl, sl], atol=1e-9)


def test_truncated_smoother_covariance_stays_psd():
    model, steps = tiny_problem(seed=33, T=5, m=8)
    recs = run_filter(model, steps, 3, 4, policy="cg")
    sm = run_smoother(model, recs, 4)
    for s in sm:
        assert np.linalg.eigvalsh(model.cov() - s.M @ s.M.T).min() > -1e-10


def _projected_evidence_grad(X, nu2, theta, dt, steps, actions):
    """Analytic d/dtheta of log N(S^T y; 0, S^T Ktilde S) + 1/2 log det S^T S."""
    ell, ell_t, s2, nv = theta
    a = math.exp(-dt / ell_t)
    n = X.shape[0]
    T = len(steps)
    Kx = matern.gram(X, X, nu2, ell, 1.0)
    dKx = matern.gram_dell(X, X, nu2, ell, 1.0)
    lag = np.abs(np.subtract.outer(np.arange(T), np.arange(T)))
    At = a ** lag
    dAt = lag * a ** lag * dt / ell_t ** 2
    blocks, ys = [], []
    for k, (idx, y) in enumerate(steps):
        H = np.zeros((len(idx), T * n))
        H[np.arange(len(idx)), k * n + np.asarray(idx)] = 1.0
        blocks.append(actions[k].T @ H)
        ys.append(actions[k].T @ y)
    SH = np.vstack(blocks)
    ys = np.concatenate(ys)
    SS = np.zeros((SH.shape[0], SH.shape[0]))
    o = 0
    for S in actions:
        i = S.shape[1]
        SS[o:o + i, o:o + i] = S.T @ S
        o += i
    Kst = np.kron(At, s2 * Kx)
    C = SH @ Kst @ SH.T + nv * SS
    dC = [SH @ np.kron(At, s2 * dKx) @ SH.T,
          SH @ np.kron(dAt, s2 * Kx) @ SH.T,
          SH @ np.kron(At, Kx) @ SH.T,
          SS]
    alpha = np.linalg.solve(C, ys)
    Ci = np.linalg.inv(C)
    return np.array([0.5 * np.trace((np.outer(alpha, alpha) - Ci) @ D) for D in dC])


def test_fd_gradient_matches_projected_gp_evidence_gradient():
    model, steps = tiny_problem(seed=34, T=3, m=7, nu2=3)
    rng = np.random.default_rng(35)
    actions = [rng.standard_normal((7, 3)) for _ in steps]
    dt = 1.0
    theta = (0.3, 5.0, 1.3, 0.05)
    base = model_at(model, dt, theta)
    recs = run_filter(base, steps, 3, 1000, policy="given", actions=actions)
    g = fd_gradient(base, dt, theta, steps, recs, 1000)
    ref = _projected_evidence_grad(base.X, base.nu2, theta, dt, steps, actions)
    np.testing.assert_allclose(g, ref, rtol=1e-6, atol=1e-8)


def test_replay_reproduces_base_run_with_truncation():
    model, steps = tiny_problem(seed=36, T=4, m=8)
    dt, theta = 1.0, (0.3, 5.0, 1.3, 0.05)
    base = model_at(model, dt, theta)
    recs = run_filter(base, steps, 3, 4, policy="cg")
    ll = sum(r.loglik for r in recs)
    assert replay_loglik(base, dt, theta, steps, recs, 4) == pytest.approx(ll, abs=1e-10)


def test_batch_replay_with_frozen_rotations_equals_the_iterative_replay():
    """With truncation in the replay, the frozen rotation acts on the factor's columns, so
    the replayed function depends on the square root of the projected Gram matrix: the
    batch form with the Cholesky root gives the columns S L^{-T} of the iterative form
    (App. B) and hence the same function and derivative; an eigen-decomposition root
    (another basis of the same span) would not."""
    model, steps = tiny_problem(seed=37, T=4, m=9)
    rng = np.random.default_rng(38)
    actions = [rng.standard_normal((9, 3)) for _ in steps]
    dt, theta = 1.0, (0.3, 5.0, 1.3, 0.05)
    base = model_at(model, dt, theta)
    recs = run_filter(base, steps, 3, 4, policy="given", actions=actions)
    assert sum(r.V_r is not None for r in recs) >= 2
    for th in (theta, (0.31, 4.9, 1.25, 0.06)):
        assert replay_loglik(base, dt, th, steps, recs, 4, form="batch") == pytest.approx(
            replay_loglik(base, dt, th, steps, recs, 4), abs=1e-10)
    g_it = fd_gradient(base, dt, theta, steps, recs, 4)
    g_b = fd_gradient(base, dt, theta, steps, recs, 4, form="batch")
    np.testing.assert_allclose(g_b, g_it, rtol=1e-7, atol=1e-9)
