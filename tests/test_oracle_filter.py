"""Pins of the oracle's computation-aware filter against the exact references.

* full actions and no truncation reduce the CAKF to the Kalman filter (Prop. A.2);
* partial given actions are exact inference with the projected observations S^T y
  (Sec. 3.1, projected observation model), checked against brute-force conditioning
  of the joint Gaussian of all states;
* the iterative and batch updates agree (Prop. B.1);
* CG actions are Krylov/Lanczos vectors (App. E);
* truncation is the Eckart-Young-Mirsky optimum and is conservative (Sec. 3.2).
"""
import math

import numpy as np
import pytest

from oracle import kalman
from oracle.cakf import (Model, run_filter, truncate, update_batch, update_iterative,
                         given_policy, cg_policy, total_loglik)
from tiny import dense_obs, tiny_problem


def _cov(model, rec):
    return model.cov() - rec.M @ rec.M.T


def _dense_kf(model, steps, actions=None):
    return kalman.kalman_filter(model.cov(), model.a, dense_obs(model, steps, actions))


@pytest.mark.parametrize("form", ["iterative", "batch"])
def test_full_actions_reduce_to_kalman_filter(form):
    model, steps = tiny_problem(seed=4, missing_steps=(3,))
    rng = np.random.default_rng(5)
    actions = [None if s is None else rng.standard_normal((8, 8)) for s in steps]
    recs = run_filter(model, steps, max_actions=8, r_cap=1000, policy="given",
                      actions=actions, form=form)
    kf = _dense_kf(model, steps)
    for rec, ref in zip(recs, kf):
        np.testing.assert_allclose(rec.m, ref["m"], atol=1e-9)
        np.testing.assert_allclose(_cov(model, rec), ref["P"], atol=1e-9)
        np.testing.assert_allclose(rec.loglik, ref["loglik"], atol=1e-9)


def test_identity_actions_reduce_to_kalman_filter():
    model, steps = tiny_problem(seed=6, nu2=5, a=0.6)
    actions = [np.eye(8) for _ in steps]
    recs = run_filter(model, steps, 8, 1000, policy="given", actions=actions)
    for rec, ref in zip(recs, _dense_kf(model, steps)):
        np.testing.assert_allclose(rec.m, ref["m"], atol=1e-9)
        np.testing.assert_allclose(_cov(model, rec), ref["P"], atol=1e-9)


def test_partial_actions_are_exact_inference_on_projected_data():
    model, steps = tiny_problem(seed=7, T=4, m=10)
    rng = np.random.default_rng(8)
    actions = [rng.standard_normal((10, 3)) for _ in steps]
    recs = run_filter(model, steps, 3, 1000, policy="given", actions=actions)
    proj = dense_obs(model, steps, actions)
    n = model.n
    for k, rec in enumerate(recs, start=1):
        mean, cov, _ = kalman.joint_posterior(model.cov(), model.a, proj, upto=k)
        sl = slice((k - 1) * n, k * n)
        np.testing.assert_allclose(rec.m, mean[sl], atol=1e-9)
        np.testing.assert_allclose(_cov(model, rec), cov[sl, sl], atol=1e-9)


def test_projected_loglik_equals_joint_density_of_projected_data():
    model, steps = tiny_problem(seed=9, T=3, m=9)
    rng = np.random.default_rng(10)
    actions = [rng.standard_normal((9, 4)) for _ in steps]
    recs = run_filter(model, steps, 4, 1000, policy="given", actions=actions)
    _, _, joint = kalman.joint_posterior(model.cov(), model.a, dense_obs(model, steps, actions))
    half_logdet = sum(0.5 * np.linalg.slogdet(S.T @ S)[1] for S in actions)
    assert total_loglik(recs) == pytest.approx(joint + half_logdet, abs=1e-9)


def test_full_action_loglik_equals_spatiotemporal_gp_evidence():
    model, steps = tiny_problem(seed=11, T=3, m=7, missing_steps=(2,))
    recs = run_filter(model, steps, 7, 1000, policy="given",
                      actions=[None if s is None else np.eye(7) for s in steps])
    _, _, joint = kalman.joint_posterior(model.cov(), model.a, dense_obs(model, steps))
    assert total_loglik(recs) == pytest.approx(joint, abs=1e-9)


def test_loglik_depends_only_on_the_span_of_the_actions():
    model, steps = tiny_problem(seed=12, T=2, m=9)
    rng = np.random.default_rng(13)
    A = [rng.standard_normal((9, 4)) for _ in steps]
    R = [rng.standard_normal((4, 4)) + 3 * np.eye(4) for _ in steps]
    r1 = run_filter(model, steps, 4, 1000, policy="given", actions=A)
    r2 = run_filter(model, steps, 4, 1000, policy="given", actions=[a @ r for a, r in zip(A, R)])
    assert total_loglik(r1) == pytest.approx(total_loglik(r2), abs=1e-9)
    for a, b in zip(r1, r2):
        np.testing.assert_allclose(a.m, b.m, atol=1e-10)
        np.testing.assert_allclose(a.M @ a.M.T, b.M @ b.M.T, atol=1e-10)


def test_iterative_and_batch_updates_agree():
    model, steps = tiny_problem(seed=14, T=1, m=12)
    rng = np.random.default_rng(15)
    n = model.n
    # a valid predictive factor: Sigma - M M^T = L (I - Z Z^T) L^T is PSD for ||Z|| < 1
    L = np.linalg.cholesky(model.cov() + 1e-10 * np.eye(n))
    Z, _ = np.linalg.qr(rng.standard_normal((n, 5)))
    M_pred = L @ (0.6 * Z)
    m_pred = rng.standard_normal(n)
    idx, y = steps[0]
    S = rng.standard_normal((12, 6))
    it = update_iterative(model, m_pred, M_pred, idx, y, given_policy(S), 6)
    for lsq in ("eigh", "chol"):
        bt = update_batch(model, m_pred, M_pred, idx, y, S, lsqrt=lsq)
        np.testing.assert_allclose(it.m, bt.m, atol=1e-10)
        np.testing.assert_allclose(it.M @ it.M.T, bt.M @ bt.M.T, atol=1e-10)
        assert it.loglik == pytest.approx(bt.loglik, abs=1e-10)
    # The iterative search directions are S L^{-T} (Cholesky left square root).
    bt = update_batch(model, m_pred, M_pred, idx, y, S, lsqrt="chol")
    np.testing.assert_allclose(it.W_obs, bt.W_obs, atol=1e-9)


def test_cg_actions_are_lanczos_vectors():
    model, steps = tiny_problem(seed=16, T=1, m=14, noise_var=0.1)
    idx, y = steps[0]
    n = model.n
    m_pred = np.zeros(n)
    M_pred = np.zeros((n, 0))
    res = update_iterative(model, m_pred, M_pred, idx, y, cg_policy(), 5)
    S = res.S / np.linalg.norm(res.S, axis=0)
    np.testing.assert_allclose(S.T @ S, np.eye(5), atol=1e-9)     # residuals orthogonal
    Ghat = model.cov(idx, idx) + model.noise_var * np.eye(14)
    T3 = S.T @ Ghat @ S
    off = T3 - np.triu(np.tril(T3, 1), -1)
    assert np.abs(off).max() < 1e-9 * np.abs(T3).max()             # tridiagonal
    # span(S) is the Krylov space K_5(Ghat, r0)
    r0 = y - m_pred[idx]
    Kr = np.column_stack([np.linalg.matrix_power(Ghat, j) @ r0 for j in range(5)])
    Q, _ = np.linalg.qr(Kr)
    np.testing.assert_allclose(S @ S.T, Q @ Q.T, atol=1e-7)


def test_cg_with_full_budget_reaches_the_kalman_filter():
    model, steps = tiny_problem(seed=17, T=3, m=6)
    recs = run_filter(model, steps, 6, 1000, policy="cg", resid_tol=1e-13)
    for rec, ref in zip(recs, _dense_kf(model, steps)):
        np.testing.assert_allclose(rec.m, ref["m"], atol=1e-7)
        np.testing.assert_allclose(_cov(model, rec), ref["P"], atol=1e-7)


def test_truncation_is_eckart_young_optimal_and_conservative():
    rng = np.random.default_rng(18)
    M = rng.standard_normal((40, 9)) @ np.diag(np.linspace(3, 0.1, 9))
    Mp, Vr, lam = truncate(M, 5)
    sv = np.linalg.svd(M, compute_uv=False)
    D = M @ M.T - Mp @ Mp.T
    assert np.linalg.norm(D, 2) == pytest.approx(sv[5] ** 2, rel=1e-10)
    assert np.linalg.eigvalsh(D).min() > -1e-10                   # M+ M+^T <= M M^T
    # invariant under a right rotation of M
    Q, _ = np.linalg.qr(rng.standard_normal((9, 9)))
    Mp2, _, _ = truncate(M @ Q, 5)
    np.testing.assert_allclose(Mp @ Mp.T, Mp2 @ Mp2.T, atol=1e-10)
    # nothing to drop: factor returned unchanged
    Mq, V, _ = truncate(M, 9)
    assert V is None and np.array_equal(Mq, M)


def test_truncated_columns_are_orthogonal_through_predict_and_update():
    """After a truncation the factor's columns M V_r are mutually orthogonal with the kept
    eigenvalues as squared norms; the OU prediction scales them by a and the update appends
    columns, so the Gram of the next untruncated factor begins with the block a^2 diag(lam)
    (the block a truncation may take as known instead of recomputing it)."""
    model, steps = tiny_problem(seed=23, T=4, m=8)
    recs = run_filter(model, steps, 3, 4, policy="cg")
    checked = 0
    for prev, cur in zip(recs, recs[1:]):
        r = prev.M_plus.shape[1]
        if prev.M.shape[1] <= r:
            continue                                   # no truncation at this step
        lam = np.sort(np.linalg.eigvalsh(prev.M.T @ prev.M))[::-1][:r]
        G = prev.M_plus.T @ prev.M_plus
        np.testing.assert_allclose(G, np.diag(lam), rtol=1e-10, atol=1e-12 * lam[0])
        np.testing.assert_allclose(cur.M_pred, model.a * prev.M_plus, rtol=1e-14, atol=0)
        Gn = cur.M.T @ cur.M
        np.testing.assert_allclose(Gn[:r, :r], model.a ** 2 * np.diag(lam), rtol=1e-10,
                                   atol=1e-12 * lam[0])
        checked += 1
    assert checked >= 2


def test_truncated_filter_covariance_is_psd_and_above_kalman():
    model, steps = tiny_problem(seed=19, T=5, m=8)
    recs = run_filter(model, steps, 3, 4, policy="cg")
    kf = _dense_kf(model, steps)
    for rec, ref in zip(recs, kf):
        P = _cov(model, rec)
        assert np.linalg.eigvalsh(P).min() > -1e-10
        assert np.linalg.eigvalsh(P - ref["P"]).min() > -1e-10
        Pt = model.cov() - rec.M_plus @ rec.M_plus.T
        assert np.linalg.eigvalsh(Pt - P).min() > -1e-10            # truncation adds variance


def test_missing_step_only_predicts_and_prior_is_stationary():
    model, steps = tiny_problem(seed=20, T=3, missing_steps=(1, 2, 3))
    recs = run_filter(model, steps, 4, 10)
    for rec in recs:
        assert rec.M.shape[1] == 0 and rec.loglik == 0.0
        np.testing.assert_allclose(rec.marginal_var(model.sigma_f2), model.sigma_f2)
        np.testing.assert_allclose(rec.m, 0.0)
    Sigma = model.cov()
    a = model.a
    np.testing.assert_allclose(a * a * Sigma + (1 - a * a) * Sigma, Sigma, atol=1e-14)


def test_breakdown_stops_on_dependent_actions():
    model, steps = tiny_problem(seed=21, T=1, m=8)
    rng = np.random.default_rng(22)
    S = rng.standard_normal((8, 3))
    S = np.column_stack([S, S[:, 0] + 2 * S[:, 1], rng.standard_normal(8)])
    idx, y = steps[0]
    res = update_iterative(model, np.zeros(model.n), np.zeros((model.n, 0)), idx, y,
                           given_policy(S), 5)
    assert res.i_eff == 3
