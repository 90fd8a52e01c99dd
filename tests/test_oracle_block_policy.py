"""Pins of the oracle's block-residual policy (actions taken b per round: the residual at
the start of the round restricted to fixed observation groups).

* b = 1 is the CG policy (every action is the full current residual);
* the actions of a round are disjoint pieces of the residual at the start of the round,
  whose sum is that residual, computed here independently as r0 - Ghat S (S^T Ghat S)^{-1}
  S^T r0 with the earlier actions S (the Galerkin residual);
* with b = m singleton groups and i = m the actions span all observations, so the update
  is the exact Kalman update;
* the result depends only on the span of the actions: the batch update with the
  recorded actions gives the same posterior.
"""
import numpy as np

from oracle import kalman
from oracle.cakf import (Model, observation_groups, run_filter, update_batch,
                         update_iterative, block_residual_policy)
from tiny import dense_obs, tiny_problem


def test_block_size_one_is_cg():
    model, steps = tiny_problem(seed=60, T=4, m=9)
    a = run_filter(model, steps, 4, 6, policy="cg")
    b = run_filter(model, steps, 4, 6, policy=("block", 1))
    for ra, rb in zip(a, b):
        np.testing.assert_allclose(ra.m, rb.m, atol=1e-12)
        np.testing.assert_allclose(ra.M_plus @ ra.M_plus.T, rb.M_plus @ rb.M_plus.T, atol=1e-12)
        assert abs(ra.loglik - rb.loglik) < 1e-10


def test_round_actions_split_the_galerkin_residual():
    model, steps = tiny_problem(seed=61, T=1, m=12)
    idx, y = steps[0]
    n = model.n
    b, imax = 3, 7
    res = update_iterative(model, np.zeros(n), np.zeros((n, 0)), idx, y,
                           block_residual_policy(b, imax), imax)
    S = res.S
    G = model.cov(idx, idx) + model.noise_var * np.eye(len(idx))
    r0 = np.asarray(y, np.float64)
    j0 = 0
    while j0 < S.shape[1]:
        bt = min(b, imax - j0)
        Sp = S[:, :j0]
        if j0:
            r = r0 - G @ Sp @ np.linalg.solve(Sp.T @ G @ Sp, Sp.T @ r0)
        else:
            r = r0
        block = S[:, j0:j0 + bt]
        for g, (g0, g1) in enumerate(observation_groups(len(idx), bt)):
            np.testing.assert_allclose(block[g0:g1, g], r[g0:g1], atol=1e-10)
            outside = np.ones(len(idx), bool)
            outside[g0:g1] = False
            assert np.all(block[outside, g] == 0.0)
        np.testing.assert_allclose(block.sum(axis=1), r, atol=1e-10)
        j0 += bt


def test_singleton_groups_give_the_exact_kalman_update():
    model, steps = tiny_problem(seed=62, T=3, m=6)
    recs = run_filter(model, steps, 6, 1000, policy=("block", 6))
    kf = kalman.kalman_filter(model.cov(), model.a, dense_obs(model, steps))
    for rec, ref in zip(recs, kf):
        np.testing.assert_allclose(rec.m, ref["m"], atol=1e-9)
        np.testing.assert_allclose(model.cov() - rec.M @ rec.M.T, ref["P"], atol=1e-9)


def test_block_actions_batch_form_agrees():
    model, steps = tiny_problem(seed=63, T=1, m=11)
    idx, y = steps[0]
    n = model.n
    res = update_iterative(model, np.zeros(n), np.zeros((n, 0)), idx, y,
                           block_residual_policy(4, 8), 8)
    bat = update_batch(model, np.zeros(n), np.zeros((n, 0)), idx, y, res.S, lsqrt="chol")
    np.testing.assert_allclose(res.m, bat.m, atol=1e-10)
    np.testing.assert_allclose(res.M @ res.M.T, bat.M @ bat.M.T, atol=1e-10)
    assert abs(res.loglik - bat.loglik) < 1e-9
