"""Pins of the oracle's path sampler (App. C, CAKF/CAKS sampler).

The sampler is affine in its draws, so its exact output distribution follows from
one call with the draws set to the columns of an identity matrix (one path per unit
draw) plus one call with zero draws.  Without truncation that distribution must be the
posterior of the projected model, computed here by brute-force conditioning of the
joint Gaussian of all states on S_k^T y_k (independent of any recursion):

* zero draws give the filter means forward and the smoother means backward;
* the smoothed paths have the joint posterior's mean and covariance, across time too;
* the forward samples of step k have the filter's marginal (data up to step k);
* with full actions (S = I) the paths follow the exact RTS posterior.
"""
import numpy as np

from oracle import kalman
from oracle.cakf import run_filter
from oracle.sampler import sample_paths
from tiny import dense_obs, tiny_problem


def _unit_draws(model, steps):
    """Draw arrays whose columns are the unit draws of every random input, scaled to
    the draw distributions: x0 = L xi, q_k = sqrt(1 - a^2) L xi_k, e_k = xi'_k."""
    n, T = model.n, len(steps)
    ms = [0 if s is None else len(s[0]) for s in steps]
    D = n * (T + 1) + sum(ms)
    L = np.linalg.cholesky(model.cov() + 1e-12 * np.eye(n))
    x0 = np.zeros((n, D))
    x0[:, :n] = L
    q, e = [], []
    col = n
    for k in range(T):
        qk = np.zeros((n, D))
        qk[:, col:col + n] = np.sqrt(1.0 - model.a ** 2) * L
        q.append(qk)
        col += n
    for k in range(T):
        if ms[k] == 0:
            e.append(None)
            continue
        ek = np.zeros((ms[k], D))
        ek[:, col:col + ms[k]] = np.eye(ms[k])
        e.append(ek)
        col += ms[k]
    return x0, q, e


def _zero_draws(model, steps, ns=1):
    n = model.n
    return (np.zeros((n, ns)), [np.zeros((n, ns)) for _ in steps],
            [None if s is None else np.zeros((len(s[0]), ns)) for s in steps])


def _moments(model, steps, recs):
    """Exact mean and covariance of the sampler's outputs (forward and smoothed)."""
    mean_f, _, mean_s = sample_paths(model, steps, recs, *_zero_draws(model, steps))
    J_f, _, J_s = sample_paths(model, steps, recs, *_unit_draws(model, steps))
    lin_f = [J - m for J, m in zip(J_f, mean_f)]
    lin_s = [J - m for J, m in zip(J_s, mean_s)]
    return mean_f, mean_s, lin_f, lin_s


def test_zero_draws_give_the_filter_and_smoother_means():
    from oracle.caks import run_smoother
    model, steps = tiny_problem(seed=40, n=14, T=4, m=6, missing_steps=(3,))
    recs = run_filter(model, steps, 4, 1000, policy="cg")
    x, _, xs = sample_paths(model, steps, recs, *_zero_draws(model, steps, ns=2))
    sm = run_smoother(model, recs, 1000)
    for k in range(len(steps)):
        np.testing.assert_allclose(x[k][:, 0], recs[k].m, atol=1e-10)
        np.testing.assert_allclose(xs[k][:, 1], sm[k].m, atol=1e-10)


def test_smoothed_paths_have_the_projected_joint_posterior():
    model, steps = tiny_problem(seed=41, n=12, T=4, m=7, missing_steps=(2,))
    rng = np.random.default_rng(42)
    actions = [None if s is None else rng.standard_normal((7, 3)) for s in steps]
    recs = run_filter(model, steps, 3, 1000, policy="given", actions=actions)
    mean, cov, _ = kalman.joint_posterior(model.cov(), model.a,
                                          dense_obs(model, steps, actions))
    _, mean_s, _, lin_s = _moments(model, steps, recs)
    n, T = model.n, len(steps)
    for j in range(T):
        sj = slice(j * n, (j + 1) * n)
        np.testing.assert_allclose(mean_s[j][:, 0], mean[sj], atol=1e-9)
        for k in range(T):
            sk = slice(k * n, (k + 1) * n)
            np.testing.assert_allclose(lin_s[j] @ lin_s[k].T, cov[sj, sk], atol=1e-9)


def test_forward_samples_have_the_filter_marginals():
    model, steps = tiny_problem(seed=43, n=12, T=3, m=6)
    recs = run_filter(model, steps, 3, 1000, policy="cg")
    _, _, lin_f, _ = _moments(model, steps, recs)
    for k in range(len(steps)):
        P = model.cov() - recs[k].M @ recs[k].M.T
        np.testing.assert_allclose(lin_f[k] @ lin_f[k].T, P, atol=1e-9)
    # the filter's covariance is the joint posterior given the data up to step k
    # (projected by the recorded CG actions)
    acts = [r.S[:, :r.i_eff] for r in recs]
    n = model.n
    for k in range(1, len(steps) + 1):
        _, cov, _ = kalman.joint_posterior(model.cov(), model.a,
                                           dense_obs(model, steps, acts), upto=k)
        sl = slice((k - 1) * n, k * n)
        np.testing.assert_allclose(lin_f[k - 1] @ lin_f[k - 1].T, cov[sl, sl], atol=1e-9)


def test_full_action_paths_follow_the_rts_posterior():
    model, steps = tiny_problem(seed=44, n=10, T=3, m=10)
    recs = run_filter(model, steps, 10, 1000, policy="given",
                      actions=[np.eye(10) for _ in steps])
    kf = kalman.kalman_filter(model.cov(), model.a, dense_obs(model, steps))
    ms, Ps = kalman.rts_smoother(model.a, kf)
    _, mean_s, _, lin_s = _moments(model, steps, recs)
    for k in range(len(steps)):
        np.testing.assert_allclose(mean_s[k][:, 0], ms[k], atol=1e-9)
        np.testing.assert_allclose(lin_s[k] @ lin_s[k].T, Ps[k], atol=1e-9)
