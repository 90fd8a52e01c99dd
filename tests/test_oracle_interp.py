"""Pins of the oracle's temporal interpolation (App. C, the corollary on temporal
interpolation): without truncation the interpolated belief at any time t equals the
brute-force conditioning of the joint Gaussian of the states at the step times and at t
(covariance exp(-|t_i - t_j| / ell_t) Sigma) on the projected data of the steps up to
t (filter) or of all steps (smoother), for t inside, before and after the steps; at a
step time it is that step's filter or smoother moments."""
import math

import numpy as np
import pytest

from oracle.caks import run_smoother
from oracle.cakf import run_filter
from oracle.interp import interpolate
from tiny import tiny_problem

DT = 1.0


def _brute(model, steps, actions, t, upto):
    """Mean and covariance at time t given the projected data of steps 1..upto."""
    n, T = model.n, len(steps)
    ell_t = -DT / math.log(model.a)
    times = np.array([k * DT for k in range(1, T + 1)] + [t])
    lag = np.abs(np.subtract.outer(times, times))
    C = np.kron(np.exp(-lag / ell_t), model.cov())
    rows, ys, Rs = [], [], []
    for k in range(min(upto, T)):
        if steps[k] is None:
            continue
        idx, y = steps[k]
        S = actions[k]
        H = np.zeros((S.shape[1], (T + 1) * n))
        H[:, k * n + np.asarray(idx)] = S.T
        rows.append(H)
        ys.append(S.T @ y)
        Rs.append(model.noise_var * S.T @ S)
    sl = slice(T * n, (T + 1) * n)
    if not rows:
        return np.zeros(n), C[sl, sl]
    Hall = np.vstack(rows)
    yall = np.concatenate(ys)
    R = np.zeros((yall.size, yall.size))
    o = 0
    for Rk in Rs:
        R[o:o + Rk.shape[0], o:o + Rk.shape[0]] = Rk
        o += Rk.shape[0]
    G = Hall @ C @ Hall.T + R
    CHt = C[sl] @ Hall.T
    return CHt @ np.linalg.solve(G, yall), C[sl, sl] - CHt @ np.linalg.solve(G, CHt.T)


@pytest.fixture(scope="module")
def run():
    model, steps = tiny_problem(seed=60, n=12, T=4, m=7, missing_steps=(3,))
    rng = np.random.default_rng(61)
    actions = [None if s is None else rng.standard_normal((7, 3)) for s in steps]
    recs = run_filter(model, steps, 3, 1000, policy="given", actions=actions)
    sm = run_smoother(model, recs, 1000)
    return model, steps, actions, recs, sm


@pytest.mark.parametrize("t", [0.3, 1.0, 1.4, 2.75, 3.5, 4.0, 5.2])
def test_interpolated_belief_is_the_joint_posterior(run, t):
    model, steps, actions, recs, sm = run
    T = len(steps)
    for smoothed in (False, True):
        m_t, M_t = interpolate(model, recs, sm, t, DT, smoothed)
        upto = T if smoothed else int(math.floor(t / DT + 1e-12))
        mean, cov = _brute(model, steps, actions, t, upto)
        np.testing.assert_allclose(m_t, mean, atol=1e-9)
        np.testing.assert_allclose(model.cov() - M_t @ M_t.T, cov, atol=1e-9)


def test_step_times_give_the_step_moments(run):
    model, steps, actions, recs, sm = run
    for k in range(1, len(steps) + 1):
        m_f, M_f = interpolate(model, recs, sm, k * DT, DT, False)
        np.testing.assert_allclose(m_f, recs[k - 1].m, atol=1e-12)
        m_s, M_s = interpolate(model, recs, sm, k * DT, DT, True)
        np.testing.assert_allclose(m_s, sm[k - 1].m, atol=1e-10)
        np.testing.assert_allclose(M_s @ M_s.T, sm[k - 1].M @ sm[k - 1].M.T, atol=1e-10)
