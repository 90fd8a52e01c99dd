"""The oracle's filter and smoother on a two-point example worked out by hand.

The fixture ``golden/two_point_filter.txt`` states the example and its exact filtering
moments and log-likelihood in closed form (the Kalman filter's predict and update steps
of Sec. 2 with a Matern-1/2 prior and an Ornstein-Uhlenbeck transition); with one
observation per step the computation-aware filter is exact (Prop. A.2), and so is its
smoother (Alg. 3), whose step-1 moments the fixture gives by the Rauch-Tung-Striebel step.
The example's total log-likelihood, written in closed form in the four parameters, also
pins the oracle's forward-mode derivative.
"""
import numpy as np
import pytest

from oracle.caks import run_smoother
from oracle.cakf import Model, run_filter
from tiny import load_golden


def _problem(g):
    X = np.array([[0.0, 0.0], [1.0, 0.0]])
    model = Model(X, 1, g["ell"], g["sigma_f2"], g["a"], g["noise_var"])
    steps = [(np.array([int(g["obs1_index"])]), np.array([g["obs1_value"]])),
             (np.array([int(g["obs2_index"])]), np.array([g["obs2_value"]]))]
    return model, steps


def test_two_point_filter_matches_the_hand_worked_moments():
    g = load_golden("two_point_filter.txt")
    model, steps = _problem(g)
    for policy in ("cg", "given"):
        actions = [np.ones((1, 1)), np.full((1, 1), -3.0)] if policy == "given" else None
        recs = run_filter(model, steps, 1, 100, policy=policy, actions=actions)
        for k, rec in enumerate(recs, start=1):
            P = model.cov() - rec.M @ rec.M.T
            np.testing.assert_allclose(rec.m, [g[f"m{k}_0"], g[f"m{k}_1"]], rtol=0, atol=1e-13)
            P_ref = [[g[f"P{k}_00"], g[f"P{k}_01"]], [g[f"P{k}_01"], g[f"P{k}_11"]]]
            np.testing.assert_allclose(P, P_ref, rtol=0, atol=1e-13)
            np.testing.assert_allclose(rec.loglik, g[f"ll{k}"], rtol=0, atol=1e-13)


def test_two_point_smoother_matches_the_hand_worked_rts_step():
    g = load_golden("two_point_filter.txt")
    model, steps = _problem(g)
    recs = run_filter(model, steps, 1, 100, policy="cg")
    sm = run_smoother(model, recs, 100)
    np.testing.assert_allclose(sm[0].m, [g["ms1_0"], g["ms1_1"]], rtol=0, atol=1e-13)
    P = model.cov() - sm[0].M @ sm[0].M.T
    P_ref = [[g["Ps1_00"], g["Ps1_01"]], [g["Ps1_01"], g["Ps1_11"]]]
    np.testing.assert_allclose(P, P_ref, rtol=0, atol=1e-13)
    # the last step's smoothed moments are the filter's
    np.testing.assert_allclose(sm[1].m, [g["m2_0"], g["m2_1"]], rtol=0, atol=1e-13)


def _two_point_loglik(theta, y1, y2, dt=1.0):
    """Total log-likelihood of the two-point example as a closed form in the parameters.

    With s = sigma_f2, rho = s exp(-1/ell) (the Matern-1/2 covariance at distance 1),
    R = noise_var and a = exp(-dt/ell_t): the first innovation is y1 with variance
    S1 = s + R; the predicted variance of location 1 at step 2 is s - a^2 rho^2 / S1, so
    the second innovation is v2 = y2 - a rho y1 / S1 with variance S2 = s - a^2 rho^2 / S1
    + R, and the log-likelihood is the sum of the two Gaussian log densities."""
    ell, ell_t, s, R = theta
    a = np.exp(-dt / ell_t)
    rho = s * np.exp(-1.0 / ell)
    S1 = s + R
    S2 = s - a * a * rho * rho / S1 + R
    v2 = y2 - a * rho * y1 / S1
    return (-0.5 * np.log(2 * np.pi * S1) - 0.5 * y1 * y1 / S1
            - 0.5 * np.log(2 * np.pi * S2) - 0.5 * v2 * v2 / S2)


def test_two_point_loglik_derivative_matches_the_closed_form():
    from oracle import tangent
    from oracle.grad import model_at

    g = load_golden("two_point_filter.txt")
    model, steps = _problem(g)
    dt = 1.0
    theta = np.array([g["ell"], dt / np.log(1.0 / g["a"]), g["sigma_f2"], g["noise_var"]])
    y1, y2 = g["obs1_value"], g["obs2_value"]
    # the closed form reproduces the fixture's step terms at the example's parameters
    assert _two_point_loglik(theta, y1, y2) == pytest.approx(g["ll1"] + g["ll2"], abs=1e-14)
    base = model_at(model, dt, theta)
    recs = run_filter(base, steps, 1, 100, policy="cg")
    value, grad = tangent.replay_tangent(base, dt, theta, steps, recs)
    assert value == pytest.approx(g["ll1"] + g["ll2"], abs=1e-12)
    ref = np.zeros(4)
    for j in range(4):
        h = 1e-6 * theta[j]
        tp, tm = theta.copy(), theta.copy()
        tp[j] += h
        tm[j] -= h
        ref[j] = (_two_point_loglik(tp, y1, y2) - _two_point_loglik(tm, y1, y2)) / (2 * h)
    assert np.all(np.abs(ref) > 1e-3)          # every parameter matters in this example
    np.testing.assert_allclose(grad, ref, rtol=1e-7, atol=1e-9)
