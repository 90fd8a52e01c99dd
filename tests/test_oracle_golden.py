"""The oracle's filter and smoother on a two-point example worked out by hand.

The fixture ``golden/two_point_filter.txt`` states the example and its exact filtering
moments and log-likelihood in closed form (the Kalman filter's predict and update steps
of Sec. 2 with a Matern-1/2 prior and an Ornstein-Uhlenbeck transition); with one
observation per step the computation-aware filter is exact (Prop. A.2), and so is its
smoother (Alg. 3), whose step-1 moments the fixture gives by the Rauch-Tung-Striebel step.
"""
import numpy as np

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
