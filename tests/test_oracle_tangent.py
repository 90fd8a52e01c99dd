"""Pins of the oracle's forward-mode likelihood derivative (oracle.tangent).

* its value is the replayed log-likelihood of the iterative filter (same frozen
  actions and rotations);
* its derivative equals the central-difference derivative of that replay, which is
  itself pinned to the textbook GP evidence gradient (test_oracle_smoother_grad);
* a planted mistake (dropping the Mo Mo^T term of the Gram derivative) is caught.
"""
import numpy as np
import pytest

from oracle import tangent
from oracle.cakf import run_filter
from oracle.grad import fd_gradient, model_at, replay_loglik
from tiny import tiny_problem


def _setup(seed, T, m, r_cap, nu2=3, missing=(), policy="cg", dim=2):
    model, steps = tiny_problem(seed=seed, T=T, m=m, nu2=nu2, missing_steps=missing, dim=dim)
    dt, theta = 1.0, (0.3, 5.0, 1.3, 0.05)
    base = model_at(model, dt, theta)
    recs = run_filter(base, steps, 3, r_cap, policy=policy)
    return base, dt, theta, steps, recs


@pytest.mark.parametrize("nu2", [1, 3, 5])
def test_tangent_matches_replay_value_and_fd(nu2):
    base, dt, theta, steps, recs = _setup(40 + nu2, T=5, m=8, r_cap=4, nu2=nu2, missing=(3,))
    assert any(r.V_r is not None for r in recs)       # truncation happens
    value, g = tangent.replay_tangent(base, dt, theta, steps, recs)
    assert value == pytest.approx(replay_loglik(base, dt, theta, steps, recs, 4), abs=1e-9)
    fd = fd_gradient(base, dt, theta, steps, recs, 4)
    np.testing.assert_allclose(g, fd, rtol=2e-6, atol=1e-8)


def test_tangent_on_the_sphere_with_geodesic_distance():
    from oracle import matern
    base, dt, theta, steps, recs = _setup(47, T=4, m=7, r_cap=5, dim=3)
    base.dist = matern.GEODESIC
    recs = run_filter(base, steps, 3, 5, policy="cg")
    _, g = tangent.replay_tangent(base, dt, theta, steps, recs)
    fd = fd_gradient(base, dt, theta, steps, recs, 5)
    np.testing.assert_allclose(g, fd, rtol=2e-6, atol=1e-8)


def test_planted_mistake_in_gram_derivative_is_caught(monkeypatch):
    base, dt, theta, steps, recs = _setup(48, T=4, m=8, r_cap=4)
    fd = fd_gradient(base, dt, theta, steps, recs, 4)
    real_phi = tangent._phi
    # plant: use the full symmetric differential instead of the triangular solve
    monkeypatch.setattr(tangent, "_phi", lambda X: np.tril(X))
    _, g_bad = tangent.replay_tangent(base, dt, theta, steps, recs)
    monkeypatch.setattr(tangent, "_phi", real_phi)
    assert not np.allclose(g_bad, fd, rtol=1e-4, atol=1e-8)
