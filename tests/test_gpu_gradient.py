"""GPU parity of the log-likelihood derivative (cakf_loglik_grad through the torch
autograd function) against the FP64 oracle.

The GPU run chooses its CG actions and truncation rotations; the oracle replays the
filter in FP64 with those actions and rotations frozen (the function the reverse sweep
differentiates) and differentiates it two ways: forward mode (oracle.tangent) and
central differences (oracle.grad.fd_gradient).  Bar: each component within 1e-4 of the
oracle, relative to its magnitude (FP32 filter).
"""
import math
from types import SimpleNamespace

import numpy as np
import pytest

from gpu_common import inputs, small_config
from oracle import tangent
from oracle.cakf import Model
from oracle.grad import fd_gradient, model_at

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-4


def _run(cfg, seed, missing=(), prec="fp32", policy="cg"):
    import torch
    from paper_2405_08971_amd.autograd import FilterLogLik

    X, steps, actions = inputs(cfg, seed=seed, missing_steps=missing, policy=policy)
    dt = 1.0
    theta0 = (cfg.ell, cfg.ell_t, cfg.sigma_f2, cfg.noise_var)
    dev_steps = [None if s is None else (torch.from_numpy(s[0]).cuda(),
                                         torch.from_numpy(s[1]).cuda()) for s in steps]
    dev_acts = None if policy == "cg" else [None if a is None else torch.from_numpy(a).cuda()
                                            for a in actions]
    theta = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    opts = dict(nu2=cfg.nu2, dist="geodesic" if cfg.dist == 1 else "euclid", dt=dt,
                max_obs=cfg.m, max_actions=cfg.i, max_rank=cfg.r, policy=policy,
                pivot_tol=1e-10, prec=prec)
    ll = FilterLogLik.apply(theta, torch.from_numpy(X).cuda(), dev_steps, dev_acts, opts)
    # the frozen actions and rotations, read back before backward releases the tape
    recs = []
    for k, keep in enumerate(FilterLogLik_last_tape(ll)):
        idx, y, rec, mean, fac, rot = keep
        if rec is None:
            recs.append(SimpleNamespace(S=None, i_eff=0, V_r=None if rot is None
                                        else rot.cpu().numpy()))
        else:
            j = int(rec.n_actions.item())
            recs.append(SimpleNamespace(S=rec.S.cpu().numpy().astype(np.float64)[:, :j],
                                        i_eff=j,
                                        V_r=None if rot is None else rot.cpu().numpy()))
    ll.backward()
    g = theta.grad.numpy().copy()
    base = Model(X.astype(np.float64), cfg.nu2, cfg.ell, cfg.sigma_f2, cfg.a, cfg.noise_var,
                 cfg.dist)
    base = model_at(base, dt, theta0)
    ost = [None if s is None else (s[0].astype(np.int64), s[1].astype(np.float64))
           for s in steps]
    value, g_tan = tangent.replay_tangent(base, dt, theta0, ost, recs)
    return float(ll.item()), g, value, g_tan, (base, dt, theta0, ost, recs)


def FilterLogLik_last_tape(ll):
    return ll.grad_fn.tape.keep


def _check(got, ref, tol):
    rel = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-12)
    print("gpu", got, "\noracle", ref, "\nrel", rel, flush=True)
    assert np.all(rel <= tol), rel


@pytest.mark.parametrize("nu2", [1, 3, 5])
def test_gradient_matches_oracle_with_truncation(nu2):
    cfg = small_config(f"g{nu2}", nu2=nu2, n=500, m=160, i=6, r=10, T=5)
    value_gpu, g, value, g_tan, _ = _run(cfg, seed=20 + nu2, missing=(3,))
    assert abs(value_gpu - value) <= 1e-5 * abs(value), (value_gpu, value)
    _check(g, g_tan, GRAD_TOL)


def test_gradient_matches_fd_of_the_fp64_replay():
    cfg = small_config("gfd", n=400, m=130, i=5, r=8, T=4)
    _, g, _, g_tan, (base, dt, theta0, ost, recs) = _run(cfg, seed=30)
    fd = fd_gradient(base, dt, theta0, ost, recs, cfg.r)
    np.testing.assert_allclose(g_tan, fd, rtol=1e-6, atol=1e-8)
    _check(g, fd, GRAD_TOL)


def test_gradient_with_more_than_160_action_columns():
    """i = 200 given actions: the kernel-term sweeps of the reverse pass take the b = 201
    columns of [W w] (and the 200 of S) in two column blocks (160 + 41)."""
    cfg = small_config("gwide", n=900, m=420, i=200, r=40, T=3)
    value_gpu, g, value, g_tan, _ = _run(cfg, seed=33, policy="given")
    assert abs(value_gpu - value) <= 1e-5 * abs(value), (value_gpu, value)
    _check(g, g_tan, GRAD_TOL)


def test_gradient_on_the_sphere_geodesic():
    cfg = small_config("ggeo", dist=1, n=600, m=200, i=8, r=12, T=4)
    _, g, _, g_tan, _ = _run(cfg, seed=31)
    _check(g, g_tan, GRAD_TOL)


def test_given_action_gradient_with_the_oracles_own_rotations():
    """Given actions, and the oracle computes its own truncation rotations (FP64 eigh of its
    own M^T M at the base parameters) instead of replaying the GPU's: the frozen-rotation
    likelihood depends on the rotation only through the projector V_r V_r^T, which both
    sides agree on, so the derivatives must agree without any GPU-produced input."""
    import torch
    from paper_2405_08971_amd.autograd import FilterLogLik
    from oracle.cakf import run_filter

    cfg = small_config("ggiv", n=500, m=160, i=6, r=10, T=5)
    X, steps, actions = inputs(cfg, seed=32, missing_steps=(3,), policy="given")
    dt = 1.0
    theta0 = (cfg.ell, cfg.ell_t, cfg.sigma_f2, cfg.noise_var)
    dev_steps = [None if s is None else (torch.from_numpy(s[0]).cuda(),
                                         torch.from_numpy(s[1]).cuda()) for s in steps]
    dev_acts = [None if a is None else torch.from_numpy(a).cuda() for a in actions]
    theta = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    opts = dict(nu2=cfg.nu2, dist="euclid", dt=dt, max_obs=cfg.m, max_actions=cfg.i,
                max_rank=cfg.r, policy="given", pivot_tol=1e-10, prec="fp32")
    ll = FilterLogLik.apply(theta, torch.from_numpy(X).cuda(), dev_steps, dev_acts, opts)
    ll.backward()
    g = theta.grad.numpy().copy()
    base = model_at(Model(X.astype(np.float64), cfg.nu2, cfg.ell, cfg.sigma_f2, cfg.a,
                          cfg.noise_var, cfg.dist), dt, theta0)
    ost = [None if s is None else (s[0].astype(np.int64), s[1].astype(np.float64))
           for s in steps]
    acts = [None if a is None else a.astype(np.float64) for a in actions]
    recs = run_filter(base, ost, cfg.i, cfg.r, policy="given", actions=acts)
    assert sum(r.V_r is not None for r in recs) >= 2     # the rotations are the oracle's
    value, g_tan = tangent.replay_tangent(base, dt, theta0, ost, recs)
    assert abs(float(ll.item()) - value) <= 1e-5 * abs(value), (float(ll.item()), value)
    _check(g, g_tan, GRAD_TOL)
