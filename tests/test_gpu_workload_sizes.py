"""The n = 16384 workloads at their own sizes, against the FP64 oracle.

Differentiation workload (n = 16384 sphere points, chordal Matern-3/2, m = 4096, i = 64 CG
actions, r = 256): the reverse sweep of cakf_loglik_grad over six steps (the last two
truncate 320 -> 256 columns) against central differences of the FP64 replay of the same
filter (batch update of Alg. 2 with the run's actions and truncation rotations frozen, the
function the sweep differentiates).  The comparison is normwise over the log-parameter
sensitivities theta_i d(loglik)/d(theta_i), within 1e-5 of the largest: the plain
components differ by four orders of magnitude (the temporal lengthscale's is the
smallest), and the FP32 forward leaves absolute errors on the scale of the largest terms,
so a per-component relative bar would test the rounding of one small component.

Great-circle workload (n = 16384 sphere points, great-circle Matern-3/2, m = 4096,
i = 64 given actions, r = 256): four filter steps and the smoother's backward pass
(Alg. 3) against the FP64 oracle on the seeded 2048-point subset: means and marginal
variances, FP32 at 1e-5 and BF16X3 at 1e-3 relative mean error.

The oracle runs on the host's cores (tens of seconds per test)."""
import os
import time
from types import SimpleNamespace

import numpy as np
import pytest

from gpu_common import MAX_FACTOR, gpu_run_smoother, rel_max_err, rel_mean_err
from oracle.caks import run_smoother
from oracle.cakf import Model, run_filter
from oracle.grad import fd_gradient, model_at, replay_loglik
from paper_2405_08971_amd.workload import CONFIGS, Workload

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-5


def _threads():
    n = max(1, min(16, os.cpu_count() or 1))
    os.environ["ORACLE_THREADS"] = str(n)
    return n


def _steps(wl, T, policy):
    steps, actions = [], []
    for k in range(1, T + 1):
        idx, y = wl.step(k)
        steps.append((idx.astype(np.int32), y.astype(np.float32)))
        actions.append(wl.actions(k).astype(np.float32) if policy == "given" else None)
    return steps, actions


def test_differentiation_workload_gradient_matches_fd_of_the_fp64_replay():
    import torch
    from paper_2405_08971_amd.autograd import FilterLogLik

    _threads()
    cfg = CONFIGS["sphere_n16384"]
    T = 6
    wl = Workload(cfg, seed=0)
    X = wl.X.astype(np.float32)
    steps, _ = _steps(wl, T, "cg")
    theta0 = (cfg.ell, cfg.ell_t, cfg.sigma_f2, cfg.noise_var)
    theta = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    opts = dict(nu2=cfg.nu2, dist="euclid", dt=cfg.dt, max_obs=cfg.m, max_actions=cfg.i,
                max_rank=cfg.r, policy="cg", pivot_tol=1e-10, prec="fp32")
    dev_steps = [(torch.from_numpy(i).cuda(), torch.from_numpy(y).cuda()) for i, y in steps]
    ll = FilterLogLik.apply(theta, torch.from_numpy(X).cuda(), dev_steps, None, opts)
    recs = []
    for idx, y, rec, mean, fac, rot in ll.grad_fn.tape.keep:
        j = int(rec.n_actions.item())
        recs.append(SimpleNamespace(S=rec.S.cpu().numpy().astype(np.float64)[:, :j], i_eff=j,
                                    V_r=None if rot is None else rot.cpu().numpy()))
    ll.backward()
    g = theta.grad.numpy().copy()
    assert sum(r.V_r is not None for r in recs) == 2          # steps 5 and 6 truncate
    base = model_at(Model(X.astype(np.float64), cfg.nu2, cfg.ell, cfg.sigma_f2, cfg.a,
                          cfg.noise_var, cfg.dist), cfg.dt, theta0)
    ost = [(i.astype(np.int64), y.astype(np.float64)) for i, y in steps]
    t0 = time.perf_counter()
    value = replay_loglik(base, cfg.dt, theta0, ost, recs, cfg.r, form="batch")
    fd = fd_gradient(base, cfg.dt, theta0, ost, recs, cfg.r, rel_step=1e-4, form="batch")
    th = np.asarray(theta0, dtype=np.float64)
    rel = np.abs(th * (g - fd)) / np.max(np.abs(th * fd))
    print(f"log-likelihood gpu {float(ll.item()):.10e} fp64 {value:.10e}\n"
          f"gradient gpu {g}\n         fd  {fd}\nlog-sensitivity error / largest {rel} "
          f"({time.perf_counter() - t0:.0f} s of FP64 replays)", flush=True)
    assert abs(float(ll.item()) - value) <= 1e-5 * abs(value)
    assert np.all(rel <= GRAD_TOL), rel


_GC = {}


def _great_circle_reference(T):
    """Inputs and the FP64 smoothed moments on the subset (computed once per session)."""
    if T not in _GC:
        cfg = CONFIGS["sphere_gc_n16384"]
        wl = Workload(cfg, seed=0)
        X = wl.X.astype(np.float32)
        steps, actions = _steps(wl, T, "given")
        sub = wl.subset(2048)
        t0 = time.perf_counter()
        model = Model(X.astype(np.float64), cfg.nu2, cfg.ell, cfg.sigma_f2, cfg.a,
                      cfg.noise_var, cfg.dist)
        recs = run_filter(model, [(i.astype(np.int64), y.astype(np.float64)) for i, y in steps],
                          cfg.i, cfg.r, policy="given",
                          actions=[a.astype(np.float64) for a in actions], form="batch",
                          lsqrt="chol")
        sm = run_smoother(model, recs, cfg.r)
        ref = [(r.m[sub], r.marginal_var(cfg.sigma_f2)[sub]) for r in sm]
        _GC[T] = (cfg, X, steps, actions, sub, ref, time.perf_counter() - t0)
    return _GC[T]


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16x3", 1e-3)])
def test_great_circle_workload_filter_and_smoother(prec, tol):
    _threads()
    T = 4
    cfg, X, steps, actions, sub, ref, secs = _great_circle_reference(T)
    gpu = gpu_run_smoother(cfg, X, steps, actions, "given", prec)
    worst = 0.0
    for k in range(T):
        ref_m, ref_v = ref[k]
        em, ev = rel_mean_err(gpu[k][0][sub], ref_m), rel_mean_err(gpu[k][1][sub], ref_v)
        xm, xv = rel_max_err(gpu[k][0][sub], ref_m), rel_max_err(gpu[k][1][sub], ref_v)
        print(f"{prec} step {k + 1}: smoothed mean {em:.2e} (max {xm:.2e}), variance {ev:.2e} "
              f"(max {xv:.2e})", flush=True)
        worst = max(worst, em, ev)
        assert em <= tol and ev <= tol, (k, em, ev)
        assert xm <= MAX_FACTOR * tol and xv <= MAX_FACTOR * tol, (k, xm, xv)
    print(f"worst {worst:.2e}; FP64 filter + smoother on the host {secs:.0f} s", flush=True)
