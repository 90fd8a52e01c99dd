"""Helpers shared by the GPU tests: run the HIP library and the FP64 oracle on the same
seeded inputs and compare.  (Not a test module.)"""
from __future__ import annotations

import math

import numpy as np

from oracle.cakf import Model, run_filter
from paper_2405_08971_amd.workload import Config, Workload


def rel_mean_err(x, ref) -> float:
    """mean |x - ref| / mean |ref| (the per-result relative error)."""
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.mean(np.abs(ref))
    return float(np.mean(np.abs(x - ref)) / (den if den > 0 else 1.0))


def rel_max_err(x, ref) -> float:
    """max |x - ref| / mean |ref|: the worst single entry on the scale of the result (an
    element-wise bound that, unlike |x - ref| / |ref|, stays finite where ref crosses 0)."""
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.mean(np.abs(ref))
    return float(np.max(np.abs(x - ref), initial=0.0) / (den if den > 0 else 1.0))


# The element-wise bar is this multiple of the relative-mean bar: the largest of ~10^3
# errors of one distribution sits a few times above their mean, while one entry that is
# entirely wrong lands near 1 and fails it.
MAX_FACTOR = 10.0


def small_config(name="p", **kw) -> Config:
    base = dict(name=name, n=800, dim=3, nu2=3, ell=0.3, sigma_f2=1.0, dt=1.0, ell_t=5.0,
                T=6, m=300, noise_var=0.05, i=8, r=20)
    base.update(kw)
    return Config(**base)


def inputs(cfg: Config, seed=0, missing_steps=(), policy="given"):
    """float32-rounded inputs shared by both sides."""
    wl = Workload(cfg, seed=seed, n_features=512)
    X = wl.X.astype(np.float32)
    steps, actions = [], []
    for k in range(1, cfg.T + 1):
        if k in missing_steps:
            steps.append(None)
            actions.append(None)
            continue
        idx, y = wl.step(k)
        steps.append((idx.astype(np.int32), y.astype(np.float32)))
        actions.append(wl.actions(k).astype(np.float32) if policy == "given" else None)
    return X, steps, actions


def oracle_run(cfg: Config, X, steps, actions, policy, pivot_tol=1e-10, resid_tol=0.0):
    model = Model(X.astype(np.float64), cfg.nu2, cfg.ell, cfg.sigma_f2, cfg.a, cfg.noise_var,
                  cfg.dist)
    st = [None if s is None else (s[0].astype(np.int64), s[1].astype(np.float64)) for s in steps]
    acts = None if policy != "given" else [None if a is None else a.astype(np.float64)
                                           for a in actions]
    return model, run_filter(model, st, cfg.i, cfg.r, policy=policy, actions=acts,
                             pivot_tol=pivot_tol, resid_tol=resid_tol)


def gpu_run(cfg: Config, X, steps, actions, policy, prec="fp32", probes=None,
            pivot_tol=1e-10, resid_tol=0.0, temporal="ou"):
    """Run the library step by step; returns per-step host results."""
    import torch
    from paper_2405_08971_amd.filter import CAKF, Record

    dev = "cuda"
    Xd = torch.from_numpy(X).to(dev)
    block_actions = 1
    if isinstance(policy, tuple):          # ("block", b), as the oracle names it
        policy, block_actions = policy[0], int(policy[1])
    f = CAKF(Xd, nu2=cfg.nu2, dist="geodesic" if cfg.dist == 1 else "euclid",
             lengthscale=cfg.ell, signal_var=cfg.sigma_f2, noise_var=cfg.noise_var,
             ou_coeff=cfg.a, max_obs=cfg.m, max_actions=cfg.i, max_rank=cfg.r, policy=policy,
             block_actions=block_actions, pivot_tol=pivot_tol, resid_tol=resid_tol, prec=prec,
             temporal=temporal)
    P = None if probes is None else torch.from_numpy(probes.astype(np.float32)).to(dev)
    out = []
    for k, item in enumerate(steps):
        f.predict()
        rec = None
        if item is None:
            f.update(None, None)
        else:
            idx = torch.from_numpy(item[0]).to(dev)
            y = torch.from_numpy(item[1]).to(dev)
            a = None if actions[k] is None else torch.from_numpy(actions[k]).to(dev)
            rec = Record(len(item[0]), cfg.i)
            f.update(idx, y, a, rec)
        mean, M = f.state()
        var = f.marginal_var()
        res = dict(mean=mean.cpu().numpy().astype(np.float64),
                   var=var.cpu().numpy().astype(np.float64), rank=M.shape[1],
                   rowsq=(M.double() ** 2).sum(1).cpu().numpy())
        if P is not None:
            res["MMt_probe"] = (M.double() @ (M.double().T @ P.double())).cpu().numpy()
        if rec is not None:
            torch.cuda.synchronize()
            res.update(loglik=float(rec.loglik.item()), n_actions=int(rec.n_actions.item()),
                       S=rec.S.cpu().numpy(), W_obs=rec.W_obs.cpu().numpy(),
                       w_obs=rec.w_obs.cpu().numpy())
        else:
            res.update(loglik=0.0, n_actions=0)
        f.truncate()
        Mp = f.state()[1]
        res["var_trunc"] = f.marginal_var().cpu().numpy().astype(np.float64)
        res["rowsq_trunc"] = (Mp.double() ** 2).sum(1).cpu().numpy()
        res["rank_trunc"] = Mp.shape[1]
        out.append(res)
    torch.cuda.synchronize()
    f.close()
    return out


def compare(cfg, model, recs, gpu, probes=None):
    """Per-step relative mean errors of mean, marginal variance and log-likelihood."""
    errs = []
    for rec, g in zip(recs, gpu):
        var = rec.marginal_var(cfg.sigma_f2)
        var_trunc = cfg.sigma_f2 - np.sum(rec.M_plus ** 2, axis=1)
        e = dict(mean=rel_mean_err(g["mean"], rec.m),
                 var=rel_mean_err(g["var"], var),
                 var_trunc=rel_mean_err(g["var_trunc"], var_trunc),
                 mean_max=rel_max_err(g["mean"], rec.m),
                 var_max=rel_max_err(g["var"], var),
                 var_trunc_max=rel_max_err(g["var_trunc"], var_trunc),
                 loglik=abs(g["loglik"] - rec.loglik) / max(abs(rec.loglik), 1e-300),
                 n_actions=(g["n_actions"], rec.i_eff))
        if probes is not None:
            e["MMt"] = rel_mean_err(g["MMt_probe"], rec.M @ (rec.M.T @ probes))
        errs.append(e)
    return errs


def gpu_run_smoother(cfg: Config, X, steps, actions, policy, prec="fp32"):
    """Filter forward keeping m_k, M_k, M_k^- and the records, then the smoother backward.
    Returns per-step (smoothed mean, smoothed marginal variance), k = 1..T."""
    import torch
    from paper_2405_08971_amd.filter import CAKF, Record

    dev = "cuda"
    Xd = torch.from_numpy(X).to(dev)
    f = CAKF(Xd, nu2=cfg.nu2, dist="geodesic" if cfg.dist == 1 else "euclid",
             lengthscale=cfg.ell, signal_var=cfg.sigma_f2, noise_var=cfg.noise_var,
             ou_coeff=cfg.a, max_obs=cfg.m, max_actions=cfg.i, max_rank=cfg.r, policy=policy,
             prec=prec, smoother=True)
    fwd = []
    for k, item in enumerate(steps):
        f.predict()
        _, Mp = f.state()
        rec, idx = None, None
        if item is None:
            f.update(None, None)
        else:
            idx = torch.from_numpy(item[0]).to(dev)
            y = torch.from_numpy(item[1]).to(dev)
            a = None if actions[k] is None else torch.from_numpy(actions[k]).to(dev)
            rec = Record(len(item[0]), cfg.i)
            f.update(idx, y, a, rec)
        mean, M = f.state()
        fwd.append((mean, M, Mp, idx, rec))
        f.truncate()
    T = len(steps)
    out = [None] * T
    mean_T, M_T = fwd[-1][0], fwd[-1][1]
    var_T = cfg.sigma_f2 - (M_T.double() ** 2).sum(1)
    out[T - 1] = (mean_T.cpu().numpy().astype(np.float64), var_T.cpu().numpy())
    f.smooth_begin(fwd[-1][3], fwd[-1][4])
    for k in range(T - 2, -1, -1):
        mean, M, Mp, idx, rec = fwd[k]
        ms, vs, _ = f.smooth_step(mean, M, Mp, idx, rec)
        out[k] = (ms.cpu().numpy().astype(np.float64), vs.cpu().numpy().astype(np.float64))
    torch.cuda.synchronize()
    f.close()
    return out
