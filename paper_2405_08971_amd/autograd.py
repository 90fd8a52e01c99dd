"""The filter's log-likelihood as a differentiable torch function.

loglik(theta, X, steps, ...) runs the filter on the device with the parameters
theta = (lengthscale, ell_t, signal_var, noise_var) (a float64 tensor of 4) and returns
the sum of the projected log-likelihood terms (cakf_loglik).  Its backward calls the
library's reverse sweep (cakf_loglik_grad), which differentiates the filter as it was run:
the actions and the truncation rotations of the forward pass are held fixed.  The OU
coefficient a = exp(-dt / ell_t) is the library's parameter; given dt, the library returns
the derivative with respect to ell_t itself, so this module only marshals arguments.

The forward pass keeps, per step, the record, the filtered mean, the truncated factor and
the truncation rotation (the tape of the reverse sweep) in device tensors until backward.
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import torch

from . import _lib as L
from .filter import CAKF, Record


class _Tape:
    def __init__(self):
        self.steps = []      # cakf_tape_step structs
        self.keep = []       # tensors referenced by the structs


class FilterLogLik(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, X, steps, actions, opts):
        ell, ell_t, sigma_f2, noise = (float(v) for v in theta.detach().cpu().tolist())
        a = math.exp(-opts["dt"] / ell_t)
        f = CAKF(X, nu2=opts["nu2"], dist=opts["dist"], lengthscale=ell, signal_var=sigma_f2,
                 noise_var=noise, ou_coeff=a, max_obs=opts["max_obs"],
                 max_actions=opts["max_actions"], max_rank=opts["max_rank"],
                 policy=opts["policy"], pivot_tol=opts["pivot_tol"], prec=opts["prec"],
                 gradient=True)
        tape = _Tape()
        i = opts["max_actions"]
        r = opts["max_rank"]
        for k, item in enumerate(steps):
            f.predict()
            if item is None:
                idx = y = None
                rec = None
                m = 0
            else:
                idx, y = item
                m = int(idx.numel())
                rec = Record(m, i)
            act = None if actions is None else actions[k]
            f.update(idx, y, act, rec)
            full = f.rank
            rot = None
            if full > r:
                rot = torch.empty((full, r), dtype=torch.float64, device="cuda")
            f.truncate(rot)
            mean, factor = f.state()
            rank = factor.shape[1]
            fac = factor if rank else torch.zeros((f.n, 1), dtype=torch.float32, device="cuda")
            st = L.cakf_tape_step(
                idx=L.ptr(idx) if m else None, y=L.ptr(y) if m else None, m=m,
                S=L.ptr(rec.S) if m else None, W_obs=L.ptr(rec.W_obs) if m else None,
                w_obs=L.ptr(rec.w_obs) if m else None, chol=L.ptr(rec.chol) if m else None,
                chol_inv=L.ptr(rec.chol_inv) if m else None,
                n_actions=L.ptr(rec.n_actions) if m else None, mean=L.ptr(mean),
                factor=L.ptr(fac), ld=fac.shape[1], rank=rank,
                rotation=L.ptr(rot) if rot is not None else None, rank_full=full)
            tape.steps.append(st)
            tape.keep.append((idx, y, rec, mean, fac, rot))
        value, _ = f.loglik()
        ctx.filter = f
        ctx.tape = tape
        ctx.dt = opts["dt"]
        return torch.tensor(value, dtype=torch.float64)

    @staticmethod
    def backward(ctx, g):
        f = ctx.filter
        d = f.loglik_grad(ctx.tape.steps, ctx.dt)
        f.close()
        ctx.tape = None
        return torch.tensor(d, dtype=torch.float64) * g.cpu(), None, None, None, None


def loglik(theta: torch.Tensor, X: torch.Tensor, steps: Sequence, *, nu2: int = 3,
           dist: str = "euclid", dt: float = 1.0, max_obs: int, max_actions: int,
           max_rank: int, policy: str = "cg", actions: Optional[Sequence] = None,
           pivot_tol: float = 1e-10, prec: str = "fp32") -> torch.Tensor:
    """Projected log-likelihood of the filter run on steps = [(idx, y) or None, ...]
    (device int32 / float32 tensors) at theta = (lengthscale, ell_t, signal_var,
    noise_var), differentiable in theta."""
    opts = dict(nu2=nu2, dist=dist, dt=dt, max_obs=max_obs, max_actions=max_actions,
                max_rank=max_rank, policy=policy, pivot_tol=pivot_tol, prec=prec)
    return FilterLogLik.apply(theta, X, list(steps), actions, opts)
