"""Convenience wrapper over the libcakf C ABI for torch device tensors.

Only argument marshalling and buffer allocation happen here; every step of the filter
runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
import math
from typing import Optional

import torch

from . import _lib as L


class Record:
    """Caller-owned device buffers for one update's record (see cakf_record)."""

    def __init__(self, m: int, i: int, device="cuda"):
        self.m, self.i = m, i
        self.S = torch.zeros((m, i), dtype=torch.float32, device=device)
        self.W_obs = torch.zeros((m, i), dtype=torch.float32, device=device)
        self.w_obs = torch.zeros((m,), dtype=torch.float32, device=device)
        self.chol = torch.zeros((i, i), dtype=torch.float64, device=device)
        self.chol_inv = torch.zeros((i, i), dtype=torch.float64, device=device)
        self.loglik = torch.zeros((1,), dtype=torch.float64, device=device)
        self.n_actions = torch.zeros((1,), dtype=torch.int32, device=device)

    def c(self) -> L.cakf_record:
        return L.cakf_record(L.ptr(self.S), L.ptr(self.W_obs), L.ptr(self.w_obs),
                             L.ptr(self.chol), L.ptr(self.chol_inv), L.ptr(self.loglik),
                             L.ptr(self.n_actions))


class CAKF:
    """One filter context (state + workspace) on the current device and stream."""

    def __init__(self, X: torch.Tensor, *, nu2: int = 3, dist: str = "euclid",
                 lengthscale: float, signal_var: float = 1.0, noise_var: float,
                 ou_coeff: float, temporal: str = "ou", max_obs: int, max_actions: int,
                 max_rank: int,
                 policy: str = "cg", block_actions: int = 8, resid_tol: float = 0.0,
                 pivot_tol: float = 1e-10,
                 prec: str = "fp32", smoother: bool = False, gradient: bool = False,
                 sample_paths: int = 0, stream: Optional[torch.cuda.Stream] = None):
        if X.dtype != torch.float32 or X.dim() != 2:
            raise ValueError("X must be a float32 (n, dim) device tensor")
        X = X.contiguous()
        self.n, self.dim = X.shape
        self.N = self.n * (2 if temporal == "matern32" else 1)   # state rows
        self.max_actions, self.max_rank, self.max_obs = max_actions, max_rank, max_obs
        self.signal_var = signal_var
        self.policy = policy
        cfg = L.cakf_config(
            n=self.n, dim=self.dim, X=L.ptr(X), kernel=L.MATERN[nu2], dist=L.DIST[dist],
            lengthscale=lengthscale, signal_var=signal_var, noise_var=noise_var,
            ou_coeff=ou_coeff, temporal=L.TEMPORAL[temporal], max_obs=max_obs,
            max_actions=max_actions, max_rank=max_rank,
            policy=L.POLICY[policy], block_actions=block_actions, resid_tol=resid_tol,
            pivot_tol=pivot_tol,
            prec=L.PREC[prec], smoother=1 if smoother else 0, sample_paths=sample_paths,
            gradient=1 if gradient else 0, stream=L.stream_handle(stream))
        self._X = X
        self.ctx = L.cakf_create(cfg)

    # -- lifecycle -------------------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None):
            L.cakf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self):
        L.cakf_reset(self.ctx)

    # -- filter ----------------------------------------------------------------------
    def predict(self):
        L.cakf_predict(self.ctx)

    def update(self, idx: Optional[torch.Tensor], y: Optional[torch.Tensor],
               actions: Optional[torch.Tensor] = None, record: Optional[Record] = None):
        m = 0 if idx is None else int(idx.numel())
        rec = record.c() if record is not None else None
        L.cakf_update(self.ctx, idx, y, m, actions, rec)

    def truncate(self, rotation: Optional[torch.Tensor] = None):
        L.cakf_truncate(self.ctx, rotation)

    def step(self, idx, y, actions=None, record: Optional[Record] = None):
        m = 0 if idx is None else int(idx.numel())
        rec = record.c() if record is not None else None
        L.cakf_step(self.ctx, idx, y, m, actions, rec)

    # -- state -----------------------------------------------------------------------
    @property
    def rank(self) -> int:
        return L.cakf_state(self.ctx)[3]

    def state(self):
        """(mean, factor) copies: float32 (N,) and (N, rank), N the state rows."""
        rank = self.rank
        mean = torch.empty(self.N, dtype=torch.float32, device="cuda")
        factor = torch.empty((self.N, max(rank, 1)), dtype=torch.float32, device="cuda")
        L.cakf_copy_state(self.ctx, mean, factor, factor.shape[1])
        return mean, factor[:, :rank]

    def set_state(self, mean: torch.Tensor, factor: torch.Tensor):
        factor = factor.contiguous()
        rank = factor.shape[1]
        L.cakf_set_state(self.ctx, mean.contiguous(), factor if rank else None,
                         max(rank, 1), rank)

    def marginal_var(self, rows: Optional[torch.Tensor] = None) -> torch.Tensor:
        count = self.n if rows is None else int(rows.numel())
        out = torch.empty(count, dtype=torch.float32, device="cuda")
        L.cakf_marginal_var(self.ctx, rows, count, out)
        return out

    def diagnostics(self):
        return L.cakf_diagnostics(self.ctx)

    def loglik(self):
        """(sum of the projected log-likelihood terms, number of updates with data)."""
        return L.cakf_loglik(self.ctx)

    # -- smoother (Alg. 3) ---------------------------------------------------------------
    def smooth_begin(self, idx=None, record: Optional[Record] = None):
        m = 0 if idx is None else int(idx.numel())
        if m:
            L.cakf_smooth_begin(self.ctx, idx, record.w_obs, record.W_obs, m)
        else:
            L.cakf_smooth_begin(self.ctx, None, None, None, 0)

    @staticmethod
    def _smooth_input(mean, factor, pred_factor, idx, record):
        m = 0 if idx is None else int(idx.numel())
        return L.cakf_smooth_input(
            mean=L.ptr(mean), factor=L.ptr(factor) if factor.shape[1] else None,
            ld=max(factor.shape[1], 1), rank=factor.shape[1],
            pred_factor=L.ptr(pred_factor) if pred_factor.shape[1] else None,
            pred_ld=max(pred_factor.shape[1], 1), pred_rank=pred_factor.shape[1],
            idx=L.ptr(idx) if m else None, w_obs=L.ptr(record.w_obs) if m else None,
            W_obs=L.ptr(record.W_obs) if m else None, m=m)

    def smooth(self, steps):
        """The whole backward pass over steps = [(mean, factor, pred_factor, idx, record)]
        (k = 1..T, as for smooth_step).  Returns the smoothed means and marginal
        variances, both (T, n)."""
        keep = [(s[0], s[1].contiguous(), s[2].contiguous()) for s in steps]
        inp = [self._smooth_input(mean, fac, pf, s[3], s[4])
               for (mean, fac, pf), s in zip(keep, steps)]
        T = len(steps)
        means = torch.empty((T, self.n), dtype=torch.float32, device="cuda")
        var = torch.empty((T, self.n), dtype=torch.float32, device="cuda")
        L.cakf_smooth(self.ctx, inp, means, var)
        return means, var

    def smooth_step(self, mean, factor, pred_factor, idx=None, record: Optional[Record] = None,
                    want_factor: bool = False):
        """One backward step; factor / pred_factor are (n, rank) float32 device tensors.
        Returns (smoothed mean, marginal variances, smoothed factor or None)."""
        factor = factor.contiguous()
        pred_factor = pred_factor.contiguous()
        m = 0 if idx is None else int(idx.numel())
        inp = L.cakf_smooth_input(
            mean=L.ptr(mean), factor=L.ptr(factor) if factor.shape[1] else None,
            ld=max(factor.shape[1], 1), rank=factor.shape[1],
            pred_factor=L.ptr(pred_factor) if pred_factor.shape[1] else None,
            pred_ld=max(pred_factor.shape[1], 1), pred_rank=pred_factor.shape[1],
            idx=L.ptr(idx) if m else None, w_obs=L.ptr(record.w_obs) if m else None,
            W_obs=L.ptr(record.W_obs) if m else None, m=m)
        out_mean = torch.empty(self.n, dtype=torch.float32, device="cuda")
        out_var = torch.empty(self.n, dtype=torch.float32, device="cuda")
        out_fac = None
        ld = 0
        if want_factor:
            ld = factor.shape[1] + self.max_rank + self.max_actions
            out_fac = torch.empty((self.n, ld), dtype=torch.float32, device="cuda")
        rank = L.cakf_smooth_step(self.ctx, inp, out_mean, out_fac, ld, out_var)
        return out_mean, out_var, (out_fac[:, :rank] if want_factor else None)

    # -- path sampler (App. C) -------------------------------------------------------------
    @staticmethod
    def _sample_input(idx, y, record: Optional[Record], pred_factor: torch.Tensor):
        pred_factor = pred_factor.contiguous()
        m = 0 if idx is None else int(idx.numel())
        pr = pred_factor.shape[1]
        return L.cakf_sample_input(
            idx=L.ptr(idx) if m else None, y=L.ptr(y) if (m and y is not None) else None, m=m,
            S=L.ptr(record.S) if m else None, W_obs=L.ptr(record.W_obs) if m else None,
            chol_inv=L.ptr(record.chol_inv) if m else None,
            pred_factor=L.ptr(pred_factor) if pr else None, pred_ld=max(pr, 1), pred_rank=pr)

    def sample_forward(self, x_prev: torch.Tensor, q: torch.Tensor, e: Optional[torch.Tensor],
                       idx, y, record: Optional[Record], pred_factor: torch.Tensor,
                       static_scratch: bool = False, out=None):
        """Forward step of the path sampler: returns (x_k, w_obs_k) for the ns paths in the
        columns of x_prev (n x ns); q (n x ns) and e (m x ns) are the step's draws.
        static_scratch: run on the library's static scratch array
        (cakf_sample_forward_static, which allocates nothing); out: optional preallocated
        (x, w) with w of at least max(m, 1) rows."""
        ns = x_prev.shape[1]
        m = 0 if idx is None else int(idx.numel())
        inp = self._sample_input(idx, y, record, pred_factor)
        if out is None:
            x = torch.empty_like(x_prev)
            w = torch.empty((max(m, 1), ns), dtype=torch.float32, device="cuda")
        else:
            x, w = out
        fn = L.cakf_sample_forward_static if static_scratch else L.cakf_sample_forward
        fn(self.ctx, ns, x_prev.contiguous(), q.contiguous(), e.contiguous() if m else None, inp,
           x, w if m else None)
        return x, w[:m]

    def sample_lift(self, idx, w_obs: torch.Tensor, ns: int) -> torch.Tensor:
        m = 0 if idx is None else int(idx.numel())
        out = torch.empty((self.n, ns), dtype=torch.float32, device="cuda")
        L.cakf_sample_lift(self.ctx, ns, idx if m else None, w_obs.contiguous() if m else None,
                           m, out)
        return out

    def sample_backward(self, x: torch.Tensor, factor: torch.Tensor, idx,
                        record: Optional[Record], pred_factor: torch.Tensor,
                        w_obs: Optional[torch.Tensor], ws_next: torch.Tensor):
        """Backward step of the path sampler: returns (xs_k, ws_k)."""
        ns = x.shape[1]
        factor = factor.contiguous()
        m = 0 if idx is None else int(idx.numel())
        inp = self._sample_input(idx, None, record, pred_factor)
        xs = torch.empty_like(x)
        ws = torch.empty_like(ws_next)
        L.cakf_sample_backward(self.ctx, ns, x.contiguous(), factor if factor.shape[1] else None,
                               max(factor.shape[1], 1), factor.shape[1], inp,
                               w_obs.contiguous() if m else None, ws_next.contiguous(), xs, ws)
        return xs, ws

    def interpolate(self, mean, factor, a_left: float, a_right: float = 1.0,
                    smoothed: bool = False, want_factor: bool = False):
        """Moments at a time between steps k and k+1 from step k's filter moments (mean,
        untruncated factor) and, smoothed, the smoother's current messages (those of
        step k+1).  Returns (mean, marginal variances, factor or None)."""
        factor = factor.contiguous()
        rank = factor.shape[1]
        inp = L.cakf_smooth_input(
            mean=L.ptr(mean), factor=L.ptr(factor) if rank else None, ld=max(rank, 1),
            rank=rank, pred_factor=None, pred_ld=1, pred_rank=0, idx=None, w_obs=None,
            W_obs=None, m=0)
        out_mean = torch.empty(self.n, dtype=torch.float32, device="cuda")
        out_var = torch.empty(self.n, dtype=torch.float32, device="cuda")
        out_fac, ld = None, 0
        if want_factor:
            ld = rank + self.max_rank + self.max_actions
            out_fac = torch.empty((self.n, ld), dtype=torch.float32, device="cuda")
        r = L.cakf_interpolate(self.ctx, inp, a_left, a_right, smoothed, out_mean, out_fac, ld,
                               out_var)
        return out_mean, out_var, (out_fac[:, :r] if want_factor else None)

    def loglik_grad(self, tape, dt: float = 0.0) -> list:
        """d loglik / d(lengthscale, ell_t, signal_var, noise_var) over a recorded run (a
        sequence of cakf_tape_step; see paper_2405_08971_amd.autograd), with ell_t the
        temporal lengthscale at time step dt > 0; dt = 0 gives d / d ou_coeff in place of
        d / d ell_t."""
        return L.cakf_loglik_grad(self.ctx, tape, dt)

    def profile(self, on=True, every=1):
        """on: True (all phases), False (off), or an iterable of phase names; every: time
        only every every-th launch of each timed phase."""
        if on is True:
            mask = -1
        elif not on:
            mask = 0
        else:
            mask = 0
            for name in on:
                mask |= 1 << L.PHASES.index(name)
        L.cakf_profile_enable(self.ctx, mask)
        L.cakf_profile_stride(self.ctx, every)

    def profile_read(self):
        return L.cakf_profile_read(self.ctx)
