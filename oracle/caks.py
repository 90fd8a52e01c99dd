"""Computation-aware RTS smoother (Alg. 3), plain FP64 (oracle).

Backward pass over the filter records (k = T-1, ..., 1):

    ms_k  = m_k + P_k A^T ws_{k+1}
    Ms_k  = (M_k, P_k A^T Ws_{k+1})
    ws_k  = w_k + (I - W_k W_k^T P_k^-) A^T ws_{k+1}
    Ws_k  = Truncate((W_k, (I - W_k W_k^T P_k^-) A^T Ws_{k+1}))

with ws_T = w_T, Ws_T = W_T, P_k = Sigma - M_k M_k^T (untruncated filter factor),
P_k^- = Sigma - M_k^- (M_k^-)^T (predictive factor built from the truncated factor of
the previous step), w_k = H_k^T v_k and W_k = H_k^T V_k (the filter's messages, stored
in observation coordinates).  The smoothed covariance is Sigma - Ms_k Ms_k^T.

Test infrastructure only; not part of the product path.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

from .cakf import Model, StepRecord, truncate


@dataclasses.dataclass
class SmoothRecord:
    k: int
    m: np.ndarray
    M: np.ndarray
    ws: np.ndarray
    Ws: np.ndarray

    def marginal_var(self, sigma_f2: float) -> np.ndarray:
        return sigma_f2 - np.sum(self.M * self.M, axis=1)


def _lift(n, idx, V):
    """H^T V for a row selector H: scatter the rows of V to the positions idx."""
    out = np.zeros((n,) + V.shape[1:])
    if idx is not None:
        out[idx] = V
    return out


def run_smoother(model: Model, recs: List[StepRecord], r_cap: int) -> List[SmoothRecord]:
    n = model.n
    a = model.a
    T = len(recs)
    out = [None] * T

    def w_of(rec):
        if rec.idx is None:
            return np.zeros(n), np.zeros((n, 0))
        return _lift(n, rec.idx, rec.w_obs), _lift(n, rec.idx, rec.W_obs)

    def Sigma_mv(V):
        return model.cov_matmul(None, None, V)

    last = recs[T - 1]
    ws, Ws = w_of(last)
    out[T - 1] = SmoothRecord(last.k, last.m, last.M, ws, Ws)
    for k in range(T - 2, -1, -1):
        rec = recs[k]
        B = np.column_stack([ws, Ws])
        AtB = a * B
        SAtB = Sigma_mv(AtB)
        # P_k A^T B with the untruncated filter factor M_k
        PAtB = SAtB - rec.M @ (rec.M.T @ AtB)
        ms = rec.m + PAtB[:, 0]
        Ms = np.hstack([rec.M, PAtB[:, 1:]])
        wk, Wk = w_of(rec)
        # (I - W_k W_k^T P_k^-) A^T B
        Pm = SAtB - rec.M_pred @ (rec.M_pred.T @ AtB)
        proj = AtB - Wk @ (Wk.T @ Pm)
        ws = wk + proj[:, 0]
        Ws, _, _ = truncate(np.hstack([Wk, proj[:, 1:]]), r_cap)
        out[k] = SmoothRecord(rec.k, ms, Ms, ws, Ws)
    return out
