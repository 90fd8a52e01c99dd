"""Temporal interpolation of the computation-aware filter and smoother (oracle, FP64).

The corollary on temporal interpolation (App. C) gives the belief at a time t between
two steps from the neighbouring steps alone.  With steps at t_k = k dt and the OU
transition A(t, s) = exp(-(t - s) / ell_t) = a^((t - s) / dt):

  filter,   t_k <= t < t_{k+1}:  m(t) = A(t, t_k) m_k,   M(t) = A(t, t_k) M_k,
                                 P(t) = Sigma - M(t) M(t)^T
  smoother, t_k <= t < t_{k+1}:  ms(t) = m(t) + P(t) A(t_{k+1}, t) ws_{k+1}
                                 Ms(t) = (M(t), P(t) A(t_{k+1}, t) Ws_{k+1})

Before the first step the filter belief is the prior (m = 0, no downdate); after the
last step the smoother's belief is the filter's.  Reading: M_k is the untruncated
factor of step k, the one the smoother uses in P_k; ws, Ws are the smoother's messages
(oracle.caks).

Test infrastructure only; not part of the product path.
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np

from .caks import SmoothRecord
from .cakf import Model, StepRecord


def interpolate(model: Model, recs: List[StepRecord], sm: List[SmoothRecord], t: float,
                dt: float, smoothed: bool) -> Tuple[np.ndarray, np.ndarray]:
    """(mean, factor) of the filter (smoothed=False) or smoother belief at time t, with
    step k (1-based) at time k dt."""
    a = model.a
    T = len(recs)
    k = int(math.floor(t / dt + 1e-12))          # t_k <= t < t_{k+1}
    k = min(k, T)
    if k >= 1:
        g = a ** ((t - k * dt) / dt)              # A(t, t_k)
        m_t = g * recs[k - 1].m
        M_t = g * recs[k - 1].M
    else:
        m_t = np.zeros(model.n)
        M_t = np.zeros((model.n, 0))
    if not smoothed or k >= T:
        return m_t, M_t
    h = a ** (((k + 1) * dt - t) / dt)            # A(t_{k+1}, t)
    nxt = sm[k]                                   # messages of step k+1
    B = h * np.column_stack([nxt.ws, nxt.Ws])
    PB = model.cov_matmul(None, None, B) - M_t @ (M_t.T @ B)
    return m_t + PB[:, 0], np.hstack([M_t, PB[:, 1:]])
