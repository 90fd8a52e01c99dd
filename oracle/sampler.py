"""Joint sample paths of the computation-aware filter and smoother (oracle, FP64).

The CAKF/CAKS sampler (App. C, Alg. "CAKF/CAKS Sampler") draws paths by pushing prior
draws through the filter's gains, in the manner of Matheron's rule:

  forward, k = 1..T    x^-_k = A x_{k-1} + q_{k-1},          q ~ N(0, Q)
                       w_k   = W_k Vc_k^T (S_k^T y_k - S_k^T H_k x^-_k - eps_k),
                                                              eps_k ~ N(0, S_k^T Lambda S_k)
                       x_k   = x^-_k + P^-_k w_k
  backward, k = T-1..1 ws_T  = w_T
                       xs_k  = x_k + P_k A^T ws_{k+1}
                       ws_k  = w_k + (I - W_k W_k^T P^-_k) A^T ws_{k+1}

with W_k = H_k^T S_k Vc_k, Vc_k Vc_k^T = (S_k^T Ghat_k S_k)^{-1} (Vc_k = L_k^{-T} from the
Cholesky factor, as in the filter), P^-_k = Sigma - M^-_k (M^-_k)^T and P_k = Sigma -
M_k M_k^T with the untruncated filter factor.  The returned path is xs_k (xs_T = x_T).

Readings: the printed return statement pairs x_k with the message of the same index;
the smoother it samples from (Alg. 3, and the RTS smoother in downdate form) pairs
P_k A^T with the message of step k+1, which is what is used here.  The random draws are
inputs: x0 ~ N(0, Sigma) and q_k ~ N(0, (1 - a^2) Sigma) (the OU prior, Lemma C.1), and
e_k ~ N(0, I_m) per observation, from which eps_k = S_k^T (sigma e_k) has the
distribution N(0, S_k^T Lambda S_k) with Lambda = sigma^2 I.  Several paths are the
columns of the arrays.

Test infrastructure only; not part of the product path.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from .cakf import Model, StepRecord


def _lift(n: int, idx, V: np.ndarray) -> np.ndarray:
    """H^T V for a row selector H."""
    out = np.zeros((n,) + V.shape[1:])
    out[np.asarray(idx)] = V
    return out


def _gain_parts(model: Model, rec: StepRecord):
    """(S, Vc) of a recorded update: the kept actions and L^{-T} of S^T Ghat S."""
    S = np.asarray(rec.S, np.float64)[:, :rec.i_eff]
    idx = np.asarray(rec.idx)
    Mo = rec.M_pred[idx]
    GS = model.cov_matmul(idx, idx, S) - Mo @ (Mo.T @ S) + model.noise_var * S
    C = S.T @ GS
    L = np.linalg.cholesky(0.5 * (C + C.T))
    return S, np.linalg.inv(L).T


def sample_paths(model: Model, steps, recs: List[StepRecord], x0: np.ndarray,
                 q: Sequence[np.ndarray], e: Sequence) -> Tuple[list, list, list]:
    """Sample paths given the records of a filter run (run_filter) and the draws.

    steps[k-1] = (idx_k, y_k) or None; x0 (n, ns); q[k-1] (n, ns) the noise added in the
    prediction of step k; e[k-1] (m_k, ns) or None.  Returns (x, w, xs): the forward
    samples x_k, the messages w_k (n, ns) and the smoothed samples xs_k, k = 1..T."""
    n = model.n
    a = model.a
    sigma = np.sqrt(model.noise_var)
    T = len(recs)
    x_prev = np.asarray(x0, np.float64)
    xs_f, ws_f, Ws_f = [], [], []
    for k in range(T):
        rec = recs[k]
        xm = a * x_prev + np.asarray(q[k], np.float64)
        if steps[k] is None or rec.i_eff == 0:
            w = np.zeros_like(xm)
            W = np.zeros((n, 0))
            x = xm
        else:
            idx, y = steps[k]
            idx = np.asarray(idx)
            S, Vc = _gain_parts(model, rec)
            W = _lift(n, idx, S @ Vc)                                   # H^T S Vc
            eps = S.T @ (sigma * np.asarray(e[k], np.float64))          # S^T Lambda^{1/2} e
            innov = S.T @ np.asarray(y, np.float64)[:, None] - S.T @ xm[idx] - eps
            w = W @ (Vc.T @ innov)
            x = xm + model.cov_matmul(None, None, w) - rec.M_pred @ (rec.M_pred.T @ w)
        xs_f.append(x)
        ws_f.append(w)
        Ws_f.append(W)
        x_prev = x
    xs = [None] * T
    xs[T - 1] = xs_f[T - 1]
    wsn = ws_f[T - 1]
    for k in range(T - 2, -1, -1):
        rec = recs[k]
        Aw = a * wsn
        SAw = model.cov_matmul(None, None, Aw)
        xs[k] = xs_f[k] + SAw - rec.M @ (rec.M.T @ Aw)                   # P_k A^T ws_{k+1}
        Pm = SAw - rec.M_pred @ (rec.M_pred.T @ Aw)                     # P^-_k A^T ws_{k+1}
        W = Ws_f[k]
        wsn = ws_f[k] + Aw - W @ (W.T @ Pm)
    return xs_f, ws_f, xs
