"""Forward-mode derivative of the replayed projected log-likelihood (oracle, FP64).

The likelihood is the sum over steps of the projected prediction-error terms l_k (see
oracle.cakf), differentiated with the actions S_k and the truncation rotations V_r,k
frozen at the values recorded in a base run (see oracle.grad).  This module carries,
next to every quantity of the replayed filter, its derivative with respect to each of

    theta = (ell, ell_t, sigma_f2, noise_var)

and applies the chain rule to each step as the filter takes it:

  predict (Alg. 1, OU prior)   m^- = a m,  M^- = a M^+,  a = exp(-dt / ell_t)
  projected Gram (Alg. 2)      C = S^T Ghat S,  Ghat = H Sigma H^T - Mo Mo^T + noise I,
                               Mo = H M^-,  Sigma = sigma_f2 K(X, X; ell)
  Cholesky form (App. B)       C = L L^T,  alpha = L^{-1} S^T r0,  r0 = y - H m^-,
                               W = S L^{-T},  w = W alpha
  log-likelihood               l_k = -1/2 (i log 2 pi + 2 sum_j log L_jj
                                           - log det S^T S + alpha^T alpha)
  block product (Alg. 2)       Y = Sigma H^T [W w] - M^- (Mo^T [W w]),
                               m = m^- + Y_w,  M = [M^-, Y_W]
  truncate (Sec. 3.2)          M^+ = M V_r  (V_r frozen)

The derivative of the Cholesky factor is dL = L Phi(L^{-1} dC L^{-T}), Phi taking the
lower triangle with the diagonal halved (the differential of C = L L^T solved for a
lower-triangular dL).  Everything is dense and FP64, for small instances.

Test infrastructure only; not part of the product path.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

from . import matern
from .cakf import LOG2PI, Model, StepRecord
from .grad import model_at

NPAR = 4


def _phi(X: np.ndarray) -> np.ndarray:
    out = np.tril(X)
    out[np.diag_indices_from(out)] *= 0.5
    return out


def replay_tangent(base: Model, dt: float, theta: Sequence[float], steps,
                   recs: List[StepRecord]) -> Tuple[float, np.ndarray]:
    """Replayed log-likelihood at theta and its derivative in each parameter.

    recs supplies the frozen actions (S[:, :i_eff]) and rotations (V_r) of a base run;
    steps[k-1] = (idx_k, y_k) or None as for run_filter."""
    ell, ell_t, s2, nv = (float(t) for t in theta)
    model = model_at(base, dt, theta)
    a = model.a
    X = model.X
    n = X.shape[0]
    K = matern.gram(X, X, model.nu2, ell, 1.0, model.dist)
    dK = matern.gram_dell(X, X, model.nu2, ell, 1.0, model.dist)
    Sigma = s2 * K
    dSigma = [s2 * dK, np.zeros_like(K), K, np.zeros_like(K)]
    da = [0.0, a * dt / ell_t ** 2, 0.0, 0.0]
    dnoise = [0.0, 0.0, 0.0, 1.0]

    m = np.zeros(n)
    M = np.zeros((n, 0))
    dm = [np.zeros(n) for _ in range(NPAR)]
    dM = [np.zeros((n, 0)) for _ in range(NPAR)]
    total = 0.0
    grad = np.zeros(NPAR)
    for k, item in enumerate(steps):
        rec = recs[k]
        m_pred = a * m
        M_pred = a * M
        dm_pred = [da[p] * m + a * dm[p] for p in range(NPAR)]
        dM_pred = [da[p] * M + a * dM[p] for p in range(NPAR)]
        if item is None or rec.i_eff == 0:
            m_new, M_new = m_pred, M_pred
            dm_new, dM_new = dm_pred, dM_pred
        else:
            idx, y = item
            idx = np.asarray(idx)
            S = np.asarray(rec.S, np.float64)[:, :rec.i_eff]
            i = S.shape[1]
            mo = idx.size
            r0 = np.asarray(y, np.float64) - m_pred[idx]
            Mo = M_pred[idx]
            G = Sigma[np.ix_(idx, idx)] - Mo @ Mo.T + nv * np.eye(mo)
            C = S.T @ G @ S
            C = 0.5 * (C + C.T)
            L = np.linalg.cholesky(C)
            Linv = np.linalg.inv(L)
            c = S.T @ r0
            alpha = Linv @ c
            _, logdet_s = np.linalg.slogdet(S.T @ S)
            total += -0.5 * (i * LOG2PI + 2.0 * np.sum(np.log(np.diag(L))) - logdet_s
                             + alpha @ alpha)
            W = S @ Linv.T
            w = W @ alpha
            B = np.column_stack([W, w])
            Q = Mo.T @ B
            SigXo = Sigma[:, idx]
            Y = SigXo @ B - M_pred @ Q
            m_new = m_pred + Y[:, -1]
            M_new = np.hstack([M_pred, Y[:, :-1]])
            dm_new, dM_new = [], []
            for p in range(NPAR):
                dMo = dM_pred[p][idx]
                dr0 = -dm_pred[p][idx]
                dG = (dSigma[p][np.ix_(idx, idx)] - dMo @ Mo.T - Mo @ dMo.T
                      + dnoise[p] * np.eye(mo))
                dC = S.T @ dG @ S
                dC = 0.5 * (dC + dC.T)
                dL = L @ _phi(Linv @ dC @ Linv.T)
                dc = S.T @ dr0
                dalpha = Linv @ (dc - dL @ alpha)
                grad[p] += -(np.sum(np.diag(dL) / np.diag(L)) + alpha @ dalpha)
                dW = -W @ (Linv @ dL).T
                dw = dW @ alpha + W @ dalpha
                dB = np.column_stack([dW, dw])
                dQ = dMo.T @ B + Mo.T @ dB
                dY = (dSigma[p][:, idx] @ B + SigXo @ dB - dM_pred[p] @ Q - M_pred @ dQ)
                dm_new.append(dm_pred[p] + dY[:, -1])
                dM_new.append(np.hstack([dM_pred[p], dY[:, :-1]]))
        if rec.V_r is not None:
            Vr = np.asarray(rec.V_r, np.float64)
            M = M_new @ Vr
            dM = [d @ Vr for d in dM_new]
        else:
            M = M_new
            dM = dM_new
        m, dm = m_new, dm_new
    return float(total), grad
