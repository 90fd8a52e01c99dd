"""Derivative of the projected log-likelihood (oracle, FP64).

The paper names evidence maximisation as future work and defines no likelihood
(Sec. 8).  The likelihood used here is the sum over steps of the projected
prediction-error terms l_k (see oracle.cakf).  Its derivative is taken with the
actions S_k and the truncation rotations V_r,k frozen at the values recorded in a run
at the base parameters, which makes the replayed filter a smooth function of

    theta = (ell, ell_t, sigma_f2, noise_var)

(spatial lengthscale, temporal lengthscale through a = exp(-dt / ell_t), signal
variance, observation noise variance).  The replay uses the iterative update with the
recorded actions, whose search directions are S L^{-T} with C = L L^T, so a frozen
rotation acts on the same factor columns as in the base run.

The oracle derivative is a central difference of the replayed FP64 likelihood.

Test infrastructure only; not part of the product path.
"""
from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np

from .cakf import Model, StepRecord, run_filter, total_loglik

PARAMS = ("ell", "ell_t", "sigma_f2", "noise_var")


def model_at(base: Model, dt: float, theta: Sequence[float]) -> Model:
    ell, ell_t, s2, nv = (float(t) for t in theta)
    return Model(base.X, base.nu2, ell, s2, math.exp(-dt / ell_t), nv, base.dist)


def replay_loglik(base: Model, dt: float, theta, steps, recs: List[StepRecord],
                  r_cap: int, form: str = "iterative") -> float:
    """Log-likelihood at theta with the actions and rotations of recs frozen.  form
    "batch" replays with the batch update and the Cholesky square root (the same factor
    columns S L^{-T} as the iterative form, App. B), which costs one projected-Gram
    product per step instead of three per action."""
    model = model_at(base, dt, theta)
    actions = [None if r.S is None else r.S for r in recs]
    rotations = [r.V_r for r in recs]
    max_i = max([0] + [r.i_eff for r in recs])
    out = run_filter(model, steps, max_actions=max_i, r_cap=r_cap, policy="given",
                     actions=actions, pivot_tol=-np.inf, rotations=rotations, form=form,
                     lsqrt="chol")
    return total_loglik(out)


def fd_gradient(base: Model, dt: float, theta, steps, recs, r_cap: int,
                rel_step: float = 1e-5, form: str = "iterative") -> np.ndarray:
    """Central differences of replay_loglik in each parameter (relative step)."""
    theta = np.asarray(theta, np.float64)
    g = np.zeros(theta.size)
    for j in range(theta.size):
        h = rel_step * abs(theta[j])
        tp = theta.copy()
        tm = theta.copy()
        tp[j] += h
        tm[j] -= h
        g[j] = (replay_loglik(base, dt, tp, steps, recs, r_cap, form)
                - replay_loglik(base, dt, tm, steps, recs, r_cap, form)) / (2.0 * h)
    return g
