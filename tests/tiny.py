"""Tiny seeded problems for the oracle pin tests (inputs only), and the reader of the
hand-worked fixtures under golden/."""
from __future__ import annotations

import math
import os

import numpy as np

from oracle import kalman
from oracle.cakf import Model


def tiny_problem(seed=0, n=30, T=4, m=8, nu2=3, ell=0.3, sigma_f2=1.3, a=0.8,
                 noise_var=0.05, missing_steps=(), dim=2):
    rng = np.random.default_rng(seed)
    X = rng.random((n, dim))
    if dim == 3:
        X /= np.linalg.norm(X, axis=1, keepdims=True)
    model = Model(X, nu2, ell, sigma_f2, a, noise_var)
    steps = []
    for k in range(1, T + 1):
        if k in missing_steps:
            steps.append(None)
            continue
        idx = rng.choice(n, m, replace=False)
        y = rng.standard_normal(m)
        steps.append((idx, y))
    return model, steps


def dense_obs(model, steps, actions=None):
    """(H, R, y) per step for the dense references; projected by S_k if given."""
    out = []
    for k, item in enumerate(steps):
        if item is None:
            out.append(None)
            continue
        idx, y = item
        H = kalman.row_selector(idx, model.n)
        R = model.noise_var * np.eye(len(idx))
        if actions is not None:
            S = actions[k]
            out.append((S.T @ H, S.T @ R @ S, S.T @ y))
        else:
            out.append((H, R, y))
    return out


GOLDEN_DIR = os.path.join(os.path.dirname(__file__), "golden")


def load_golden(name):
    """Values of a golden/ fixture: lines "name = expression", evaluated in order with
    e = exp(-1), log and pi (and the names defined above them) in scope."""
    env = {"e": math.exp(-1.0), "log": math.log, "pi": math.pi}
    vals = {}
    with open(os.path.join(GOLDEN_DIR, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, expr = (t.strip() for t in line.split("=", 1))
            vals[key] = eval(expr, {"__builtins__": {}}, {**env, **vals})
    return vals
