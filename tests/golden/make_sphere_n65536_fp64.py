"""Write the FP64 reference of the n = 65536 workload's first steps.

Runs the FP64 oracle (the batch update of Alg. 2 with given actions, then Truncate of
Sec. 3.2) on the first STEPS steps of the n = 65536 sphere workload (65536
Fibonacci-sphere points, Matern-5/2 chordal kernel with lengthscale 0.3, m = 16384
observations per step, i = 128 actions, rank cap r = 512, noise variance 0.05) with
the input generator's Gaussian actions, and stores on its seeded 2048-point subset:

  mean       m_k after the update of step k                        (STEPS x 2048)
  var        diag(Sigma - M_k M_k^T), untruncated factor              (STEPS x 2048)
  var_trunc  diag(Sigma - M_k^+ M_k^+^T), after the truncation         (STEPS x 2048)
  loglik     the projected log-likelihood term l_k                    (STEPS)

Inputs (points, observations, actions) are rounded to FP32 first, exactly as the GPU
receives them, so that a comparison measures the arithmetic alone.  The rank reaches
640 at step 5, where truncation starts.

Usage:  python tests/golden/make_sphere_n65536_fp64.py
Only oracle/ and the input generator are called.  Runtime: a few minutes on 8 cores.
"""
from __future__ import annotations

import os
import subprocess
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.cakf import Model, run_filter          # noqa: E402
from paper_2405_08971_amd.workload import CONFIGS, Workload   # noqa: E402

NAME = "sphere_n65536"
STEPS = 6
SEED = 0
SUBSET = 2048
OUT = os.path.join(HERE, "sphere_n65536_fp64.npz")


def git_sha() -> str:
    try:
        sha = subprocess.run(["git", "rev-parse", "HEAD"], cwd=ROOT, capture_output=True,
                             text=True).stdout.strip()
        dirty = subprocess.run(["git", "status", "--porcelain", "oracle"], cwd=ROOT,
                               capture_output=True, text=True).stdout.strip()
        return sha + ("+dirty-oracle" if dirty else "")
    except Exception:
        return "unknown"


def main():
    cfg = CONFIGS[NAME]
    wl = Workload(cfg, seed=SEED)
    X = wl.X.astype(np.float32).astype(np.float64)
    steps, actions = [], []
    for k in range(1, STEPS + 1):
        idx, y = wl.step(k)
        steps.append((idx.astype(np.int64), y.astype(np.float32).astype(np.float64)))
        actions.append(wl.actions(k).astype(np.float32).astype(np.float64))
    sub = wl.subset(SUBSET)
    model = Model(X, cfg.nu2, cfg.ell, cfg.sigma_f2, cfg.a, cfg.noise_var, cfg.dist)
    t0 = time.perf_counter()
    recs = run_filter(model, steps, cfg.i, cfg.r, policy="given", actions=actions,
                      form="batch")
    dt = time.perf_counter() - t0
    mean = np.stack([r.m[sub] for r in recs])
    var = np.stack([r.marginal_var(cfg.sigma_f2)[sub] for r in recs])
    var_trunc = np.stack([cfg.sigma_f2 - np.sum(r.M_plus[sub] ** 2, axis=1) for r in recs])
    loglik = np.array([r.loglik for r in recs])
    i_eff = np.array([r.i_eff for r in recs])
    meta = (f"workload={NAME} seed={SEED} steps={STEPS} subset={SUBSET} policy=given "
            f"form=batch inputs=fp32-rounded oracle_sha={git_sha()} "
            f"command='python tests/golden/make_sphere_n65536_fp64.py' "
            f"oracle_seconds={dt:.0f}")
    np.savez_compressed(OUT, subset=sub, mean=mean, var=var, var_trunc=var_trunc,
                        loglik=loglik, i_eff=i_eff, meta=np.array(meta))
    print(meta)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
