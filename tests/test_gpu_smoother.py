"""GPU parity of the computation-aware RTS smoother (Alg. 3) against the FP64 oracle:
smoothed means and marginal variances per step, same seeded inputs and actions, with and
without truncation."""
import numpy as np
import pytest

from gpu_common import gpu_run_smoother, inputs, oracle_run, rel_mean_err, small_config
from oracle.caks import run_smoother

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case,kw", [
    ("no_trunc", dict(n=500, m=150, i=6, r=1000, T=4)),
    ("trunc", dict(n=600, m=200, i=8, r=12, T=5)),
    ("plane_missing", dict(dim=2, nu2=5, ell=0.2, n=400, m=130, i=6, r=10, T=5)),
])
def test_smoother_matches_oracle(case, kw):
    cfg = small_config(case, **kw)
    X, steps, actions = inputs(cfg, seed=21, missing_steps=(3,) if case == "plane_missing" else ())
    model, recs = oracle_run(cfg, X, steps, actions, "given")
    sm = run_smoother(model, recs, cfg.r)
    gpu = gpu_run_smoother(cfg, X, steps, actions, "given", "fp32")
    for k in range(cfg.T):
        em = rel_mean_err(gpu[k][0], sm[k].m)
        ev = rel_mean_err(gpu[k][1], sm[k].marginal_var(cfg.sigma_f2))
        print(f"step {k + 1}: mean {em:.2e} var {ev:.2e}", flush=True)
        assert em <= 1e-5 and ev <= 1e-5, (k, em, ev)


def test_smoother_bf16x3_and_cg_policy():
    cfg = small_config("cgs", n=500, m=180, i=6, r=10, T=4)
    X, steps, _ = inputs(cfg, seed=22, policy="cg")
    model, recs = oracle_run(cfg, X, steps, None, "cg")
    sm = run_smoother(model, recs, cfg.r)
    gpu = gpu_run_smoother(cfg, X, steps, [None] * cfg.T, "cg", "bf16x3")
    for k in range(cfg.T):
        em = rel_mean_err(gpu[k][0], sm[k].m)
        ev = rel_mean_err(gpu[k][1], sm[k].marginal_var(cfg.sigma_f2))
        print(f"step {k + 1}: mean {em:.2e} var {ev:.2e}", flush=True)
        assert em <= 1e-4 and ev <= 1e-4, (k, em, ev)
