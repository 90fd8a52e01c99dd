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


def test_smoother_bf16x3_more_than_8_column_tiles():
    """Given actions with r = 300: the smoothed factor reaches the b = r + 1 = 301 columns of
    [ws Ws], whose 300 BF16X3 columns (ws, column 0, is summed in FP32) take two launches of
    five 32-column tiles; the truncating steps take the Gram of their kept block as known."""
    cfg = small_config("sm_wide", n=1200, m=330, i=110, r=300, T=5)
    X, steps, actions = inputs(cfg, seed=24)
    model, recs = oracle_run(cfg, X, steps, actions, "given")
    sm = run_smoother(model, recs, cfg.r)
    gpu = gpu_run_smoother(cfg, X, steps, actions, "given", "bf16x3")
    for k in range(cfg.T):
        em = rel_mean_err(gpu[k][0], sm[k].m)
        ev = rel_mean_err(gpu[k][1], sm[k].marginal_var(cfg.sigma_f2))
        print(f"step {k + 1}: mean {em:.2e} var {ev:.2e}", flush=True)
        assert em <= 1e-4 and ev <= 1e-4, (k, em, ev)


def test_whole_backward_pass_entry_point():
    """cakf_smooth (all steps in one call) against the oracle smoother."""
    import torch
    from paper_2405_08971_amd.filter import CAKF, Record
    cfg = small_config("whole", n=500, m=160, i=6, r=10, T=5)
    X, steps, actions = inputs(cfg, seed=23, missing_steps=(2,))
    model, recs = oracle_run(cfg, X, steps, actions, "given")
    sm = run_smoother(model, recs, cfg.r)
    dev = "cuda"
    f = CAKF(torch.from_numpy(X).to(dev), nu2=cfg.nu2, lengthscale=cfg.ell,
             signal_var=cfg.sigma_f2, noise_var=cfg.noise_var, ou_coeff=cfg.a,
             max_obs=cfg.m, max_actions=cfg.i, max_rank=cfg.r, policy="given", smoother=True)
    fwd = []
    for k, item in enumerate(steps):
        f.predict()
        _, Mp = f.state()
        rec, idx = None, None
        if item is None:
            f.update(None, None)
        else:
            idx = torch.from_numpy(item[0]).to(dev)
            rec = Record(len(item[0]), cfg.i)
            f.update(idx, torch.from_numpy(item[1]).to(dev),
                     torch.from_numpy(actions[k]).to(dev), rec)
        mean, M = f.state()
        fwd.append((mean, M, Mp, idx, rec))
        f.truncate()
    means, var = f.smooth(fwd)
    means, var = means.cpu().numpy(), var.cpu().numpy()
    f.close()
    for k in range(cfg.T):
        em = rel_mean_err(means[k], sm[k].m)
        ev = rel_mean_err(var[k], sm[k].marginal_var(cfg.sigma_f2))
        print(f"step {k + 1}: mean {em:.2e} var {ev:.2e}", flush=True)
        assert em <= 1e-5 and ev <= 1e-5, (k, em, ev)
