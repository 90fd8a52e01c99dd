"""GPU parity of the block-residual policy (rounds of b actions, the residual at the start
of a round split over fixed contiguous observation groups) against the FP64 oracle's
policy ("block", b), end to end: both sides choose their own actions, so the bar is that
of the CG comparison (the FP32 and FP64 residuals drift apart slowly)."""
import numpy as np
import pytest

from gpu_common import compare, gpu_run, inputs, oracle_run, rel_mean_err, small_config

pytestmark = pytest.mark.gpu

END_TO_END_TOL = 1e-4


def _check(errs, tol):
    for k, e in enumerate(errs, start=1):
        print(f"step {k}: " + " ".join(f"{a}={b}" for a, b in e.items()), flush=True)
    for k, e in enumerate(errs, start=1):
        assert e["n_actions"][0] == e["n_actions"][1], (k, e)
        for key in ("mean", "var", "var_trunc", "MMt", "loglik"):
            if key in e:
                assert e[key] <= tol, (k, key, e)


def _actions_match(recs, gpu, tol):
    """The GPU's own actions against the oracle's, column by column."""
    for rec, g in zip(recs, gpu):
        if rec.S is None:
            continue
        i = rec.i_eff
        for j in range(i):
            err = rel_mean_err(g["S"][:, j], rec.S[:, j])
            assert err <= tol, (j, err)
        assert not np.any(g["S"][:, i:])


# (b, i): full rounds, a ragged last round (12 = 5 + 5 + 2), and b = i (one round)
@pytest.mark.parametrize("b,i", [(4, 8), (5, 12), (6, 6)])
def test_block_policy_fp32_matches_oracle(b, i):
    cfg = small_config(f"blk{b}", n=700, m=230, i=i, r=16, T=5)
    X, steps, _ = inputs(cfg, seed=11, policy="block", missing_steps=(3,))
    probes = np.random.default_rng(2).standard_normal((cfg.n, 3))
    model, recs = oracle_run(cfg, X, steps, None, ("block", b))
    gpu = gpu_run(cfg, X, steps, [None] * cfg.T, ("block", b), "fp32", probes=probes)
    _check(compare(cfg, model, recs, gpu, probes), END_TO_END_TOL)
    _actions_match(recs, gpu, END_TO_END_TOL)


def test_block_policy_with_one_action_per_round_is_cg():
    """b = 1: every action is the full residual, as in the CG policy."""
    cfg = small_config("blk1", n=600, m=200, i=6, r=14, T=4)
    X, steps, _ = inputs(cfg, seed=12, policy="cg")
    model, recs = oracle_run(cfg, X, steps, None, "cg")
    gpu = gpu_run(cfg, X, steps, [None] * cfg.T, ("block", 1), "fp32")
    _check(compare(cfg, model, recs, gpu), END_TO_END_TOL)


def test_block_policy_bf16x3_geodesic_matches_oracle():
    cfg = small_config("blkg", dist=1, nu2=3, n=650, m=300, i=10, r=20, T=4)
    X, steps, _ = inputs(cfg, seed=13, policy="block")
    model, recs = oracle_run(cfg, X, steps, None, ("block", 5))
    gpu = gpu_run(cfg, X, steps, [None] * cfg.T, ("block", 5), "bf16x3")
    _check(compare(cfg, model, recs, gpu), END_TO_END_TOL)


def test_block_policy_more_actions_than_observations():
    """m < max_actions: at most m actions are taken (the last round is cut short)."""
    cfg = small_config("blkfew", n=300, m=7, i=10, r=12, T=3)
    X, steps, _ = inputs(cfg, seed=14, policy="block")
    # the oracle's action budget is the GPU's effective one, min(i, m)
    cfg_o = small_config("blkfew", n=300, m=7, i=7, r=12, T=3)
    model, recs = oracle_run(cfg_o, X, steps, None, ("block", 3))
    gpu = gpu_run(cfg, X, steps, [None] * cfg.T, ("block", 3), "fp32")
    errs = compare(cfg, model, recs, gpu)
    _check(errs, END_TO_END_TOL)
