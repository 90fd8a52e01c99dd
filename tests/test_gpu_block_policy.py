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


def test_block_policy_work_precision_against_the_exact_filter():
    """Work-precision study: the error of the GPU filter (final step, posterior mean and
    marginal variance) against the exact Kalman filter, for the CG policy and the
    block-residual policy, as the action budget i grows.  The rank cap holds every
    column (no truncation), so the projection is the only approximation.  Work is counted
    in kernel-matrix entries over the observed points per update: the CG loop evaluates
    half of the symmetric m x m matrix per action, a block round the whole matrix once
    for its b actions.  Both errors must fall as the budget grows."""
    from oracle.kalman import kalman_filter
    from oracle import matern

    budgets = (8, 16, 32, 64)
    cfg0 = small_config("wp", dim=2, nu2=3, ell=0.2, n=1024, m=256, T=4, noise_var=0.01,
                        i=max(budgets), r=256)
    X, steps, _ = inputs(cfg0, seed=15, policy="cg")
    X64 = X.astype(np.float64)
    Sigma = matern.gram(X64, X64, cfg0.nu2, cfg0.ell, cfg0.sigma_f2)
    obs = []
    for item in steps:
        idx, y = item
        H = np.zeros((idx.size, cfg0.n))
        H[np.arange(idx.size), idx] = 1.0
        obs.append((H, cfg0.noise_var * np.eye(idx.size), y.astype(np.float64)))
    exact = kalman_filter(Sigma, cfg0.a, obs)[-1]
    ex_m, ex_v = exact["m"], np.diag(exact["P"])

    rows = []
    for policy in ("cg", ("block", 4), ("block", 8)):
        errs = []
        for i in budgets:
            cfg = small_config("wp", dim=2, nu2=3, ell=0.2, n=1024, m=256, T=4,
                               noise_var=0.01, i=i, r=256)
            g = gpu_run(cfg, X, steps, [None] * cfg.T, policy, "fp32")[-1]
            # the computation-aware variance never falls below the exact one (Sec. 3.2:
            # incomplete computation adds uncertainty)
            assert np.min(g["var"] - ex_v) >= -1e-4 * cfg.sigma_f2, (policy, i)
            e_m = rel_mean_err(g["mean"], ex_m)
            e_v = rel_mean_err(g["var"], ex_v)
            b = 1 if policy == "cg" else policy[1]
            entries = (i * cfg.m * cfg.m // 2) if policy == "cg" else \
                (-(-i // b)) * cfg.m * cfg.m
            errs.append((e_m, e_v))
            rows.append((str(policy), i, entries, e_m, e_v))
        for (m_a, v_a), (m_b, v_b) in zip(errs, errs[1:]):
            assert m_b <= 1.1 * m_a and v_b <= 1.1 * v_a, (policy, errs)
        assert errs[-1][0] < 0.5 * errs[0][0] and errs[-1][1] < 0.5 * errs[0][1], (policy, errs)
    print("\npolicy        i   kernel entries / update   mean rel err   var rel err")
    for pol, i, ent, e_m, e_v in rows:
        print(f"{pol:12s} {i:3d}   {ent:22d}   {e_m:12.3e}   {e_v:11.3e}", flush=True)
