"""GPU parity: the HIP library against the FP64 oracle on the same seeded inputs.

The bar (relative mean error mean|x - x64| / mean|x64| per result and per step) is 1e-5
for the FP32 path and 1e-3 for the BF16 block product, and every single entry must stay
within MAX_FACTOR times that bar on the scale of the result (max|x - x64| / mean|x64|);
the number of kept actions must match exactly.  Given-action runs make the actions inputs, so both sides condition on
the same S; CG runs are compared end to end (the FP32 and FP64 Krylov bases drift apart
slowly, so their bar is looser and stated per test).
"""
import numpy as np
import pytest

from gpu_common import MAX_FACTOR, compare, gpu_run, inputs, oracle_run, small_config

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5


def _check(errs, tol, tol_ll=None):
    tol_ll = tol if tol_ll is None else tol_ll
    for k, e in enumerate(errs, start=1):
        print(f"step {k}: " + " ".join(f"{a}={b}" for a, b in e.items()), flush=True)
    for k, e in enumerate(errs, start=1):
        assert e["n_actions"][0] == e["n_actions"][1], (k, e)
        assert e["mean"] <= tol, (k, e)
        assert e["var"] <= tol, (k, e)
        assert e["var_trunc"] <= tol, (k, e)
        for key in ("mean_max", "var_max", "var_trunc_max"):
            assert e[key] <= MAX_FACTOR * tol, (k, key, e)
        if "MMt" in e:
            assert e["MMt"] <= tol, (k, e)
        if e["n_actions"][1] > 0:
            assert e["loglik"] <= tol_ll, (k, e)


CASES = {
    # name: config overrides (all ragged: m is not a multiple of the 128 tile)
    "sphere_m32": dict(),
    "plane_m52": dict(dim=2, nu2=5, ell=0.2, n=500, m=190, i=12, r=30, T=5, noise_var=0.01),
    "sphere_m12_geodesic": dict(nu2=1, dist=1, n=700, m=257, i=6, r=14, T=5),
    "sphere_m32_geodesic": dict(dist=1, n=600, m=129, i=10, r=16, T=4),
    "plane_m12": dict(dim=2, nu2=1, ell=0.25, n=450, m=200, i=8, r=18, T=4),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_given_actions_fp32_matches_oracle(case):
    cfg = small_config(case, **CASES[case])
    X, steps, actions = inputs(cfg, seed=1, missing_steps=(3,) if cfg.T >= 5 else ())
    model, recs = oracle_run(cfg, X, steps, actions, "given")
    probes = np.random.default_rng(0).standard_normal((cfg.n, 3))
    gpu = gpu_run(cfg, X, steps, actions, "given", "fp32", probes=probes)
    _check(compare(cfg, model, recs, gpu, probes), FP32_TOL)


@pytest.mark.parametrize("prec,tol", [("fp32", FP32_TOL), ("bf16x3", 1e-4)])
def test_more_than_160_block_columns(prec, tol):
    """i + 1 = 171 columns of [W w]: the block product runs two column blocks (160 + 11)."""
    cfg = small_config("wide", dim=2, nu2=3, ell=0.25, n=800, m=600, i=170, r=20, T=2)
    X, steps, actions = inputs(cfg, seed=12)
    model, recs = oracle_run(cfg, X, steps, actions, "given")
    probes = np.random.default_rng(3).standard_normal((cfg.n, 3))
    gpu = gpu_run(cfg, X, steps, actions, "given", prec, probes=probes)
    _check(compare(cfg, model, recs, gpu, probes), tol)


def test_truncation_with_the_kept_columns_gram_block_known():
    """r = 128 (two full 64-column Gram tiles), i = 64: after the first truncation (step 3)
    the kept columns are orthogonal with the kept eigenvalues as squared norms, so the
    truncations of steps 4 and 6 take that block of M^T M as diag(a^2 lam) (a^4 across the
    missing step 5) and compute only the products with the appended columns.  The oracle
    forms every Gram entry in FP64."""
    cfg = small_config("orth", n=2000, m=500, i=64, r=128, T=6)
    X, steps, actions = inputs(cfg, seed=21, missing_steps=(5,))
    model, recs = oracle_run(cfg, X, steps, actions, "given")
    probes = np.random.default_rng(5).standard_normal((cfg.n, 3))
    gpu = gpu_run(cfg, X, steps, actions, "given", "fp32", probes=probes)
    _check(compare(cfg, model, recs, gpu, probes), FP32_TOL)


def test_cg_fp32_matches_oracle_end_to_end():
    cfg = small_config("cg", n=700, m=220, i=6, r=15, T=5)
    X, steps, _ = inputs(cfg, seed=2, policy="cg")
    model, recs = oracle_run(cfg, X, steps, None, "cg")
    gpu = gpu_run(cfg, X, steps, [None] * cfg.T, "cg", "fp32")
    errs = compare(cfg, model, recs, gpu)
    _check(errs, 1e-4)


def test_cg_actions_are_orthogonal_residuals():
    """Validity of the GPU's own CG actions (any size): normalised residual actions are
    orthonormal to FP32 accuracy, as Lanczos vectors are."""
    cfg = small_config("cgo", n=900, m=400, i=16, r=32, T=2)
    X, steps, _ = inputs(cfg, seed=3, policy="cg")
    gpu = gpu_run(cfg, X, steps, [None] * cfg.T, "cg", "fp32")
    for g in gpu:
        S = g["S"][:, :g["n_actions"]].astype(np.float64)
        Sn = S / np.linalg.norm(S, axis=0)
        G = Sn.T @ Sn
        assert np.abs(G - np.eye(G.shape[0])).max() < 1e-3, np.abs(G - np.eye(G.shape[0])).max()


def test_fewer_observations_than_actions_and_single_observation():
    cfg = small_config("few", n=300, m=5, i=8, r=12, T=4)
    X, steps, actions = inputs(cfg, seed=4)
    # the action budget exceeds m: only m actions can be kept
    acts = [a[:, :8] for a in actions]
    model, recs = oracle_run(cfg, X, steps, acts, "given")
    gpu = gpu_run(cfg, X, steps, acts, "given", "fp32")
    _check(compare(cfg, model, recs, gpu), FP32_TOL)
    cfg1 = small_config("one", n=200, m=1, i=1, r=3, T=4)
    X, steps, actions = inputs(cfg1, seed=5)
    model, recs = oracle_run(cfg1, X, steps, actions, "given")
    gpu = gpu_run(cfg1, X, steps, actions, "given", "fp32")
    _check(compare(cfg1, model, recs, gpu), FP32_TOL)


def test_breakdown_drops_dependent_actions_like_the_oracle():
    cfg = small_config("brk", n=400, m=150, i=6, r=12, T=3)
    X, steps, actions = inputs(cfg, seed=6)
    # action 3 (0-based) is a combination of actions 0 and 1 at every step
    for a in actions:
        a[:, 3] = a[:, 0] - 2.0 * a[:, 1]
    model, recs = oracle_run(cfg, X, steps, actions, "given", pivot_tol=1e-6)
    gpu = gpu_run(cfg, X, steps, actions, "given", "fp32", pivot_tol=1e-6)
    errs = compare(cfg, model, recs, gpu)
    assert all(e["n_actions"] == (3, 3) for e in errs), errs
    _check(errs, FP32_TOL)


def test_deterministic_bitwise():
    cfg = small_config("det", n=600, m=270, i=8, r=16, T=3)
    X, steps, _ = inputs(cfg, seed=7, policy="cg")
    a = gpu_run(cfg, X, steps, [None] * cfg.T, "cg", "fp32")
    b = gpu_run(cfg, X, steps, [None] * cfg.T, "cg", "fp32")
    for ga, gb in zip(a, b):
        assert np.array_equal(ga["mean"], gb["mean"])
        assert np.array_equal(ga["var_trunc"], gb["var_trunc"])
        assert ga["loglik"] == gb["loglik"]


# Bars for the BF16 block product.  The split form (Kh Bh + Kl Bh + Kh Bl) is the mode
# that meets the 1e-3 requirement of the BF16 path, and is held to 1e-4 here (measured
# about 1e-5).  Plain BF16 rounding of the kernel tile and of [W w] leaves 2e-3 to 7e-3
# on these cases: it does NOT meet 1e-3 and is held only to 1e-2.
PREC_TOL = {"bf16": 1e-2, "bf16x3": 1e-4}


# Euclidean Matern-3/2 and -5/2 take the squared distances of the kernel tile from FP32
# MFMA; Matern-1/2 and the great-circle distance evaluate the tile on the VALU.
@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
@pytest.mark.parametrize("case", ["sphere_m32", "plane_m52", "plane_m12", "sphere_m12_geodesic"])
def test_given_actions_bf16_block_product_matches_oracle(case, prec):
    cfg = small_config(case, **CASES[case])
    X, steps, actions = inputs(cfg, seed=8, missing_steps=(3,) if cfg.T >= 5 else ())
    model, recs = oracle_run(cfg, X, steps, actions, "given")
    probes = np.random.default_rng(1).standard_normal((cfg.n, 3))
    gpu = gpu_run(cfg, X, steps, actions, "given", prec, probes=probes)
    _check(compare(cfg, model, recs, gpu, probes), PREC_TOL[prec])


def test_loglik_entry_point_sums_the_step_terms():
    import torch
    from paper_2405_08971_amd.filter import CAKF
    from oracle.cakf import total_loglik
    cfg = small_config("ll", n=500, m=160, i=6, r=10, T=4)
    X, steps, actions = inputs(cfg, seed=9, missing_steps=(2,))
    model, recs = oracle_run(cfg, X, steps, actions, "given")
    f = CAKF(torch.from_numpy(X).cuda(), nu2=cfg.nu2, lengthscale=cfg.ell,
             signal_var=cfg.sigma_f2, noise_var=cfg.noise_var, ou_coeff=cfg.a,
             max_obs=cfg.m, max_actions=cfg.i, max_rank=cfg.r, policy="given")
    for k, item in enumerate(steps):
        if item is None:
            f.step(None, None)
        else:
            f.step(torch.from_numpy(item[0]).cuda(), torch.from_numpy(item[1]).cuda(),
                   torch.from_numpy(actions[k]).cuda())
    value, nsteps = f.loglik()
    f.close()
    ref = total_loglik(recs)
    assert nsteps == 3
    assert abs(value - ref) <= 1e-5 * abs(ref), (value, ref)
