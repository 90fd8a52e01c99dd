"""The no-allocation entry point cakf_sample_forward_static (the sampler's forward step on
the library's static scratch array) against cakf_sample_forward on the same inputs.

Two calls in a row, the second with fewer paths and fewer observations, so that the scratch
holds the first call's larger contents when the second starts.  The static variant runs on
a context created without sampler workspace.  Both entry points run the same kernels in the
same order, so the results agree to the last bit; the assertion allows the FP32 bar's
rounding headroom all the same.  The observation count (1100, two 512-point ranges) makes
the block product take its observation-split path, whose partials also live in the scratch.
"""
import numpy as np
import pytest

from gpu_common import inputs, rel_max_err, rel_mean_err, small_config

pytestmark = pytest.mark.gpu


def _context(cfg, X, prec, sample_paths):
    import torch
    from paper_2405_08971_amd.filter import CAKF

    return CAKF(torch.from_numpy(X).to("cuda"), nu2=cfg.nu2,
                dist="geodesic" if cfg.dist == 1 else "euclid", lengthscale=cfg.ell,
                signal_var=cfg.sigma_f2, noise_var=cfg.noise_var, ou_coeff=cfg.a,
                max_obs=cfg.m, max_actions=cfg.i, max_rank=cfg.r, policy="given", prec=prec,
                sample_paths=sample_paths)


def _records(f, cfg, steps, actions):
    """Filter run keeping, per step, the predictive factor and the update's record."""
    import torch
    from paper_2405_08971_amd.filter import Record

    out = []
    for k, (idx, y) in enumerate(steps):
        f.predict()
        Mp = f.state()[1].clone()
        idx_d = torch.from_numpy(idx).to("cuda")
        y_d = torch.from_numpy(y).to("cuda")
        rec = Record(len(idx), cfg.i)
        f.update(idx_d, y_d, torch.from_numpy(actions[k]).to("cuda"), rec)
        f.truncate()
        out.append((Mp, idx_d, y_d, rec))
    return out


def _row_subset(rec, m2, cfg):
    """The first m2 observations of a record (row slices of the row-major m x i arrays)."""
    from paper_2405_08971_amd.filter import Record

    sub = Record(m2, cfg.i)
    sub.S.copy_(rec.S[:m2])
    sub.W_obs.copy_(rec.W_obs[:m2])
    sub.chol_inv.copy_(rec.chol_inv)
    return sub


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_static_scratch_forward_matches_the_allocating_entry(prec):
    import torch

    cfg = small_config("noalloc", n=2000, m=1100, i=6, r=10, T=3)
    X, steps, actions = inputs(cfg, seed=61)
    f = _context(cfg, X, prec, sample_paths=8)        # regular entry point's workspace
    g = _context(cfg, X, prec, sample_paths=0)        # no sampler workspace at all
    fwd = _records(f, cfg, steps, actions)
    rng = np.random.default_rng(62)
    calls = [(2, 8, cfg.m), (1, 3, 700)]               # (step, paths, observations)
    for k, ns, m in calls:
        Mp, idx, y, rec = fwd[k]
        if m < cfg.m:
            idx, y, rec = idx[:m].contiguous(), y[:m].contiguous(), _row_subset(rec, m, cfg)
        x_prev = torch.from_numpy(rng.standard_normal((cfg.n, ns)).astype(np.float32)).cuda()
        q = torch.from_numpy(0.3 * rng.standard_normal((cfg.n, ns)).astype(np.float32)).cuda()
        e = torch.from_numpy(rng.standard_normal((m, ns)).astype(np.float32)).cuda()
        print(f"prec {prec}: step {k + 1}, {ns} paths, {m} observations, "
              f"predictive rank {Mp.shape[1]}", flush=True)
        x_ref, w_ref = f.sample_forward(x_prev, q, e, idx, y, rec, Mp)
        x_st, w_st = g.sample_forward(x_prev, q, e, idx, y, rec, Mp, static_scratch=True)
        torch.cuda.synchronize()
        for name, got, ref in (("x", x_st, x_ref), ("w_obs", w_st, w_ref)):
            got64, ref64 = got.double().cpu().numpy(), ref.double().cpu().numpy()
            em, ex = rel_mean_err(got64, ref64), rel_max_err(got64, ref64)
            print(f"  {name}: bitwise {torch.equal(got, ref)}, rel mean {em:.1e}, "
                  f"rel max {ex:.1e}", flush=True)
            assert em <= 1e-6 and ex <= 1e-5, (name, em, ex)
    f.close()
    g.close()


def test_static_scratch_rejects_what_does_not_fit():
    """A layout beyond the array is CAKF_E_SCRATCH before anything is enqueued (the
    buffers passed are of full size all the same); more paths than the limit is an
    argument error."""
    import torch
    from paper_2405_08971_amd import _lib as L

    cfg = small_config("noalloc_big", n=40000, m=200, i=2, r=4, T=1)
    X, steps, actions = inputs(cfg, seed=63)
    f = _context(cfg, X, "fp32", sample_paths=0)
    (Mp, idx, y, rec), = _records(f, cfg, steps, actions)
    ns = 256                                           # n x 256 FP32 alone is 41 MB
    cols = L.CAKF_STATIC_MAX_PATHS + 1                 # room for both calls' path counts
    x_prev = torch.zeros((cfg.n, cols), device="cuda")
    q = torch.zeros_like(x_prev)
    e = torch.zeros((cfg.m, cols), device="cuda")
    inp = f._sample_input(idx, y, rec, Mp)
    x = torch.empty_like(x_prev)
    w = torch.empty((cfg.m, cols), device="cuda")
    rc = L.lib().cakf_sample_forward_static(f.ctx, ns, L.ptr(x_prev), L.ptr(q), L.ptr(e),
                                            ctypes_byref(inp), L.ptr(x), L.ptr(w))
    assert rc == L.CAKF_E_SCRATCH, rc
    rc = L.lib().cakf_sample_forward_static(f.ctx, L.CAKF_STATIC_MAX_PATHS + 1, L.ptr(x_prev),
                                            L.ptr(q), L.ptr(e), ctypes_byref(inp), L.ptr(x),
                                            L.ptr(w))
    assert rc == L.CAKF_E_ARG, rc
    torch.cuda.synchronize()
    f.close()


def ctypes_byref(obj):
    import ctypes
    return ctypes.byref(obj)
