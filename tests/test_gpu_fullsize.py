"""Full-size checks in the benchmark's launch configuration (n = 65536 sphere points,
Matern-5/2, m = 16384, i = 128 CG actions, r = 512), with the BF16X3 block product and
with the FP32 one.

The FP64 oracle cannot run whole steps at this size, so the GPU's outputs are checked
against properties that hold at any size, each evaluated in FP64 with the oracle's
covariance function on the same inputs:

* the projected Gram matrix: L L^T z = S^T Ghat (S z) for a random probe z, with
  Ghat = Sigma_oo + noise_var I at the first step (one FP64 matrix-free product);
* the block product on sampled state rows p: the new factor columns and the mean
  increment equal sigma_f2 K(x_p, Xo) [W w] - M^-[p] (Mo^T [W w]) (Alg. 2);
* the truncation keeps the r leading directions of M M^T: the columns of M^+ are
  mutually orthogonal with squared norms equal to the r largest eigenvalues of M^T M
  (host LAPACK on the FP64 Gram of the GPU's untruncated factor);
* marginal variances lie in [0, sigma_f2]; no action is dropped; the CG actions are
  numerically independent.  (In FP32 the recomputed residuals lose orthogonality in
  proportion to eps_32 |r0| / |rho_j|, which reaches 1e-1 once the residual has fallen by
  1e-5; the method needs only independent actions, since log det S^T S is factored
  separately.  Orthogonality itself is checked at small sizes.)
"""
import numpy as np
import pytest

from oracle import matern
from paper_2405_08971_amd.workload import CONFIGS, Workload

pytestmark = pytest.mark.gpu


def _rel(x, ref):
    return float(np.mean(np.abs(np.asarray(x) - ref)) / np.mean(np.abs(ref)))


def check_truncation(M, Mplus, r):
    """M: untruncated factor (device, FP32), Mplus: truncated (device).  The squared
    column norms of M^+ are the r largest eigenvalues of M^T M and its columns are
    mutually orthogonal (FP64 Grams of the device factors, host eigenvalues)."""
    G = (M.double().T @ M.double()).cpu().numpy()
    lam = np.sort(np.linalg.eigvalsh(0.5 * (G + G.T)))[::-1][:r]
    Gp = (Mplus.double().T @ Mplus.double()).cpu().numpy()
    d = np.sort(np.diag(Gp))[::-1]
    e_val = float(np.max(np.abs(d - lam)) / lam[0])
    off = Gp - np.diag(np.diag(Gp))
    e_off = float(np.max(np.abs(off)) / lam[0])
    kept = float(np.sum(d) / np.sum(lam))
    print(f"  truncation: eigenvalue err {e_val:.2e}, off-diagonal {e_off:.2e}, "
          f"kept trace ratio {kept:.8f}", flush=True)
    assert e_val < 1e-5 and e_off < 1e-5 and abs(kept - 1.0) < 1e-6


@pytest.mark.parametrize("prec,tol_bp", [("bf16x3", 1e-3), ("fp32", 1e-4)])
def test_full_size_step_properties(prec, tol_bp):
    import torch
    from paper_2405_08971_amd.filter import CAKF, Record

    cfg = CONFIGS["sphere_n65536"]
    wl = Workload(cfg, seed=0)
    X32 = wl.X.astype(np.float32)
    X64 = X32.astype(np.float64)
    f = CAKF(torch.from_numpy(X32).cuda(), nu2=cfg.nu2, lengthscale=cfg.ell,
             signal_var=cfg.sigma_f2, noise_var=cfg.noise_var, ou_coeff=cfg.a,
             max_obs=cfg.m, max_actions=cfg.i, max_rank=cfg.r, policy="cg", prec=prec)
    rng = np.random.default_rng(0)
    check_steps = (1, 6)
    for k in range(1, 7):
        idx, y = wl.step(k)
        idx32, y32 = idx.astype(np.int32), y.astype(np.float32)
        f.predict()
        mean_pred, M_pred = f.state()
        rec = Record(cfg.m, cfg.i)
        f.update(torch.from_numpy(idx32).cuda(), torch.from_numpy(y32).cuda(), record=rec)
        mean, M = f.state()
        var = f.marginal_var().cpu().numpy()
        torch.cuda.synchronize()
        n_act = int(rec.n_actions.item())
        print(f"step {k}: actions {n_act}, rank {M.shape[1]}, loglik {rec.loglik.item():.6e}",
              flush=True)
        assert n_act == cfg.i
        assert np.isfinite(rec.loglik.item())
        assert var.min() >= -1e-4 and var.max() <= cfg.sigma_f2 + 1e-4, (var.min(), var.max())
        S = rec.S.cpu().numpy().astype(np.float64)
        Sn = S / np.linalg.norm(S, axis=0)
        ortho = np.abs(Sn.T @ Sn - np.eye(cfg.i)).max()
        smin = np.linalg.svd(Sn, compute_uv=False).min()
        print(f"  normalised actions: max |S^T S - I| {ortho:.2e}, sigma_min {smin:.3f}",
              flush=True)
        assert smin > 0.5
        if k not in check_steps:
            f.truncate()
            continue
        W = rec.W_obs.cpu().numpy().astype(np.float64)
        w = rec.w_obs.cpu().numpy().astype(np.float64)
        L = rec.chol.cpu().numpy()
        Xo = X64[idx]
        if k == 1:
            # L L^T z = S^T Ghat S z, Ghat = Sigma_oo + noise I (no downdate yet)
            z = rng.standard_normal(cfg.i)
            v = S @ z
            Gv = (matern.gram_matmul(Xo, Xo, v, cfg.nu2, cfg.ell, cfg.sigma_f2)
                  + cfg.noise_var * v)
            lhs = L @ (L.T @ z)
            e = _rel(lhs, S.T @ Gv)
            print(f"  Gram probe rel err {e:.2e}", flush=True)
            assert e < 1e-4
        # block product on sampled rows
        rows = np.sort(rng.choice(cfg.n, 256, replace=False))
        B = np.column_stack([W, w])
        Mp = M_pred.cpu().numpy().astype(np.float64)
        ref = matern.gram(X64[rows], Xo, cfg.nu2, cfg.ell, cfg.sigma_f2) @ B
        if Mp.shape[1]:
            Q = Mp[idx].T @ B
            ref -= Mp[rows] @ Q
        Mn = M.cpu().numpy().astype(np.float64)
        got = np.column_stack([Mn[rows, Mp.shape[1]:Mp.shape[1] + cfg.i],
                               mean.cpu().numpy()[rows] - mean_pred.cpu().numpy()[rows]])
        e = _rel(got, ref)
        print(f"  block product rel err on sampled rows {e:.2e}", flush=True)
        assert e < tol_bp
        f.truncate()
        if M.shape[1] > cfg.r:
            check_truncation(M, f.state()[1], cfg.r)
    f.close()
