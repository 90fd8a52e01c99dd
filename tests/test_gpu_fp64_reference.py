"""The n = 65536 workload against its FP64 reference (the update of Alg. 2 and Truncate of
Sec. 3.2 at full size).

tests/golden/sphere_n65536_fp64.npz holds the FP64 oracle's results for the first six
steps of the workload (65536 Fibonacci-sphere points, chordal Matern-5/2 with lengthscale
0.3, m = 16384 observations per step, i = 128 Gaussian actions from the input generator,
rank cap r = 512, noise variance 0.05) on its seeded 2048-point subset, written by
tests/golden/make_sphere_n65536_fp64.py from the oracle alone (batch form with the given
actions; the inputs rounded to FP32 as the GPU receives them).  The rank reaches 640 at
step 5, so steps 5 and 6 include the truncation.

The GPU runs the same steps through the C ABI with the same actions, in FP32 and with
the BF16X3 block product, and every result is compared element by element on the subset:
the filter mean, the marginal variance of the untruncated factor and of the truncated
one, and the log-likelihood term.  Bars: relative mean error 1e-5 (FP32) and 1e-3
(BF16X3), and the largest single entry within MAX_FACTOR times that bar.
"""
import os

import numpy as np
import pytest

from gpu_common import MAX_FACTOR, rel_max_err, rel_mean_err
from paper_2405_08971_amd.workload import CONFIGS, Workload

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "sphere_n65536_fp64.npz")


def run_gpu(prec):
    import torch
    from paper_2405_08971_amd.filter import CAKF, Record

    ref = np.load(GOLDEN)
    steps = ref["mean"].shape[0]
    cfg = CONFIGS["sphere_n65536"]
    wl = Workload(cfg, seed=0)
    sub = wl.subset(ref["subset"].size)
    assert np.array_equal(sub, ref["subset"])
    rows = torch.from_numpy(sub.astype(np.int32)).cuda()
    f = CAKF(torch.from_numpy(wl.X.astype(np.float32)).cuda(), nu2=cfg.nu2,
             lengthscale=cfg.ell, signal_var=cfg.sigma_f2, noise_var=cfg.noise_var,
             ou_coeff=cfg.a, max_obs=cfg.m, max_actions=cfg.i, max_rank=cfg.r,
             policy="given", prec=prec)
    out = dict(mean=[], var=[], var_trunc=[], loglik=[], n_actions=[])
    for k in range(1, steps + 1):
        idx, y = wl.step(k)
        S = wl.actions(k).astype(np.float32)
        rec = Record(cfg.m, cfg.i)
        f.predict()
        f.update(torch.from_numpy(idx.astype(np.int32)).cuda(),
                 torch.from_numpy(y.astype(np.float32)).cuda(), torch.from_numpy(S).cuda(), rec)
        mean, _ = f.state()
        out["mean"].append(mean[rows.long()].double().cpu().numpy())
        out["var"].append(f.marginal_var(rows).double().cpu().numpy())
        f.truncate()
        out["var_trunc"].append(f.marginal_var(rows).double().cpu().numpy())
        torch.cuda.synchronize()
        out["loglik"].append(float(rec.loglik.item()))
        out["n_actions"].append(int(rec.n_actions.item()))
    f.close()
    return ref, out


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16x3", 1e-3)])
def test_sphere_n65536_against_fp64_reference(prec, tol):
    ref, gpu = run_gpu(prec)
    worst = {}
    for k in range(ref["mean"].shape[0]):
        errs = {}
        for key in ("mean", "var", "var_trunc"):
            errs[key] = rel_mean_err(gpu[key][k], ref[key][k])
            errs[key + "_max"] = rel_max_err(gpu[key][k], ref[key][k])
        errs["loglik"] = abs(gpu["loglik"][k] - ref["loglik"][k]) / abs(ref["loglik"][k])
        print(f"{prec} step {k + 1}: " + " ".join(f"{a}={b:.2e}" for a, b in errs.items()),
              flush=True)
        assert gpu["n_actions"][k] == int(ref["i_eff"][k])
        for key, v in errs.items():
            worst[key] = max(worst.get(key, 0.0), v)
    print(f"{prec} worst over steps: {worst}", flush=True)
    for key in ("mean", "var", "var_trunc", "loglik"):
        assert worst[key] <= tol, (key, worst)
    for key in ("mean_max", "var_max", "var_trunc_max"):
        assert worst[key] <= MAX_FACTOR * tol, (key, worst)
