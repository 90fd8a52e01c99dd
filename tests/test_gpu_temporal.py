"""GPU parity of the filter with the Matérn-3/2 temporal factor (state: values and scaled
time derivatives at the n points) against the FP64 oracle on the same model
(oracle.temporal): means of both components, marginal variances of all 2n state rows
before and after truncation, and the log-likelihood terms, per step."""
import numpy as np
import pytest

from gpu_common import gpu_run, inputs, rel_mean_err, small_config
from oracle.cakf import run_filter
from oracle.temporal import Matern32TimeModel

pytestmark = pytest.mark.gpu


def _oracle(cfg, X, steps, actions, policy):
    model = Matern32TimeModel(X.astype(np.float64), cfg.nu2, cfg.ell, cfg.sigma_f2, cfg.a,
                              cfg.noise_var, cfg.dist)
    st = [None if s is None else (s[0].astype(np.int64), s[1].astype(np.float64))
          for s in steps]
    acts = None if policy != "given" else [None if a is None else a.astype(np.float64)
                                           for a in actions]
    return run_filter(model, st, cfg.i, cfg.r, policy=policy, actions=acts)


def _check(cfg, recs, gpu, tol):
    for k, (rec, g) in enumerate(zip(recs, gpu), start=1):
        e = dict(
            mean=rel_mean_err(g["mean"], rec.m),
            var=rel_mean_err(cfg.sigma_f2 - g["rowsq"], cfg.sigma_f2 - np.sum(rec.M ** 2, 1)),
            var_trunc=rel_mean_err(cfg.sigma_f2 - g["rowsq_trunc"],
                                   cfg.sigma_f2 - np.sum(rec.M_plus ** 2, 1)),
            value_var=rel_mean_err(g["var"], cfg.sigma_f2 - np.sum(rec.M[:cfg.n] ** 2, 1)),
            loglik=abs(g["loglik"] - rec.loglik) / max(abs(rec.loglik), 1e-300))
        print(f"step {k}: " + " ".join(f"{a}={b:.2e}" for a, b in e.items()), flush=True)
        assert g["mean"].shape[0] == 2 * cfg.n
        assert g["n_actions"] == rec.i_eff
        for key, v in e.items():
            if key == "loglik" and rec.i_eff == 0:
                continue
            assert v <= tol, (k, key, v)


@pytest.mark.parametrize("case,kw,prec,tol", [
    ("sphere_fp32", dict(n=600, m=200, i=8, r=12, T=5), "fp32", 1e-5),
    ("plane_bf16x3", dict(dim=2, nu2=5, ell=0.2, n=400, m=130, i=6, r=10, T=5), "bf16x3",
     1e-4),
])
def test_matern32_time_given_actions_matches_oracle(case, kw, prec, tol):
    cfg = small_config(case, **kw)
    X, steps, actions = inputs(cfg, seed=81, missing_steps=(3,))
    recs = _oracle(cfg, X, steps, actions, "given")
    gpu = gpu_run(cfg, X, steps, actions, "given", prec, temporal="matern32")
    _check(cfg, recs, gpu, tol)


def test_matern32_time_cg_end_to_end():
    cfg = small_config("m32cg", n=700, m=220, i=6, r=15, T=5)
    X, steps, _ = inputs(cfg, seed=82, policy="cg")
    recs = _oracle(cfg, X, steps, None, "cg")
    gpu = gpu_run(cfg, X, steps, [None] * cfg.T, "cg", "fp32", temporal="matern32")
    _check(cfg, recs, gpu, 1e-4)
