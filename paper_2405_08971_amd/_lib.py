"""ctypes binding of libcakf.so (argument marshalling only).

Every function here has the name of the C entry point it calls (include/cakf.h) and
passes device pointers of torch tensors through unchanged; no arithmetic happens here.
The library must have been built (paper_2405_08971_amd/build.py); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcakf.so")

CAKF_OK, CAKF_E_ARG, CAKF_E_HIP, CAKF_E_NOMEM, CAKF_E_STATE, CAKF_E_SOLVER = 0, -1, -2, -3, -4, -5
CAKF_E_SCRATCH = -6
CAKF_STATIC_SCRATCH_BYTES = 32 << 20
CAKF_STATIC_MAX_PATHS = 256
MATERN = {1: 1, 3: 3, 5: 5}
DIST = {"euclid": 0, "geodesic": 1}
PREC = {"fp32": 0, "bf16": 1, "bf16x3": 2}
TEMPORAL = {"ou": 0, "matern32": 1}
POLICY = {"cg": 0, "given": 1, "block": 2}
PHASES = ("sym_tiles", "form_u", "tail", "next_action", "block_product", "gram", "eig",
          "rotate", "predict", "update", "truncate")
_ERR = {CAKF_E_ARG: "invalid argument", CAKF_E_HIP: "HIP runtime error",
        CAKF_E_NOMEM: "device allocation failed", CAKF_E_STATE: "call out of order",
        CAKF_E_SOLVER: "rocBLAS/rocSOLVER error",
        CAKF_E_SCRATCH: "the call needs more than the static scratch array holds"}


class cakf_config(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int), ("dim", ctypes.c_int), ("X", ctypes.c_void_p),
        ("kernel", ctypes.c_int), ("dist", ctypes.c_int),
        ("lengthscale", ctypes.c_double), ("signal_var", ctypes.c_double),
        ("noise_var", ctypes.c_double), ("ou_coeff", ctypes.c_double),
        ("temporal", ctypes.c_int),
        ("max_obs", ctypes.c_int), ("max_actions", ctypes.c_int), ("max_rank", ctypes.c_int),
        ("policy", ctypes.c_int), ("block_actions", ctypes.c_int),
        ("resid_tol", ctypes.c_double),
        ("pivot_tol", ctypes.c_double), ("prec", ctypes.c_int), ("smoother", ctypes.c_int),
        ("sample_paths", ctypes.c_int), ("gradient", ctypes.c_int),
        ("stream", ctypes.c_void_p),
    ]


class cakf_record(ctypes.Structure):
    _fields_ = [
        ("S", ctypes.c_void_p), ("W_obs", ctypes.c_void_p), ("w_obs", ctypes.c_void_p),
        ("chol", ctypes.c_void_p), ("chol_inv", ctypes.c_void_p), ("loglik", ctypes.c_void_p),
        ("n_actions", ctypes.c_void_p),
    ]


class cakf_smooth_input(ctypes.Structure):
    _fields_ = [
        ("mean", ctypes.c_void_p), ("factor", ctypes.c_void_p), ("ld", ctypes.c_int),
        ("rank", ctypes.c_int), ("pred_factor", ctypes.c_void_p), ("pred_ld", ctypes.c_int),
        ("pred_rank", ctypes.c_int), ("idx", ctypes.c_void_p), ("w_obs", ctypes.c_void_p),
        ("W_obs", ctypes.c_void_p), ("m", ctypes.c_int),
    ]


class cakf_sample_input(ctypes.Structure):
    _fields_ = [
        ("idx", ctypes.c_void_p), ("y", ctypes.c_void_p), ("m", ctypes.c_int),
        ("S", ctypes.c_void_p), ("W_obs", ctypes.c_void_p), ("chol_inv", ctypes.c_void_p),
        ("pred_factor", ctypes.c_void_p), ("pred_ld", ctypes.c_int),
        ("pred_rank", ctypes.c_int),
    ]


class cakf_tape_step(ctypes.Structure):
    _fields_ = [
        ("idx", ctypes.c_void_p), ("y", ctypes.c_void_p), ("m", ctypes.c_int),
        ("S", ctypes.c_void_p), ("W_obs", ctypes.c_void_p), ("w_obs", ctypes.c_void_p),
        ("chol", ctypes.c_void_p), ("chol_inv", ctypes.c_void_p),
        ("n_actions", ctypes.c_void_p), ("mean", ctypes.c_void_p),
        ("factor", ctypes.c_void_p), ("ld", ctypes.c_int), ("rank", ctypes.c_int),
        ("rotation", ctypes.c_void_p), ("rank_full", ctypes.c_int),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libcakf.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python paper_2405_08971_amd/build.py`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        sigs = {
            "cakf_create": (i, [ctypes.POINTER(cakf_config), ctypes.POINTER(vp)]),
            "cakf_destroy": (None, [vp]),
            "cakf_reset": (i, [vp]),
            "cakf_state": (i, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp),
                               ctypes.POINTER(i), ctypes.POINTER(i)]),
            "cakf_copy_state": (i, [vp, vp, vp, i]),
            "cakf_set_state": (i, [vp, vp, vp, i, i]),
            "cakf_predict": (i, [vp]),
            "cakf_update": (i, [vp, vp, vp, i, vp, ctypes.POINTER(cakf_record)]),
            "cakf_truncate": (i, [vp, vp]),
            "cakf_step": (i, [vp, vp, vp, i, vp, ctypes.POINTER(cakf_record)]),
            "cakf_marginal_var": (i, [vp, vp, i, vp]),
            "cakf_diagnostics": (i, [vp, ctypes.POINTER(i), ctypes.POINTER(i),
                                     ctypes.POINTER(i)]),
            "cakf_loglik": (i, [vp, ctypes.POINTER(d), ctypes.POINTER(i)]),
            "cakf_smooth_begin": (i, [vp, vp, vp, vp, i]),
            "cakf_smooth_step": (i, [vp, ctypes.POINTER(cakf_smooth_input), vp, vp, i, vp,
                                     ctypes.POINTER(i)]),
            "cakf_smooth": (i, [vp, i, ctypes.POINTER(cakf_smooth_input), vp, vp]),
            "cakf_interpolate": (i, [vp, ctypes.POINTER(cakf_smooth_input), d, d, i, vp, vp,
                                     i, vp, ctypes.POINTER(i)]),
            "cakf_sample_forward": (i, [vp, i, vp, vp, vp, ctypes.POINTER(cakf_sample_input),
                                        vp, vp]),
            "cakf_sample_forward_static": (i, [vp, i, vp, vp, vp,
                                               ctypes.POINTER(cakf_sample_input), vp, vp]),
            "cakf_sample_lift": (i, [vp, i, vp, vp, i, vp]),
            "cakf_sample_backward": (i, [vp, i, vp, vp, i, i,
                                         ctypes.POINTER(cakf_sample_input), vp, vp, vp, vp]),
            "cakf_loglik_grad": (i, [vp, i, ctypes.POINTER(cakf_tape_step), d,
                                     ctypes.POINTER(d)]),
            "cakf_profile_enable": (i, [vp, i]),
            "cakf_profile_stride": (i, [vp, i]),
            "cakf_profile_read": (i, [vp, ctypes.POINTER(d), ctypes.POINTER(i)]),
            "cakf_profile_rates": (i, [ctypes.POINTER(d)]),
        }
        for name, (res, args) in sigs.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc: int, what: str) -> None:
    if rc != CAKF_OK:
        raise RuntimeError(f"{what} failed: {_ERR.get(rc, rc)} ({rc})")


def ptr(t) -> int:
    """Device pointer of a torch tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libcakf takes device tensors")
    if not t.is_contiguous():
        raise ValueError("libcakf takes contiguous tensors")
    return t.data_ptr()


def stream_handle(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


# --- one wrapper per entry point ------------------------------------------------------
def cakf_create(cfg: cakf_config) -> int:
    h = ctypes.c_void_p()
    check(lib().cakf_create(ctypes.byref(cfg), ctypes.byref(h)), "cakf_create")
    return h.value


def cakf_destroy(ctx: int) -> None:
    lib().cakf_destroy(ctx)


def cakf_reset(ctx: int) -> None:
    check(lib().cakf_reset(ctx), "cakf_reset")


def cakf_state(ctx: int):
    mean, factor = ctypes.c_void_p(), ctypes.c_void_p()
    ld, rank = ctypes.c_int(), ctypes.c_int()
    check(lib().cakf_state(ctx, ctypes.byref(mean), ctypes.byref(factor), ctypes.byref(ld),
                           ctypes.byref(rank)), "cakf_state")
    return mean.value, factor.value, ld.value, rank.value


def cakf_copy_state(ctx: int, mean, factor, ld: int) -> None:
    check(lib().cakf_copy_state(ctx, ptr(mean), ptr(factor), ld), "cakf_copy_state")


def cakf_set_state(ctx: int, mean, factor, ld: int, rank: int) -> None:
    check(lib().cakf_set_state(ctx, ptr(mean), ptr(factor), ld, rank), "cakf_set_state")


def cakf_predict(ctx: int) -> None:
    check(lib().cakf_predict(ctx), "cakf_predict")


def cakf_update(ctx: int, idx, y, m: int, actions=None, rec: cakf_record = None) -> None:
    check(lib().cakf_update(ctx, ptr(idx), ptr(y), m, ptr(actions),
                            ctypes.byref(rec) if rec is not None else None), "cakf_update")


def cakf_truncate(ctx: int, rotation=None) -> None:
    check(lib().cakf_truncate(ctx, ptr(rotation)), "cakf_truncate")


def cakf_step(ctx: int, idx, y, m: int, actions=None, rec: cakf_record = None) -> None:
    check(lib().cakf_step(ctx, ptr(idx), ptr(y), m, ptr(actions),
                          ctypes.byref(rec) if rec is not None else None), "cakf_step")


def cakf_marginal_var(ctx: int, rows, count: int, out) -> None:
    check(lib().cakf_marginal_var(ctx, ptr(rows), count, ptr(out)), "cakf_marginal_var")


def cakf_diagnostics(ctx: int):
    dr, nf, bi = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    check(lib().cakf_diagnostics(ctx, ctypes.byref(dr), ctypes.byref(nf), ctypes.byref(bi)),
          "cakf_diagnostics")
    return dr.value, nf.value, bi.value


def cakf_profile_enable(ctx: int, on: int) -> None:
    check(lib().cakf_profile_enable(ctx, int(on)), "cakf_profile_enable")


def cakf_profile_stride(ctx: int, every: int) -> None:
    check(lib().cakf_profile_stride(ctx, int(every)), "cakf_profile_stride")


def cakf_profile_read(ctx: int):
    """{phase: (total_ms, launches)}; resets the counters."""
    n = len(PHASES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int * n)()
    check(lib().cakf_profile_read(ctx, ms, cnt), "cakf_profile_read")
    return {PHASES[k]: (ms[k], cnt[k]) for k in range(n)}


def cakf_smooth_begin(ctx: int, idx, w_obs, W_obs, m: int) -> None:
    check(lib().cakf_smooth_begin(ctx, ptr(idx), ptr(w_obs), ptr(W_obs), m), "cakf_smooth_begin")


def cakf_smooth_step(ctx: int, inp: cakf_smooth_input, mean_out=None, factor_out=None,
                     ld_out: int = 0, var_out=None) -> int:
    rank = ctypes.c_int()
    check(lib().cakf_smooth_step(ctx, ctypes.byref(inp), ptr(mean_out), ptr(factor_out), ld_out,
                                 ptr(var_out), ctypes.byref(rank)), "cakf_smooth_step")
    return rank.value


def cakf_loglik(ctx: int):
    v, n = ctypes.c_double(), ctypes.c_int()
    check(lib().cakf_loglik(ctx, ctypes.byref(v), ctypes.byref(n)), "cakf_loglik")
    return v.value, n.value


def cakf_loglik_grad(ctx: int, tape, dt: float = 0.0) -> list:
    """tape: a sequence of cakf_tape_step; returns the 4 derivatives (host doubles), the
    second with respect to ell_t when dt > 0, else with respect to the OU coefficient."""
    arr = (cakf_tape_step * len(tape))(*tape)
    g = (ctypes.c_double * 4)()
    check(lib().cakf_loglik_grad(ctx, len(tape), arr, dt, g), "cakf_loglik_grad")
    return list(g)


def cakf_sample_forward(ctx: int, ns: int, x_prev, q, e, inp: cakf_sample_input, x_out,
                        w_obs_out) -> None:
    check(lib().cakf_sample_forward(ctx, ns, ptr(x_prev), ptr(q), ptr(e), ctypes.byref(inp),
                                    ptr(x_out), ptr(w_obs_out)), "cakf_sample_forward")


def cakf_sample_forward_static(ctx: int, ns: int, x_prev, q, e, inp: cakf_sample_input,
                               x_out, w_obs_out) -> None:
    check(lib().cakf_sample_forward_static(ctx, ns, ptr(x_prev), ptr(q), ptr(e),
                                           ctypes.byref(inp), ptr(x_out), ptr(w_obs_out)),
          "cakf_sample_forward_static")


def cakf_sample_lift(ctx: int, ns: int, idx, w_obs, m: int, ws_out) -> None:
    check(lib().cakf_sample_lift(ctx, ns, ptr(idx), ptr(w_obs), m, ptr(ws_out)),
          "cakf_sample_lift")


def cakf_sample_backward(ctx: int, ns: int, x, factor, ld: int, rank: int,
                         inp: cakf_sample_input, w_obs, ws_next, xs_out, ws_out) -> None:
    check(lib().cakf_sample_backward(ctx, ns, ptr(x), ptr(factor), ld, rank, ctypes.byref(inp),
                                     ptr(w_obs), ptr(ws_next), ptr(xs_out), ptr(ws_out)),
          "cakf_sample_backward")


def cakf_interpolate(ctx: int, inp: cakf_smooth_input, a_left: float, a_right: float,
                     smoothed: bool, mean_out=None, factor_out=None, ld_out: int = 0,
                     var_out=None) -> int:
    rank = ctypes.c_int()
    check(lib().cakf_interpolate(ctx, ctypes.byref(inp), a_left, a_right, 1 if smoothed else 0,
                                 ptr(mean_out), ptr(factor_out), ld_out, ptr(var_out),
                                 ctypes.byref(rank)), "cakf_interpolate")
    return rank.value


def cakf_smooth(ctx: int, steps, mean_out=None, var_out=None) -> None:
    """steps: a sequence of cakf_smooth_input, k = 1..T."""
    arr = (cakf_smooth_input * len(steps))(*steps)
    check(lib().cakf_smooth(ctx, len(steps), arr, ptr(mean_out), ptr(var_out)), "cakf_smooth")


def cakf_profile_rates() -> list:
    """Lane operations per second of v_exp_f32, v_sqrt_f32 and v_fma_f32 on the current
    device (measured by the library's probe kernels)."""
    out = (ctypes.c_double * 3)()
    check(lib().cakf_profile_rates(out), "cakf_profile_rates")
    return list(out)
