"""The C ABI: libcakf.so loads and exports every function include/cakf.h declares, and
the ctypes structures match the header's field order.  No GPU calls are made."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cakf.h")
LIB = os.path.join(ROOT, "paper_2405_08971_amd", "libcakf.so")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void)\s+(cakf_\w+)\s*\(", text, re.M)))


def header_struct_fields(name):
    text = open(HEADER).read()
    body = re.search(r"typedef struct \{((?:(?!typedef struct).)*?)\}\s*" + name + ";", text,
                     re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        pieces = decl.replace("*", " ").split(",")
        fields += [piece.split()[-1] for piece in pieces]
    return fields


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcakf.so not built")
def test_library_exports_every_declared_function():
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_structs_follow_the_header():
    from paper_2405_08971_amd import _lib
    for cname, pyname in [("cakf_config", _lib.cakf_config), ("cakf_record", _lib.cakf_record),
                          ("cakf_smooth_input", _lib.cakf_smooth_input),
                          ("cakf_tape_step", _lib.cakf_tape_step),
                          ("cakf_sample_input", _lib.cakf_sample_input)]:
        assert [f[0] for f in pyname._fields_] == header_struct_fields(cname), cname


def test_binding_wraps_every_declared_function():
    from paper_2405_08971_amd import _lib
    for n in declared_functions():
        assert hasattr(_lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcakf.so not built")
def test_residual_tolerance_is_rejected_without_cg_actions():
    """cakf_create validates its arguments before any device call: the residual-tolerance
    stop is defined for residual (CG) actions only, so GIVEN and BLOCK with resid_tol != 0
    are argument errors (for CG the value passes validation)."""
    from paper_2405_08971_amd import _lib
    lib = ctypes.CDLL(LIB)
    dummy = ctypes.c_float(0.0)
    for policy, expect_arg_error in (("given", True), ("block", True)):
        cfg = _lib.cakf_config(n=16, dim=3, X=ctypes.cast(ctypes.pointer(dummy), ctypes.c_void_p),
                               kernel=3, dist=0, lengthscale=0.3, signal_var=1.0,
                               noise_var=0.05, ou_coeff=0.8, temporal=0, max_obs=8,
                               max_actions=4, max_rank=4, policy=_lib.POLICY[policy],
                               block_actions=2, resid_tol=1e-3, pivot_tol=1e-10, prec=0)
        ctx = ctypes.c_void_p()
        rc = lib.cakf_create(ctypes.byref(cfg), ctypes.byref(ctx))
        assert rc == _lib.CAKF_E_ARG, (policy, rc)
        assert not ctx.value
