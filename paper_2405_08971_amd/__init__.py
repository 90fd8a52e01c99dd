"""MI355X computation-aware Kalman filter (arXiv 2405.08971): the update step's hot path
as a HIP library (libcakf.so, C ABI in include/cakf.h) with a thin ctypes binding."""

__all__ = ["CAKF", "Record", "workload"]


def __getattr__(name):
    if name in ("CAKF", "Record"):
        from . import filter as _f
        return getattr(_f, name)
    if name == "workload":
        from . import workload as _w
        return _w
    raise AttributeError(name)
