"""Matern covariance functions used by the paper's priors (oracle, FP64).

The paper uses Matern(nu) kernels with nu in {1/2, 3/2, 5/2} for space and time
(Sec. 6 "Model"; App. D.2.1-D.2.3) but never prints their formulas.  This module writes
out the standard half-integer closed forms with u = d / ell:

    nu = 1/2 :  s2 * exp(-u)
    nu = 3/2 :  s2 * (1 + sqrt(3) u) exp(-sqrt(3) u)
    nu = 5/2 :  s2 * (1 + sqrt(5) u + 5 u^2 / 3) exp(-sqrt(5) u)

and their derivatives with respect to the lengthscale.  Distances are Euclidean (for
points on the unit sphere this is the chordal/extrinsic distance of App. D.2.3) or
great-circle: the angle between the two position vectors, atan2(|a x b|, <a, b>),
which equals arccos(<a, b>) for unit vectors and stays exact when the inputs carry
rounding in their length.

Test infrastructure only; not part of the product path.
"""
from __future__ import annotations

import numpy as np

EUCLID = 0
GEODESIC = 1


def distances(A: np.ndarray, B: np.ndarray, dist: int = EUCLID) -> np.ndarray:
    """Pairwise distances between the rows of A (p x d) and B (q x d), FP64."""
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    if dist == EUCLID:
        diff = A[:, None, :] - B[None, :, :]
        return np.sqrt(np.sum(diff * diff, axis=-1))
    if dist == GEODESIC:
        ax, ay, az = (A[:, k][:, None] for k in range(3))
        bx, by, bz = (B[:, k][None, :] for k in range(3))
        cross = np.sqrt((ay * bz - az * by) ** 2 + (az * bx - ax * bz) ** 2
                        + (ax * by - ay * bx) ** 2)
        return np.arctan2(cross, A @ B.T)
    raise ValueError("unknown distance")


def matern(nu2: int, d: np.ndarray, ell: float, s2: float = 1.0) -> np.ndarray:
    """Half-integer Matern covariance at distances d; nu2 = 2*nu in {1, 3, 5}."""
    u = np.asarray(d, np.float64) / ell
    if nu2 == 1:
        return s2 * np.exp(-u)
    if nu2 == 3:
        c = np.sqrt(3.0) * u
        return s2 * (1.0 + c) * np.exp(-c)
    if nu2 == 5:
        c = np.sqrt(5.0) * u
        return s2 * (1.0 + c + c * c / 3.0) * np.exp(-c)
    raise ValueError("nu2 must be 1, 3 or 5")


def matern_dell(nu2: int, d: np.ndarray, ell: float, s2: float = 1.0) -> np.ndarray:
    """Derivative of matern(nu2, d, ell, s2) with respect to ell."""
    u = np.asarray(d, np.float64) / ell
    if nu2 == 1:
        return s2 * (u / ell) * np.exp(-u)
    if nu2 == 3:
        c = np.sqrt(3.0) * u
        return s2 * (c * c / ell) * np.exp(-c)
    if nu2 == 5:
        c = np.sqrt(5.0) * u
        return s2 * (c * c / (3.0 * ell)) * (1.0 + c) * np.exp(-c)
    raise ValueError("nu2 must be 1, 3 or 5")


def gram(A, B, nu2, ell, s2=1.0, dist=EUCLID) -> np.ndarray:
    """Dense covariance matrix k(A, B)."""
    return matern(nu2, distances(A, B, dist), ell, s2)


def gram_dell(A, B, nu2, ell, s2=1.0, dist=EUCLID) -> np.ndarray:
    return matern_dell(nu2, distances(A, B, dist), ell, s2)


def _threads() -> int:
    """Worker threads for gram_matmul: ORACLE_THREADS, else every host core."""
    import os
    env = os.environ.get("ORACLE_THREADS")
    if env:
        return max(1, int(env))
    return max(1, os.cpu_count() or 1)


def gram_matmul(A, B, V, nu2, ell, s2=1.0, dist=EUCLID, rows_per_chunk=512) -> np.ndarray:
    """k(A, B) @ V.  The covariance rows are formed a slab of rows of A at a time only
    to bound memory: each output row is the plain sum over B.  Large products spread
    the slabs over a pool of threads (NumPy releases the interpreter lock inside its
    array operations); every slab is computed exactly as it would be alone, and the
    matrix library runs single-threaded inside the pool."""
    V = np.asarray(V, np.float64)
    out = np.empty((A.shape[0],) + V.shape[1:], np.float64)
    slabs = [(p0, min(A.shape[0], p0 + rows_per_chunk))
             for p0 in range(0, A.shape[0], rows_per_chunk)]

    def one(sl):
        p0, p1 = sl
        out[p0:p1] = gram(A[p0:p1], B, nu2, ell, s2, dist) @ V

    nthreads = min(_threads(), len(slabs))
    if nthreads <= 1 or A.shape[0] * B.shape[0] < (1 << 22):
        for sl in slabs:
            one(sl)
        return out
    from concurrent.futures import ThreadPoolExecutor
    try:
        from threadpoolctl import threadpool_limits
        limit = threadpool_limits(1)
    except Exception:                       # threadpoolctl missing: BLAS keeps its threads
        limit = None
    try:
        with ThreadPoolExecutor(nthreads) as ex:
            list(ex.map(one, slabs))
    finally:
        if limit is not None:
            limit.restore_original_limits()
    return out
