"""Separable spatiotemporal prior with a Matérn-3/2 temporal factor (oracle, FP64).

A temporal kernel whose spectral density is rational (the remark on converting
spatiotemporal GP priors, App. C) makes the separable prior a space-time separable
Gauss-Markov process (Lemma C.1).  For the Matérn-3/2 kernel
k_t(tau) = (1 + lam |tau|) exp(-lam |tau|), lam = sqrt(3) / ell_t, the temporal state is
(f, f' / lam) (the derivative scaled so that the stationary covariance is the identity),
and one step of length dt has, with s = lam dt and a = exp(-s),

    A^t = a [[1 + s, s], [-s, 1 - s]],    P_inf = I_2,    Q^t = I_2 - A^t A^t^T.

The state of the filter stacks the two components over the n points, value rows first:
u = (f(X), f'(X) / lam), state covariance Sigma_inf = I_2 (x) Sigma, transition
A = A^t (x) I_n, and an observation picks value rows (indices < n).  Since
A Sigma_inf A^T + Q = Sigma_inf, the downdate form P = Sigma_inf - M M^T of the filter
carries over with M^- = A M^+ (Prop. A.2), and the filter of oracle.cakf runs on this
model unchanged (it only calls transition and cov_matmul).

Test infrastructure only; not part of the product path.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import matern


@dataclasses.dataclass
class Matern32TimeModel:
    X: np.ndarray           # n x d spatial points
    nu2: int                # 2 * nu of the spatial Matern kernel
    ell: float              # spatial lengthscale
    sigma_f2: float         # signal variance
    a: float                # exp(-lam dt), lam = sqrt(3) / ell_t
    noise_var: float        # observation noise variance
    dist: int = matern.EUCLID

    @property
    def points(self) -> int:
        return self.X.shape[0]

    @property
    def n(self) -> int:
        """State dimension (value and scaled derivative per point)."""
        return 2 * self.points

    @property
    def s(self) -> float:
        return -math.log(self.a)

    def At(self) -> np.ndarray:
        s = self.s
        return self.a * np.array([[1.0 + s, s], [-s, 1.0 - s]])

    def transition(self, V: np.ndarray) -> np.ndarray:
        """(A^t (x) I_n) V."""
        At = self.At()
        p = self.points
        V0, V1 = V[:p], V[p:]
        return np.concatenate([At[0, 0] * V0 + At[0, 1] * V1, At[1, 0] * V0 + At[1, 1] * V1])

    def _split(self, idx):
        idx = np.arange(self.n) if idx is None else np.asarray(idx)
        return idx // self.points, idx % self.points

    def cov(self, rows=None, cols=None) -> np.ndarray:
        """Sigma_inf[rows, cols] = [component(rows) == component(cols)] Sigma(x, x')."""
        cr, pr = self._split(rows)
        cc, pc = self._split(cols)
        K = matern.gram(self.X[pr], self.X[pc], self.nu2, self.ell, self.sigma_f2, self.dist)
        return np.where(np.equal.outer(cr, cc), K, 0.0)

    def cov_matmul(self, rows, cols, V) -> np.ndarray:
        return self.cov(rows, cols) @ V

