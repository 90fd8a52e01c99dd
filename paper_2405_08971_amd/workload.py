"""Seeded synthetic spatiotemporal workloads for the computation-aware Kalman filter.

This module only draws inputs: spatial point sets, per-step observation index sets,
observation vectors and (for the given-actions policy) action matrices.  It holds none
of the filter's arithmetic and evaluates no covariance function; both the FP64 oracle
and the GPU library receive what it returns as plain arrays.

Stand-in for the paper's workloads (Sec. 6 and App. D): the paper's on-model
experiments draw data from the prior on grids and its large-scale experiment uses the
ERA5 2 m temperature field on the sphere (App. D.2.3, Table 3).  ERA5 is not available
here, so every configuration below uses synthetic points and a prior sample instead:

* points: uniform in the unit square (planar case) or a deterministic Fibonacci
  lattice on the unit sphere (sphere cases, the extrinsic/chordal embedding the paper
  uses for ERA5 in App. D.2.3);
* data: a random-Fourier-feature surrogate of a Matern(nu) prior sample (the spectral
  measure of Matern(nu) with lengthscale l is a Student-t with 2 nu degrees of freedom
  scaled by 1/l), evolved in time by Ornstein-Uhlenbeck weights
  w_k = a w_{k-1} + sqrt(1 - a^2) xi_k, plus iid Gaussian noise of variance noise_var;
* observation sets: m distinct indices per step, redrawn every step; optionally a fixed
  fraction of locations is never observed.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = ["Config", "CONFIGS", "Workload", "make_workload", "fibonacci_sphere",
           "uniform_square"]


@dataclasses.dataclass(frozen=True)
class Config:
    """One workload.  Field names follow the paper's notation where one exists.

    n: number of spatial points (state dimension D, output dimension D' = 1 for the
       Ornstein-Uhlenbeck temporal prior); dim: 2 (unit square) or 3 (unit sphere);
    nu2: 2*nu of the spatial Matern kernel (1, 3 or 5); ell: spatial lengthscale;
    sigma_f2: signal variance; dt, ell_t: time step and temporal lengthscale of the
    Ornstein-Uhlenbeck prior (A = exp(-dt/ell_t) I); T: number of time steps K;
    m: observations per step N_k; noise_var: observation noise variance (Lambda = noise_var I);
    i: actions per step (the action budget); r: rank cap of the truncated downdate factor;
    dist: 0 = Euclidean (chordal on the sphere), 1 = great-circle;
    missing_frac: fraction of locations never observed.
    """

    name: str
    n: int
    dim: int
    nu2: int
    ell: float
    sigma_f2: float
    dt: float
    ell_t: float
    T: int
    m: int
    noise_var: float
    i: int
    r: int
    dist: int = 0
    missing_frac: float = 0.0

    @property
    def a(self) -> float:
        """Ornstein-Uhlenbeck transition coefficient exp(-dt/ell_t)."""
        return math.exp(-self.dt / self.ell_t)

    def replace(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)


# The five workloads of the hot path (small planar case, the FP32 sphere case, the
# n = 65536 precision case, the differentiation case and the large case).
CONFIGS = {
    "plane_n1024": Config(
        "plane_n1024", n=1024, dim=2, nu2=3, ell=0.2, sigma_f2=1.0, dt=1.0, ell_t=5.0,
        T=20, m=256, noise_var=0.01, i=16, r=64),
    "sphere_gc_n16384": Config(
        "sphere_gc_n16384", n=16384, dim=3, nu2=3, ell=0.3, sigma_f2=1.0, dt=1.0, ell_t=5.0,
        T=100, m=4096, noise_var=0.05, i=64, r=256, dist=1),
    "sphere_n65536": Config(
        "sphere_n65536", n=65536, dim=3, nu2=5, ell=0.3, sigma_f2=1.0, dt=1.0, ell_t=5.0,
        T=200, m=16384, noise_var=0.05, i=128, r=512),
    "sphere_n16384": Config(
        "sphere_n16384", n=16384, dim=3, nu2=3, ell=0.3, sigma_f2=1.0, dt=1.0, ell_t=5.0,
        T=50, m=4096, noise_var=0.05, i=64, r=256),
    "sphere_n262144": Config(
        "sphere_n262144", n=262144, dim=3, nu2=3, ell=0.3, sigma_f2=1.0, dt=1.0, ell_t=5.0,
        T=50, m=32768, noise_var=0.02, i=256, r=1024, missing_frac=0.1),
}


def fibonacci_sphere(n: int) -> np.ndarray:
    """n unit vectors of the Fibonacci lattice: z_j = 1-(2j+1)/n, phi_j = j*pi*(3-sqrt 5)."""
    j = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * j + 1.0) / n
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = j * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def uniform_square(n: int, rng: np.random.Generator) -> np.ndarray:
    return rng.random((n, 2))


class Workload:
    """Lazily drawn, seeded inputs of one configuration.

    Every per-step quantity is a deterministic function of (config, seed, step), so a
    step can be regenerated without drawing the earlier ones.
    """

    N_FEATURES = 2048

    def __init__(self, cfg: Config, seed: int = 0, n_features: Optional[int] = None):
        self.cfg = cfg
        self.seed = seed
        ss = np.random.SeedSequence([seed, cfg.n, cfg.m, cfg.T])
        (self._ss_points, self._ss_idx, self._ss_prior, self._ss_noise,
         self._ss_subset, self._ss_actions, self._ss_missing) = ss.spawn(7)
        if cfg.dim == 2:
            self.X = uniform_square(cfg.n, np.random.default_rng(self._ss_points))
        elif cfg.dim == 3:
            self.X = fibonacci_sphere(cfg.n)
        else:
            raise ValueError("dim must be 2 or 3")
        n_missing = int(round(cfg.missing_frac * cfg.n))
        rng_miss = np.random.default_rng(self._ss_missing)
        missing = rng_miss.choice(cfg.n, n_missing, replace=False) if n_missing else \
            np.zeros(0, np.int64)
        mask = np.ones(cfg.n, bool)
        mask[missing] = False
        self.observable = np.nonzero(mask)[0]
        if cfg.m > self.observable.size:
            raise ValueError("more observations per step than observable locations")
        self.n_features = n_features or self.N_FEATURES
        self._prior_ready = False

    # -- random Fourier features of the spatial prior ---------------------------------
    def _init_prior(self):
        cfg = self.cfg
        rng = np.random.default_rng(self._ss_prior)
        J, d = self.n_features, cfg.dim
        nu = cfg.nu2 / 2.0
        z = rng.standard_normal((J, d))
        g = rng.chisquare(2.0 * nu, size=J)
        self._omega = z / (cfg.ell * np.sqrt(g / (2.0 * nu)))[:, None]
        self._phase = rng.uniform(0.0, 2.0 * math.pi, size=J)
        self._w0 = rng.standard_normal(J)
        self._prior_ready = True

    def _weights(self, k: int) -> np.ndarray:
        """OU-evolved feature weights at step k (k = 0 is the initial state)."""
        if not self._prior_ready:
            self._init_prior()
        a = self.cfg.a
        w = self._w0.copy()
        for s in range(1, k + 1):
            rng = np.random.default_rng(np.random.SeedSequence([self.seed, 17, s]))
            w = a * w + math.sqrt(1.0 - a * a) * rng.standard_normal(w.size)
        return w

    def latent(self, k: int, idx: Optional[np.ndarray] = None) -> np.ndarray:
        """Surrogate prior sample u_k at the points idx (all points if None)."""
        if not self._prior_ready:
            self._init_prior()
        Xs = self.X if idx is None else self.X[idx]
        w = self._weights(k)
        scale = math.sqrt(self.cfg.sigma_f2 * 2.0 / self.n_features)
        out = np.empty(Xs.shape[0], np.float64)

        def rows(p0, p1):
            feats = np.cos(Xs[p0:p1] @ self._omega.T + self._phase)
            out[p0:p1] = scale * (feats @ w)

        chunk = 2048
        spans = [(p0, min(Xs.shape[0], p0 + chunk)) for p0 in range(0, Xs.shape[0], chunk)]
        if len(spans) == 1:
            rows(*spans[0])
        else:                     # NumPy releases the interpreter lock in cos and matmul
            from concurrent.futures import ThreadPoolExecutor
            import os
            with ThreadPoolExecutor(min(len(spans), os.cpu_count() or 1)) as ex:
                list(ex.map(lambda sp: rows(*sp), spans))
        return out

    def feature_map(self):
        """(omega, phase, scale) of the random-Fourier-feature surrogate of the spatial
        prior: phi(x) = scale * cos(omega x + phase), so that phi(x)^T w with w ~ N(0, I)
        is an approximate draw from N(0, Sigma)."""
        if not self._prior_ready:
            self._init_prior()
        return self._omega, self._phase, math.sqrt(self.cfg.sigma_f2 * 2.0 / self.n_features)

    def obs_indices(self, k: int) -> np.ndarray:
        """m distinct observed indices at step k >= 1 (int64, unsorted)."""
        rng = np.random.default_rng(np.random.SeedSequence([self.seed, 23, k, self.cfg.n]))
        pick = rng.choice(self.observable.size, self.cfg.m, replace=False)
        return self.observable[pick].astype(np.int64)

    def observations(self, k: int, idx: Optional[np.ndarray] = None) -> np.ndarray:
        """y_k = u_k[idx] + noise."""
        if idx is None:
            idx = self.obs_indices(k)
        rng = np.random.default_rng(np.random.SeedSequence([self.seed, 29, k]))
        u = self.latent(k, idx)
        return u + math.sqrt(self.cfg.noise_var) * rng.standard_normal(idx.size)

    def step(self, k: int):
        """(idx_k, y_k) for step k >= 1."""
        idx = self.obs_indices(k)
        return idx, self.observations(k, idx)

    def actions(self, k: int, m: Optional[int] = None, i: Optional[int] = None) -> np.ndarray:
        """Random Gaussian actions S_k (m x i) for the given-actions policy (App. E)."""
        m = self.cfg.m if m is None else m
        i = self.cfg.i if i is None else i
        rng = np.random.default_rng(np.random.SeedSequence([self.seed, 31, k]))
        return rng.standard_normal((m, i))

    def subset(self, size: int = 2048) -> np.ndarray:
        """Fixed seeded subset of state indices on which results are compared."""
        rng = np.random.default_rng(self._ss_subset)
        size = min(size, self.cfg.n)
        return np.sort(rng.choice(self.cfg.n, size, replace=False))


def make_workload(name_or_cfg, seed: int = 0, **overrides) -> Workload:
    cfg = CONFIGS[name_or_cfg] if isinstance(name_or_cfg, str) else name_or_cfg
    if overrides:
        cfg = cfg.replace(**overrides)
    return Workload(cfg, seed)
