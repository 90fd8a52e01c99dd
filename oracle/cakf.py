"""Computation-aware Kalman filter, plain FP64 (oracle).

Follows the paper step by step:

* Filter loop                    - Alg. 1 (Sec. 3.1): predict, update unless the step
                                   has no data, truncate.
* Iterative update               - the iterative CAKF update of App. B (Alg. "CAKF
                                   Update Step (Iterative Version)"): successive
                                   conditioning on one action at a time with
                                   Ghat-orthogonalised search directions.
* Batch update                   - Alg. 2 (Sec. 3.1): one projection S, pseudo-inverse
                                   and a left square root of the projected Gram matrix.
* Policies                       - CG/Lanczos residual actions (Sec. 3.3, App. E),
                                   block-residual actions (the residual split over fixed
                                   observation groups, b per round) and given actions
                                   (any admissible S, App. E).
* Truncate                       - Sec. 3.2: keep the leading r singular directions of
                                   the downdate factor (Eckart-Young-Mirsky).
* Downdate form of the covariance - Prop. A.2: P_k = Sigma - M_k M_k^T.

The state-space model is the separable spatiotemporal prior with an Ornstein-Uhlenbeck
temporal factor (Lemma C.1): Sigma = sigma_f2 * K(X, X) for every k, A = a I,
Q = (1 - a^2) Sigma, H_k selects the observed rows idx_k, Lambda = noise_var I.

Readings where the paper is silent (each is also listed with the design notes):
* Policy index: the action of iteration i is the residual after i - 1 actions,
  s^(i) = r^(0) - Ghat v^(i-1) (the first action is r^(0)).
* StoppingCriterion: stop after max_actions actions, when the residual norm falls to
  resid_tol * ||r^(0)||, or on breakdown, i.e. when the Ghat-orthogonalised direction
  keeps no more than pivot_tol of the action's Ghat-norm (eta <= pivot_tol * s^T Ghat s).
* Truncation rank: keep min(r_cap, number of columns) leading directions; no rotation
  when the factor already has at most r_cap columns.
* Log-likelihood (not defined in the paper): the prediction-error term of the projected
  observation in the model the filter solves exactly, made independent of the scaling
  of the actions:
      l_k = -1/2 [ i log 2 pi + log det(S^T Ghat S) - log det(S^T S)
                   + (S^T r0)^T (S^T Ghat S)^{-1} (S^T r0) ].

Test infrastructure only; not part of the product path.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np

from . import matern

LOG2PI = math.log(2.0 * math.pi)


@dataclasses.dataclass
class Model:
    """Separable spatiotemporal prior with OU temporal factor (Lemma C.1)."""

    X: np.ndarray           # n x d spatial points
    nu2: int                # 2 * nu of the spatial Matern kernel
    ell: float              # spatial lengthscale
    sigma_f2: float         # signal variance
    a: float                # OU transition coefficient exp(-dt / ell_t)
    noise_var: float        # observation noise variance
    dist: int = matern.EUCLID

    @property
    def n(self) -> int:
        return self.X.shape[0]

    def transition(self, V: np.ndarray) -> np.ndarray:
        """A V for the state transition of one step (OU: A = a I, Lemma C.1)."""
        return self.a * V

    def cov_matmul(self, rows, cols, V) -> np.ndarray:
        """Sigma[rows, cols] @ V  (rows/cols are index arrays or None for all)."""
        A = self.X if rows is None else self.X[rows]
        B = self.X if cols is None else self.X[cols]
        return matern.gram_matmul(A, B, V, self.nu2, self.ell, self.sigma_f2, self.dist)

    def cov(self, rows=None, cols=None) -> np.ndarray:
        A = self.X if rows is None else self.X[rows]
        B = self.X if cols is None else self.X[cols]
        return matern.gram(A, B, self.nu2, self.ell, self.sigma_f2, self.dist)


# ----------------------------------------------------------------------------- policies
def cg_policy():
    """CG/Lanczos actions: the current residual is the next action (Sec. 3.3)."""
    def policy(i: int, residual: np.ndarray):
        return residual
    return policy


def observation_groups(m: int, b: int):
    """The fixed partition of the m observations of a step into b contiguous ranges
    [floor(g m / b), floor((g + 1) m / b)), g = 0 .. b-1 (used by block_residual_policy)."""
    return [(g * m // b, (g + 1) * m // b) for g in range(b)]


def block_residual_policy(b: int, max_actions: int):
    """Block-residual actions (an admissible choice of S, App. E; not one of the paper's
    experiments): actions are taken in rounds of b; at the start of a round the current
    residual r is split over the fixed observation groups, and the round's actions are
    r restricted to group 0, 1, ..., b_t - 1, b_t = min(b, actions left).  With b = 1
    every action is the full residual, i.e. the CG policy."""
    state = {}

    def policy(i: int, residual: np.ndarray):
        k = (i - 1) % b
        if k == 0:
            bt = min(b, max_actions - (i - 1))
            state["r"] = np.array(residual, np.float64)
            state["groups"] = observation_groups(residual.size, bt)
        r = state["r"]
        g0, g1 = state["groups"][k]
        s = np.zeros_like(r)
        s[g0:g1] = r[g0:g1]
        return s
    return policy


def given_policy(S: np.ndarray):
    """Actions taken column by column from a given matrix (any S is admissible)."""
    def policy(i: int, residual: np.ndarray):
        return S[:, i - 1] if i - 1 < S.shape[1] else None
    return policy


# ---------------------------------------------------------------------- update steps
@dataclasses.dataclass
class UpdateResult:
    m: np.ndarray            # filter mean
    M: np.ndarray            # untruncated downdate factor (M_pred | P_pred H^T W)
    S: np.ndarray            # actions actually used (m_obs x i_eff)
    w_obs: np.ndarray        # v in observation coordinates (w = H^T v)
    W_obs: np.ndarray        # V in observation coordinates (W = H^T V)
    loglik: float
    i_eff: int


class _ProjectedGram:
    """Matrix-free Ghat = H P_pred H^T + Lambda on the observed points."""

    def __init__(self, model: Model, M_pred: np.ndarray, idx: np.ndarray):
        self.model = model
        self.idx = idx
        self.Mo = M_pred[idx]

    def __call__(self, V: np.ndarray) -> np.ndarray:
        md = self.model
        return (md.cov_matmul(self.idx, self.idx, V) - self.Mo @ (self.Mo.T @ V)
                + md.noise_var * V)


def projected_loglik(S: np.ndarray, Ghat_S: np.ndarray, r0: np.ndarray) -> float:
    """l_k from its definition: S (m x i), Ghat_S = Ghat @ S, r0 = y - H m_pred."""
    i = S.shape[1]
    if i == 0:
        return 0.0
    C = S.T @ Ghat_S
    C = 0.5 * (C + C.T)
    c = S.T @ r0
    sign_c, logdet_c = np.linalg.slogdet(C)
    sign_s, logdet_s = np.linalg.slogdet(S.T @ S)
    if sign_c <= 0 or sign_s <= 0:
        raise np.linalg.LinAlgError("projected Gram matrix is not positive definite")
    return float(-0.5 * (i * LOG2PI + logdet_c - logdet_s + c @ np.linalg.solve(C, c)))


def _posterior_products(model, m_pred, M_pred, idx, w_obs, W_obs):
    """m = m_pred + P_pred H^T w_obs and M = (M_pred, P_pred H^T W_obs)."""
    B = np.column_stack([W_obs, w_obs])
    Mo = M_pred[idx]
    Y = model.cov_matmul(None, idx, B) - M_pred @ (Mo.T @ B)
    m = m_pred + Y[:, -1]
    M = np.hstack([M_pred, Y[:, :-1]])
    return m, M


def update_iterative(model: Model, m_pred, M_pred, idx, y, policy: Callable,
                     max_actions: int, resid_tol: float = 0.0,
                     pivot_tol: float = 1e-10) -> UpdateResult:
    """Iterative CAKF update (App. B): one action at a time."""
    idx = np.asarray(idx)
    Ghat = _ProjectedGram(model, M_pred, idx)
    r0 = np.asarray(y, np.float64) - m_pred[idx]
    mo = r0.size
    v = np.zeros(mo)
    Vd = np.zeros((mo, 0))
    actions = []
    r0_norm = np.linalg.norm(r0)
    for i in range(1, max_actions + 1):
        r = r0 - Ghat(v)                       # residual after i - 1 actions
        if np.linalg.norm(r) <= resid_tol * r0_norm:
            break
        s = policy(i, r)
        if s is None:
            break
        s = np.asarray(s, np.float64)
        alpha = s @ r
        Gs = Ghat(s)
        d = s - Vd @ (Vd.T @ Gs)               # Ghat-orthogonalise against earlier actions
        eta = s @ Ghat(d)
        if not eta > pivot_tol * (s @ Gs):     # breakdown: s adds no new direction
            break
        v = v + (alpha / eta) * d
        Vd = np.column_stack([Vd, d / math.sqrt(eta)])
        actions.append(s)
    S = np.column_stack(actions) if actions else np.zeros((mo, 0))
    m, M = _posterior_products(model, m_pred, M_pred, idx, v, Vd)
    ll = projected_loglik(S, Ghat(S), r0) if S.shape[1] else 0.0
    return UpdateResult(m, M, S, v, Vd, ll, S.shape[1])


def lsqrt_pinv(C: np.ndarray, rtol: float = 1e-12) -> np.ndarray:
    """A left square root V of the pseudo-inverse of a symmetric PSD C: V V^T = C^+."""
    lam, U = np.linalg.eigh(0.5 * (C + C.T))
    keep = lam > rtol * max(lam.max(initial=0.0), 0.0)
    return U[:, keep] / np.sqrt(lam[keep])


def update_batch(model: Model, m_pred, M_pred, idx, y, S: np.ndarray,
                 lsqrt: str = "eigh") -> UpdateResult:
    """Batch CAKF update (Alg. 2) for a given action matrix S.

    lsqrt selects the left square root of the pseudo-inverse: "eigh" (any V with
    V V^T = C^+, from an eigendecomposition) or "chol" (V = L^{-T} from the Cholesky
    factor C = L L^T, which is what the iterative form produces)."""
    idx = np.asarray(idx)
    Ghat = _ProjectedGram(model, M_pred, idx)
    r0 = np.asarray(y, np.float64) - m_pred[idx]
    GS = Ghat(S)
    C = S.T @ GS                                # Hcheck P_pred Hcheck^T + Lambdacheck
    if lsqrt == "eigh":
        Vc = lsqrt_pinv(C)
    elif lsqrt == "chol":
        L = np.linalg.cholesky(0.5 * (C + C.T))
        Vc = np.linalg.inv(L).T
    else:
        raise ValueError(lsqrt)
    Cp = Vc @ Vc.T                              # Ghat^+ on the projected space
    w_obs = S @ (Cp @ (S.T @ r0))
    W_obs = S @ Vc
    m, M = _posterior_products(model, m_pred, M_pred, idx, w_obs, W_obs)
    ll = projected_loglik(S, GS, r0)
    return UpdateResult(m, M, S, w_obs, W_obs, ll, S.shape[1])


# -------------------------------------------------------------------------- truncation
def truncate(M: np.ndarray, r_cap: int, V_fixed: Optional[np.ndarray] = None):
    """Truncate (Sec. 3.2): keep the top min(r_cap, cols) directions of M M^T.

    Returns (M_plus, V_r, eigenvalues of M^T M in descending order).  With V_fixed the
    rotation is replayed instead of recomputed (used for frozen-rotation derivatives)."""
    k = M.shape[1]
    if V_fixed is not None:
        return M @ V_fixed, V_fixed, None
    if k <= r_cap:
        return M, None, None
    lam, V = np.linalg.eigh(M.T @ M)
    order = np.argsort(lam)[::-1]
    lam, V = lam[order], V[:, order]
    Vr = V[:, :r_cap]
    return M @ Vr, Vr, lam


# ------------------------------------------------------------------------- filter loop
@dataclasses.dataclass
class StepRecord:
    k: int
    m_pred: np.ndarray
    M_pred: np.ndarray
    m: np.ndarray
    M: np.ndarray              # untruncated factor of the filter covariance
    M_plus: np.ndarray         # truncated factor carried to the next step
    idx: Optional[np.ndarray]
    S: Optional[np.ndarray]
    w_obs: Optional[np.ndarray]
    W_obs: Optional[np.ndarray]
    loglik: float
    i_eff: int
    V_r: Optional[np.ndarray]
    eigvals: Optional[np.ndarray]

    def marginal_var(self, sigma_f2: float) -> np.ndarray:
        """diag(P_k) = sigma_f2 - row sums of M_k^2 (Prop. A.2, k(x, x) = sigma_f2)."""
        return sigma_f2 - np.sum(self.M * self.M, axis=1)


def run_filter(model: Model, steps, max_actions: int, r_cap: int, policy: str = "cg",
               actions=None, resid_tol: float = 0.0, pivot_tol: float = 1e-10,
               form: str = "iterative", rotations=None, m0=None, M0=None,
               lsqrt: str = "eigh") -> List[StepRecord]:
    """Alg. 1.  steps[k-1] = (idx_k, y_k) or None (no data) for k = 1..T.

    policy "cg": residual actions; policy ("block", b): block-residual actions in rounds
    of b; policy "given": actions[k-1] is S_k (m_k x i).
    rotations[k-1], if given, replays the truncation rotation of step k.
    form "batch" (given actions only) takes the square root lsqrt of update_batch; "chol"
    gives the factor columns of the iterative form (S L^{-T})."""
    n = model.n
    m = np.zeros(n) if m0 is None else np.asarray(m0, np.float64)
    Mp = np.zeros((n, 0)) if M0 is None else np.asarray(M0, np.float64)
    recs = []
    for k, item in enumerate(steps, start=1):
        m_pred = model.transition(m)
        M_pred = model.transition(Mp)
        if item is None:
            m, M = m_pred, M_pred
            idx = S = w_obs = W_obs = None
            ll, i_eff = 0.0, 0
        else:
            idx, y = item
            idx = np.asarray(idx)
            if policy == "cg":
                pol = cg_policy()
            elif isinstance(policy, tuple) and policy[0] == "block":
                pol = block_residual_policy(int(policy[1]), max_actions)
            elif policy == "given":
                pol = given_policy(np.asarray(actions[k - 1], np.float64))
            else:
                raise ValueError(policy)
            if form == "iterative":
                res = update_iterative(model, m_pred, M_pred, idx, y, pol, max_actions,
                                       resid_tol, pivot_tol)
            elif form == "batch":
                if policy != "given":
                    raise ValueError("the batch form needs given actions")
                res = update_batch(model, m_pred, M_pred, idx, y,
                                   np.asarray(actions[k - 1], np.float64)[:, :max_actions],
                                   lsqrt=lsqrt)
            else:
                raise ValueError(form)
            m, M = res.m, res.M
            S, w_obs, W_obs, ll, i_eff = res.S, res.w_obs, res.W_obs, res.loglik, res.i_eff
        V_fixed = None if rotations is None else rotations[k - 1]
        Mp, Vr, lam = truncate(M, r_cap, V_fixed)
        recs.append(StepRecord(k, m_pred, M_pred, m, M, Mp, idx, S, w_obs, W_obs, ll,
                               i_eff, Vr, lam))
    return recs


def total_loglik(recs: List[StepRecord]) -> float:
    return float(sum(r.loglik for r in recs))
