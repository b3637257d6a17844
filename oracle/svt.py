"""Plain FP64 oracle of fast SVT with R4SVD (test infrastructure only).

Follows Li & Yu, "A Fast Implementation of Singular Value Thresholding
Algorithm using Recycling Rank Revealing Randomized SVD":
  * the SVT iteration X = D_tau(Y), Y += delta P_Lambda(A - X)   (Sec. 1, Eq. 4)
  * the SVT operator D_tau as a sum over singular triplets      (Sec. 1, Eq. 5)
  * the error percentage and its QB form                        (Sec. 2.2, Eq. 8, 10, 11)
  * R3SVD on the first SVT iteration                            (Sec. 2.2, Alg. 2)
  * R4SVD with recycling of the previous left singular vectors  (Sec. 2.4, Alg. 3)
  * the annealing of the precision threshold and Fast SVT       (Sec. 2.5, Eq. 13-14, Alg. 4)

The steps are taken in the paper's order with scipy sparse products, numpy
Householder QR and numpy SVD as library primitives.  Where the paper is silent
or garbled the reading taken is stated at the point of use (readings R0 / S1..S30
of the design notes).  Nothing here is tuned; nothing here is used by the
device path.
"""
from dataclasses import dataclass, field, replace
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .philox import omega_block

DROP_TOL = 1e-10  # a projected column at most this fraction of its norm before lies in span(Q)
DEP_TOL = 1e-6    # an R diagonal at most this fraction of the projected column norm means dependence


# ----------------------------------------------------------------------------------------------
# Exact definitions (used for pins and as the "SVT-full SVD" reference of Sec. 3)
# ----------------------------------------------------------------------------------------------

def d_tau(Y, tau):
    """Singular value thresholding operator of Eq. 5 by a full SVD of a dense Y."""
    U, s, Vt = np.linalg.svd(Y, full_matrices=False)
    keep = s > tau  # sigma == tau contributes a zero term either way (Eq. 5 uses >=)
    return (U[:, keep] * (s[keep] - tau)) @ Vt[keep]


def dense(m, n, rows, cols, vals):
    Y = np.zeros((m, n))
    Y[rows, cols] = vals
    return Y


def spectral_norm(m, n, rows, cols, vals):
    """||P_Lambda(A)||_2: dense SVD for small matrices, else ARPACK to 1e-14."""
    if m * n <= 4_000_000:
        return float(np.linalg.norm(dense(m, n, rows, cols, vals), 2))
    M = sp.csr_matrix((vals, (rows, cols)), shape=(m, n))
    s = spla.svds(M, k=1, tol=1e-14, return_singular_vectors=False, random_state=0)
    return float(s[0])


def kicking_k0(tau, delta, sigma1):
    """Kicking step count of Alg. 4's initialisation (reading S14: spectral norm, k0 = ceil(tau/(delta sigma1)))."""
    return int(math.ceil(tau / (delta * sigma1)))


# ----------------------------------------------------------------------------------------------
# Problem, parameters, state
# ----------------------------------------------------------------------------------------------

@dataclass
class Problem:
    """Observed set Lambda as COO (rows, cols) and the sampled entries a = P_Lambda(A) on it."""
    m: int
    n: int
    rows: np.ndarray
    cols: np.ndarray
    a: np.ndarray

    def __post_init__(self):
        self.rows = np.asarray(self.rows, dtype=np.int64)
        self.cols = np.asarray(self.cols, dtype=np.int64)
        self.a = np.asarray(self.a, dtype=np.float64)
        self.norm_a = float(np.linalg.norm(self.a))

    def sparse(self, y):
        return sp.csr_matrix((y, (self.rows, self.cols)), shape=(self.m, self.n))


@dataclass
class Params:
    """Inputs of Alg. 4 plus the parameters the paper leaves unstated (readings in brackets)."""
    tau: float
    delta: float
    tol: float = 1e-4
    maxit: int = 500            # [S20] not given in the paper
    t0: int = 0                 # <= 0: floor(0.05 min(m, n)) (Sec. 3 setup), at least 1
    dt: int = 10                # Delta t (Sec. 3 setup)
    npow: int = 0               # [S3] power iterations, X <- Y (Y^T X) after re-orthonormalisation
    beta: float = 0.95          # annealing factor (Sec. 3 setup)
    eta: float = 0.0            # [S12] strict "stops decreasing" test when 0
    eps_thr0: float = -1.0      # [S1] < 0: (1 + eps_1) / 2 from the first t-block
    r_max: int = 0              # [S19] <= 0: m (an orthonormal basis in R^m holds at most m columns)
    seed: int = 0               # Omega stream key
    k0: int = -1                # < 0: kicking count computed from ||P_Lambda A||_2
    # Variants of the operator (all default to Alg. 4 with R4SVD):
    #   mode "r4svd": recycle the previous left singular vectors (Alg. 3);
    #   mode "r3svd": no recycling, Alg. 2 from a fresh t-block in every SVT iteration;
    #   mode "rsvd":  fixed-rank randomized SVD (Alg. 1) with `rank` + `oversample` samples and the
    #                 `rank` leading singular triplets thresholded.
    mode: str = "r4svd"
    recycle_extra: int = -1     # >= 0: recycle only the leading k + recycle_extra left singular vectors
    rank: int = 0               # rank of the "rsvd" mode
    oversample: int = 10        # oversampling p of the "rsvd" mode
    mae_tol: float = 0.0        # > 0: also stop when the sample MAE on Lambda falls below it (Eq. 15, Sec. 3)

    def resolved(self, m, n):
        if self.mode not in ("r4svd", "r3svd", "rsvd"):
            raise ValueError(f"unknown mode {self.mode!r}")
        if self.mode == "rsvd" and self.rank <= 0:
            raise ValueError("the rsvd mode needs rank > 0")
        t0 = self.t0 if self.t0 > 0 else max(1, int(math.floor(0.05 * min(m, n))))
        r_max = min(self.r_max, m) if self.r_max > 0 else m
        if self.mode == "rsvd":
            t0 = self.rank + max(self.oversample, 0)
        return replace(self, t0=min(t0, r_max), r_max=r_max)


@dataclass
class State:
    """What carries over between SVT iterations: Y on Lambda, the recycled basis, the annealing state."""
    it: int                      # SVT iterations completed so far
    y: np.ndarray                # Y^(it+1) on Lambda, in the problem's COO order
    Q: np.ndarray = None         # recycled left singular vectors U_L^(it), m x r (None before the first call)
    eps_thr: float = None        # epsilon_threshold (None until the first t-block fixes it, S1)
    eps_min: float = math.inf


@dataclass
class StepInfo:
    it: int
    r: int = 0
    k: int = 0
    blocks: int = 0              # growth blocks added in this iteration
    exhausted: bool = False      # a growth block lost every column (range exhausted)
    eps: float = 0.0             # error percentage when R4SVD returned
    eps_hist: list = field(default_factory=list)  # eps after the first projection and after each block
    grow_margins: list = field(default_factory=list)  # (eps - eps_thr) / eps_thr at each growth test
    eps_thr_used: float = 0.0    # threshold R4SVD ran with
    normY: float = 0.0
    normB: float = 0.0
    sigma: np.ndarray = None     # all singular values of B
    x: np.ndarray = None         # X^(i) on Lambda
    rel: float = 0.0             # ||P_Lambda(A - X)||_F / ||P_Lambda A||_F   (S10)
    mae: float = 0.0             # sample MAE (1/|Lambda|) sum |A - X| on Lambda (Sec. 3)
    annealed: bool = False
    anneal_margin: float = 0.0   # (rel - eps_min (1 - eta)) / eps_min before the update
    stopped: bool = False
    U: np.ndarray = None         # U_L on the thresholded set K (m x k)
    s_minus_tau: np.ndarray = None
    V: np.ndarray = None         # V_L on K (n x k)
    Q: np.ndarray = None         # basis before the final rotation (m x r)
    W: np.ndarray = None         # B^T = Y^T Q (n x r)


# ----------------------------------------------------------------------------------------------
# R3SVD / R4SVD (Alg. 2 and Alg. 3)
# ----------------------------------------------------------------------------------------------

def _orthonormal_block(X, pre_norms):
    """Householder QR of a projected block with the column-drop reading of S5.

    A column whose norm after projection is at most DROP_TOL times its norm
    before projection lies in span(Q) to working precision and is dropped.
    The kept columns go through numpy's Householder QR; a column whose R
    diagonal is at most DEP_TOL times its projected norm depends on the
    columns before it and is also dropped.
    """
    post = np.linalg.norm(X, axis=0)
    keep = post > DROP_TOL * pre_norms
    X = X[:, keep]
    post = post[keep]
    if X.shape[1] == 0:
        return X
    Qb, R = np.linalg.qr(X)
    ok = np.abs(np.diag(R)) > DEP_TOL * post
    if not ok.all():
        Qb, _ = np.linalg.qr(X[:, ok]) if ok.any() else (X[:, :0], None)
    return Qb


def _sample_block(Y, seed, it, blk, w, npow):
    """X = Y Omega followed by npow power iterations X <- Y (Y^T X) (reading S3)."""
    n = Y.shape[1]
    X = Y @ omega_block(seed, it, blk, n, w)
    for _ in range(npow):
        X, _ = np.linalg.qr(X)
        X = Y @ (Y.T @ X)
    return X


def r4svd(Y, normY, Q, eps_thr, p, it, replay_blocks=None, info=None):
    """Alg. 3 (Alg. 2 when Q is None) on the sparse iterate Y.

    Returns (Q, W, normB, eps, eps_thr) with W = B^T = Y^T Q, and fills `info`
    with the decision trace.  eps_thr is returned because the first call fixes
    it from the first t-block (reading S1).
    """
    if Q is None:
        # Alg. 2, initial QB decomposition from a t-block (reading S2: first SVT iteration only).
        X = _sample_block(Y, p.seed, it, 0, p.t0, p.npow)
        Q = _orthonormal_block(X, np.linalg.norm(X, axis=0))
    W = np.asarray(Y.T @ Q)                       # B = Q^T Y, kept transposed
    normB = float(np.sum(W * W))                  # ||B||_F^2
    eps = (normY - normB) / normY                 # Eq. 10 with the numerator read as ||Y||^2 - ||B||^2 (S6)
    if eps_thr is None:
        eps_thr = p.eps_thr0 if p.eps_thr0 >= 0 else 0.5 * (1.0 + eps)   # reading S1
    info.eps_thr_used = eps_thr
    info.eps_hist.append(eps)
    blk = 0
    while p.mode != "rsvd":              # Alg. 1 takes one sample of fixed width, no growth
        r = Q.shape[1]
        room = min(p.dt, p.r_max - r)
        if replay_blocks is not None:
            grow = blk < replay_blocks
        else:
            grow = eps > eps_thr
            info.grow_margins.append((eps - eps_thr) / eps_thr if eps_thr > 0 else math.inf)
        if not grow or room <= 0:
            break
        blk += 1
        X = _sample_block(Y, p.seed, it, blk, room, p.npow)
        pre = np.linalg.norm(X, axis=0)
        for _ in range(2):                        # X <- X - Q Q^T X, twice (reading S4)
            X = X - Q @ (Q.T @ X)
        Qn = _orthonormal_block(X, pre)
        if Qn.shape[1] == 0:
            info.exhausted = True
            break
        Wn = np.asarray(Y.T @ Qn)                 # B' = Q'^T Y
        Q = np.hstack([Qn, Q])                    # Q <- [Q', Q]
        W = np.hstack([Wn, W])                    # B <- [B'; B]
        normB += float(np.sum(Wn * Wn))           # Eq. 11
        eps = (normY - normB) / normY
        info.eps_hist.append(eps)
    info.blocks = blk
    return Q, W, normB, eps, eps_thr


# ----------------------------------------------------------------------------------------------
# Fast SVT (Alg. 4)
# ----------------------------------------------------------------------------------------------

def initial_state(prob, p):
    """Kicking initialisation of Alg. 4 (reading S14): Y^(0) = k0 delta P_Lambda(A)."""
    k0 = p.k0
    if k0 < 0:
        k0 = kicking_k0(p.tau, p.delta, spectral_norm(prob.m, prob.n, prob.rows, prob.cols, prob.a))
    return State(it=0, y=k0 * p.delta * prob.a.copy()), k0


def svt_step(prob, p, state, replay=None):
    """One iteration of Alg. 4 under reading S11: R4SVD, X on Lambda, residual, annealing, stop, dual update.

    replay: optional (blocks, annealed) pair that forces the two discrete decisions.
    Returns (new_state, info).
    """
    p = p.resolved(prob.m, prob.n)
    it = state.it + 1
    info = StepInfo(it=it)
    Y = prob.sparse(state.y)
    normY = float(state.y @ state.y)
    Q0 = state.Q if p.mode == "r4svd" else None   # R3SVD / RSVD start every iteration from a fresh sample
    Q, W, normB, eps, eps_thr = r4svd(Y, normY, Q0, state.eps_thr, p, it,
                                      replay_blocks=None if replay is None else replay[0], info=info)
    info.r, info.eps, info.normY, info.normB, info.Q, info.W = Q.shape[1], eps, normY, normB, Q, W

    # svd(B) with B = W^T (r x n); U_L = Q U_B.  When r > n the thin SVD has only n left vectors;
    # the full one keeps all r columns so that the whole basis is recycled (reading S8).
    U_B, s, VBt = np.linalg.svd(W.T, full_matrices=W.shape[1] > W.shape[0])
    K = np.flatnonzero(s > p.tau)                  # reading S16
    if p.mode == "rsvd":
        K = K[K < p.rank]                          # Alg. 1 keeps the `rank` leading triplets
    info.sigma, info.k = s, int(K.size)
    U_L = Q @ U_B
    info.U, info.s_minus_tau, info.V = U_L[:, K], s[K] - p.tau, VBt[K].T

    # X^(i) = D_tau(U_L, Sigma_L, V_L) sampled on Lambda (Eq. 5), then the residual (S10).
    x = np.zeros_like(prob.a)
    for l in K:
        x += (s[l] - p.tau) * U_L[prob.rows, l] * VBt[l, prob.cols]
    res = prob.a - x
    rel = float(np.linalg.norm(res)) / prob.norm_a
    info.x, info.rel = x, rel
    info.mae = float(np.mean(np.abs(res)))

    # Annealing (Eq. 14): a residual that does not decrease tightens the threshold.
    eps_min = state.eps_min
    target = eps_min * (1.0 - p.eta)
    info.anneal_margin = (rel - target) / eps_min if math.isfinite(eps_min) else -math.inf
    annealed = (rel >= target) if replay is None else bool(replay[1])
    if annealed:
        eps_thr = p.beta * eps_thr
    else:
        eps_min = rel
    info.annealed = annealed

    # recycle U_L: all r columns (S8), or the leading k + recycle_extra (truncated recycling)
    keep = U_L.shape[1] if p.recycle_extra < 0 else min(U_L.shape[1], info.k + p.recycle_extra)
    new = State(it=it, y=state.y.copy(), Q=U_L[:, :keep] if keep > 0 else None, eps_thr=eps_thr, eps_min=eps_min)
    if rel < p.tol or (p.mae_tol > 0 and info.mae < p.mae_tol):
        info.stopped = True
        return new, info
    new.y = state.y + p.delta * res                # Eq. 4, dual update on Lambda
    return new, info


def svt_run(prob, p, state=None, max_steps=None, replay=None, keep_infos=False):
    """Alg. 4 until rel < tol or maxit.  Returns (state, infos or last info, k0)."""
    k0 = None
    if state is None:
        state, k0 = initial_state(prob, p)
    infos = []
    steps = p.maxit if max_steps is None else max_steps
    info = None
    for s in range(steps):
        rp = None if replay is None or s >= len(replay) else replay[s]
        state, info = svt_step(prob, p, state, rp)
        if keep_infos:
            infos.append(info)
        if info.stopped:
            break
    return state, (infos if keep_infos else info), k0


# ----------------------------------------------------------------------------------------------
# SVT with an exact D_tau (the "SVT-full SVD" variant of Sec. 3), same initialisation and stop rule
# ----------------------------------------------------------------------------------------------

def svt_exact_step(prob, p, y):
    X = d_tau(dense(prob.m, prob.n, prob.rows, prob.cols, y), p.tau)
    x = X[prob.rows, prob.cols]
    res = prob.a - x
    return x, res, float(np.linalg.norm(res)) / prob.norm_a, X


def svt_exact_run(prob, p, y0=None, max_steps=None):
    if y0 is None:
        y0 = initial_state(prob, p)[0].y
    y = y0.copy()
    hist = []
    steps = p.maxit if max_steps is None else max_steps
    X = None
    for _ in range(steps):
        x, res, rel, X = svt_exact_step(prob, p, y)
        hist.append(rel)
        if rel < p.tol:
            break
        y = y + p.delta * res
    return y, X, hist
