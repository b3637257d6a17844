"""Seeded synthetic inputs for matrix completion (shared by the oracle's tests and the device path).

This module only builds inputs: observed index sets Lambda (COO, sorted by
linear index i*n + j), the sampled values P_Lambda(A), the threshold tau and
step size delta.  It contains none of the SVT / R4SVD arithmetic.

The paper's own inputs (two images and MovieLens 10M, Sec. 3) are not
available; these generators stand in for them with the shapes and structure
of the image-recovery and recommendation workloads.
"""
from dataclasses import dataclass
import math

import numpy as np

__all__ = ["Workload", "planted", "image", "ratings", "image_adjoint", "large_sparse", "tiny_dense", "heavy_columns",
           "by_name"]


@dataclass
class Workload:
    name: str
    m: int
    n: int
    rows: np.ndarray          # int32, observed row indices
    cols: np.ndarray          # int32, observed column indices
    a: np.ndarray             # float64 observed values
    tau: float
    delta: float
    tol: float
    A: np.ndarray = None      # full matrix when small enough to keep (tests only)
    held_rows: np.ndarray = None
    held_cols: np.ndarray = None
    held_a: np.ndarray = None

    @property
    def nnz(self):
        return int(self.a.size)


def _sample_lambda(rng, m, n, count):
    lin = np.sort(rng.choice(m * n, size=count, replace=False))
    return (lin // n).astype(np.int32), (lin % n).astype(np.int32)


def planted(m=1000, n=1000, rank=10, frac=0.2, seed=1, tau=None, delta=None, tol=1e-4):
    """Planted low-rank A = M N with i.i.d. N(0,1) factors and a uniform sample of round(frac*m*n) entries.

    Defaults are the 1000x1000 rank-10, 20%-observed problem with tau = 5 sqrt(mn)
    and delta = 1.2 mn / |Lambda| (the Cai-Candes-Shen choices).
    """
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((m, rank))
    N = rng.standard_normal((rank, n))
    A = M @ N
    count = int(round(frac * m * n))
    rows, cols = _sample_lambda(rng, m, n, count)
    a = A[rows, cols].astype(np.float64)
    tau = 5.0 * math.sqrt(m * n) if tau is None else tau
    delta = 1.2 * m * n / count if delta is None else delta
    return Workload("planted", m, n, rows, cols, a, tau, delta, tol, A=A if m * n <= 4_000_000 else None)


def _image_matrix(rng, N, terms=40, noise=0.01):
    ii = np.arange(N) + 0.5
    S = np.zeros((N, N))
    for k in range(1, terms + 1):
        f, g = rng.integers(0, 9, size=2)
        ph, ps = rng.uniform(0.0, 2.0 * np.pi, size=2)
        u = np.cos(np.pi * f * ii / N + ph)
        v = np.cos(np.pi * g * ii / N + ps)
        S += k ** -1.5 * np.outer(u, v)
    A = 0.5 + 0.5 * S / np.abs(S).max() + rng.normal(0.0, noise, size=(N, N))
    return np.clip(A, 0.0, 1.0).astype(np.float32).astype(np.float64)


def image(N=1024, frac=0.5, seed=2, tol=1e-4):
    """Image-recovery shape: sum of 40 separable low-frequency cosine patterns with k^-1.5 amplitudes,
    plus N(0, 0.01^2) noise, clipped to [0, 1] and stored FP32; a uniform sample of frac*N^2 pixels.
    tau = ||P_Lambda A||_F and delta = sqrt(mn/|Lambda|) (the paper's Sec. 3 settings)."""
    rng = np.random.default_rng(seed)
    A = _image_matrix(rng, N)
    count = int(round(frac * N * N))
    rows, cols = _sample_lambda(rng, N, N, count)
    a = A[rows, cols]
    tau = float(np.linalg.norm(a))
    delta = math.sqrt(N * N / count)
    return Workload("image", N, N, rows, cols, a, tau, delta, tol, A=A)


def image_adjoint(N=1024, frac=0.5, held_frac=0.05, seed=2, held_seed=4):
    """The image workload plus a held-out set H of held_frac*N^2 pixels drawn from the unobserved ones."""
    w = image(N, frac, seed)
    rng = np.random.default_rng(held_seed)
    obs = np.zeros(N * N, dtype=bool)
    obs[w.rows.astype(np.int64) * N + w.cols] = True
    free = np.flatnonzero(~obs)
    h = np.sort(rng.choice(free, size=int(round(held_frac * N * N)), replace=False))
    w.held_rows, w.held_cols = (h // N).astype(np.int32), (h % N).astype(np.int32)
    w.held_a = w.A[w.held_rows, w.held_cols]
    w.name = "image_adjoint"
    return w


def ratings(m=6040, n=3706, total=1_000_209, zipf=1.2, min_deg=20, rank=10, seed=3, held_frac=0.1, tol=1e-4):
    """Recommendation shape: power-law row and column degrees, ratings 1..5 from a rank-10 factor model.

    Row degrees are min_deg plus a share of the remainder proportional to rank^-zipf over a random
    permutation of users (capped at n); each user picks distinct movies with probability weights
    proportional to movie-popularity rank^-zipf (Efraimidis-Spirakis keys u^(1/w)).  A random
    held_frac of the entries is held out; tau and delta come from the training entries.
    """
    rng = np.random.default_rng(seed)
    extra = total - min_deg * m
    wrow = np.arange(1, m + 1, dtype=np.float64) ** -zipf
    deg = min_deg + np.floor(extra * wrow / wrow.sum()).astype(np.int64)
    deg = np.minimum(deg, n)
    short = total - int(deg.sum())
    order = np.argsort(-wrow, kind="stable")
    i = 0
    while short > 0:                                   # hand out the rounding remainder, heaviest users first
        u = order[i % m]
        if deg[u] < n:
            deg[u] += 1
            short -= 1
        i += 1
    deg = deg[rng.permutation(m)]
    wcol = (np.arange(1, n + 1, dtype=np.float64) ** -zipf)[rng.permutation(n)]
    rows_l, cols_l = [], []
    for u in range(m):
        keys = rng.random(n) ** (1.0 / wcol)
        pick = np.argpartition(-keys, deg[u] - 1)[: deg[u]]
        rows_l.append(np.full(deg[u], u, dtype=np.int64))
        cols_l.append(np.sort(pick))
    rows = np.concatenate(rows_l)
    cols = np.concatenate(cols_l)
    U = rng.standard_normal((m, rank))
    V = rng.standard_normal((n, rank))
    F = np.einsum("ij,ij->i", U[rows], V[cols])
    z = 3.6 + 1.1 * (F - F.mean()) / F.std() + rng.normal(0.0, 0.5, size=F.size)
    val = np.clip(np.rint(z), 1, 5).astype(np.float32).astype(np.float64)
    perm = rng.permutation(total)
    n_held = int(round(held_frac * total))
    held, train = np.sort(perm[:n_held]), np.sort(perm[n_held:])
    tr_r, tr_c, tr_a = rows[train], cols[train], val[train]
    lin = tr_r * n + tr_c
    o = np.argsort(lin)
    w = Workload("ratings", m, n, tr_r[o].astype(np.int32), tr_c[o].astype(np.int32), tr_a[o],
                 float(np.linalg.norm(tr_a)), math.sqrt(m * n / tr_a.size), tol)
    w.held_rows, w.held_cols, w.held_a = rows[held].astype(np.int32), cols[held].astype(np.int32), val[held]
    return w


def _round_bf16(x):
    """Round float64 -> bfloat16 (nearest, ties to even) via float32, returned as float64."""
    f = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (f >> np.uint64(16)) & np.uint64(1)
    f = (f + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return f.astype(np.uint32).view(np.float32).astype(np.float64)


def _alias_table(w):
    """Vose's alias method for drawing index i with probability w_i / sum(w) in O(1) per draw."""
    k = w.size
    prob = w * (k / w.sum())
    alias = np.zeros(k, dtype=np.int64)
    small = [i for i in range(k) if prob[i] < 1.0]
    large = [i for i in range(k) if prob[i] >= 1.0]
    prob = prob.tolist()
    while small and large:
        s_, l_ = small.pop(), large.pop()
        alias[s_] = l_
        prob[l_] = prob[l_] + prob[s_] - 1.0
        (small if prob[l_] < 1.0 else large).append(l_)
    for i in small + large:
        prob[i] = 1.0
    return np.asarray(prob), alias


def _alias_draw(rng, table, size):
    prob, alias = table
    i = rng.integers(0, prob.size, size=size)
    return np.where(rng.random(size) < prob[i], i, alias[i])


def large_sparse(m=100_000, n=50_000, rank=20, total=20_000_000, zipf=1.1, noise=0.1, seed=5, tol=1e-3):
    """Large sparse: planted rank-20 Gaussian factors plus N(0, noise^2), Chung-Lu pattern with
    power-law row/column weights, exactly `total` unique entries, values rounded to BF16."""
    rng = np.random.default_rng(seed)
    wr = (np.arange(1, m + 1, dtype=np.float64) ** -zipf)[rng.permutation(m)]
    wc = (np.arange(1, n + 1, dtype=np.float64) ** -zipf)[rng.permutation(n)]
    tr, tc = _alias_table(wr), _alias_table(wc)
    lin = np.empty(0, dtype=np.int64)
    while lin.size < total:
        # heavy rows and columns saturate, so late draws are mostly repeats: draw in large batches
        need = int((total - lin.size) * 1.3) + total // 4
        r = _alias_draw(rng, tr, need)       # row i with probability wr_i / sum wr (Chung-Lu)
        c = _alias_draw(rng, tc, need)
        lin = np.unique(np.concatenate([lin, r * n + c]))
    lin = np.sort(rng.choice(lin, size=total, replace=False))
    rows, cols = (lin // n).astype(np.int32), (lin % n).astype(np.int32)
    M = rng.standard_normal((m, rank))
    N = rng.standard_normal((n, rank))
    a = np.empty(total)
    for s in range(0, total, 2_000_000):
        e = min(total, s + 2_000_000)
        a[s:e] = np.einsum("ij,ij->i", M[rows[s:e]], N[cols[s:e]]) + rng.normal(0.0, noise, size=e - s)
    a = _round_bf16(a)
    return Workload("large_sparse", m, n, rows, cols, a, float(np.linalg.norm(a)), math.sqrt(m * n / total), tol)


def tiny_dense(m, n, rank, frac, seed, scale=1.0, tau=None, delta=None, tol=1e-4):
    """Small planted problem for unit tests (any shape, any sampling fraction including 1)."""
    rng = np.random.default_rng(seed)
    A = scale * (rng.standard_normal((m, rank)) @ rng.standard_normal((rank, n)))
    count = max(1, int(round(frac * m * n)))
    rows, cols = _sample_lambda(rng, m, n, count)
    a = A[rows, cols]
    tau = 5.0 * math.sqrt(m * n) * scale if tau is None else tau
    delta = 1.2 * m * n / count if delta is None else delta
    return Workload("tiny", m, n, rows, cols, a, tau, delta, tol, A=A)


def heavy_columns(m, n, rank, heavy, base, seed, tau=None, delta=None, tol=1e-4):
    """Planted rank-`rank` problem whose first len(heavy) columns hold heavy[t] observed rows each and
    every other column `base` rows (a sparse pattern with a few very long columns, as in power-law
    degree distributions)."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, rank)) @ rng.standard_normal((rank, n))
    lin = []
    for j in range(n):
        cnt = heavy[j] if j < len(heavy) else base
        rows = rng.choice(m, size=cnt, replace=False)
        lin.append(rows.astype(np.int64) * n + j)
    lin = np.sort(np.concatenate(lin))
    rows, cols = (lin // n).astype(np.int32), (lin % n).astype(np.int32)
    a = A[rows, cols].astype(np.float64)
    tau = 5.0 * math.sqrt(m * n) if tau is None else tau
    delta = 1.2 * m * n / lin.size if delta is None else delta
    return Workload("heavy_columns", m, n, rows, cols, a, tau, delta, tol, A=A)


def by_name(name, **kw):
    return {"planted": planted, "image": image, "ratings": ratings, "image_adjoint": image_adjoint,
            "large_sparse": large_sparse}[name](**kw)
