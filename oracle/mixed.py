"""Emulated reduced-precision forms of the oracle (test infrastructure only).

The same steps as svt.svt_step (Alg. 3 / Alg. 4, readings of svt.py), with every
quantity that the mixed form stores in float32 rounded to float32 at the point
where it is stored: the iterate Y and the data a on Lambda, the Gaussian block,
the sampled block X, the basis Q, the projection W = Y^T Q, the factors of X,
the sampled product x, the residual and the updated Y.  Gram matrices, the
Cholesky factors, the small SVD and all norms stay float64.  Products whose
result is stored in float32 are formed in float64 and rounded once; the device
accumulates some of them in float32, which differs from this by accumulation
noise only.  The operator variants of svt.py are the same here: R3SVD from a
fresh t-block in every iteration, the fixed-rank randomized SVD of Alg. 1 and
truncated recycling.

The BF16 form (svt_step_bf16) stores the basis in bfloat16 as well: each sampled block is
orthonormalised in float32 (CholeskyQR2 on the device) and then rounded to bfloat16, round to
nearest even, through float32.  The rounded basis Q^ is no longer orthonormal, so the projected
SVD is taken on the exact orthogonal projector onto span(Q^): with G_Q = Q^T Q^ = L L^T (float64
Cholesky), Q_o = Q^ L^{-T} is orthonormal and B_o = Q_o^T Y = L^{-1} W^T with W = Y^T Q^.
Then ||B_o||_F^2 = trace(L^{-1} W^T W L^{-T}) replaces ||W||_F^2 in the energy of Eq. 10-11,
svd(B_o) the projected SVD of Alg. 3, and the factors of X are Q^ (L^{-T} U_K diag(s - tau)) and
W (L^{-T} U_K diag(1/s)).  The basis is recycled as it is stored (new blocks are appended, the
stored columns never change), since re-rounding a rotated basis would move its span.  Growth
blocks are projected against Q^ with plain CGS2 (X - Q^ Q^T X, twice, in float32): the exact
projector makes the basis orthonormal whatever component in span(Q^) a new block keeps.
"""
import math

import numpy as np

from .philox import omega_block
from .svt import DEP_TOL, DROP_TOL, State, StepInfo


def f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def _orthonormal_block(X, pre_norms):
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
    return f32(Qb)


def _sample_block(Y, seed, it, blk, w, npow):
    X = f32(Y @ f32(omega_block(seed, it, blk, Y.shape[1], w)))
    for _ in range(npow):
        X, _ = np.linalg.qr(X)
        X = f32(Y @ f32(Y.T @ f32(X)))
    return X


def r4svd_mixed(Y, normY, Q, eps_thr, p, it, replay_blocks=None, info=None):
    if Q is None:
        X = _sample_block(Y, p.seed, it, 0, p.t0, p.npow)
        Q = _orthonormal_block(X, np.linalg.norm(X, axis=0))
    W = f32(np.asarray(Y.T @ Q))
    normB = float(np.sum(W * W))
    eps = (normY - normB) / normY
    if eps_thr is None:
        eps_thr = p.eps_thr0 if p.eps_thr0 >= 0 else 0.5 * (1.0 + eps)
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
        for _ in range(2):
            X = f32(X - Q @ (Q.T @ X))
        Qn = _orthonormal_block(X, pre)
        if Qn.shape[1] == 0:
            info.exhausted = True
            break
        Wn = f32(np.asarray(Y.T @ Qn))
        Q = np.hstack([Qn, Q])
        W = np.hstack([Wn, W])
        normB += float(np.sum(Wn * Wn))
        eps = (normY - normB) / normY
        info.eps_hist.append(eps)
    info.blocks = blk
    return Q, W, normB, eps, eps_thr


def svt_step_mixed(prob, p, state, replay=None):
    """One iteration of Alg. 4 in the emulated mixed form; state.y and the basis are float32-valued."""
    p = p.resolved(prob.m, prob.n)
    it = state.it + 1
    info = StepInfo(it=it)
    a = f32(prob.a)
    y = f32(state.y)
    Y = prob.sparse(y)
    normY = float(y @ y)
    # R3SVD / RSVD start every iteration from a fresh sample
    Q0 = None if state.Q is None or p.mode != "r4svd" else f32(state.Q)
    Q, W, normB, eps, eps_thr = r4svd_mixed(Y, normY, Q0, state.eps_thr, p, it,
                                            replay_blocks=None if replay is None else replay[0], info=info)
    info.r, info.eps, info.normY, info.normB, info.Q, info.W = Q.shape[1], eps, normY, normB, Q, W

    U_B, s, VBt = np.linalg.svd(W.T, full_matrices=W.shape[1] > W.shape[0])
    K = np.flatnonzero(s > p.tau)
    if p.mode == "rsvd":
        K = K[K < p.rank]                          # Alg. 1 keeps the `rank` leading triplets
    info.sigma, info.k = s, int(K.size)
    # factors stored in float32: Ut = Q U_K diag(sigma - tau), Vt = W U_K diag(1 / sigma) = V_K
    Ut = f32(Q @ (U_B[:, K] * (s[K] - p.tau)))
    Vt = f32(W @ (U_B[:, K] / s[K]))
    info.U, info.s_minus_tau, info.V = Q @ U_B[:, K], s[K] - p.tau, VBt[K].T
    x = f32(np.einsum("ij,ij->i", Ut[prob.rows], Vt[prob.cols])) if K.size else np.zeros_like(a)
    res = f32(a - x)
    rel = float(np.linalg.norm(res)) / float(np.linalg.norm(a))
    info.x, info.rel = x, rel
    info.mae = float(np.mean(np.abs(res)))

    eps_min = state.eps_min
    target = eps_min * (1.0 - p.eta)
    info.anneal_margin = (rel - target) / eps_min if math.isfinite(eps_min) else -math.inf
    annealed = (rel >= target) if replay is None else bool(replay[1])
    if annealed:
        eps_thr = p.beta * eps_thr
    else:
        eps_min = rel
    info.annealed = annealed

    # recycle U_L: all r columns, or the leading k + recycle_extra (truncated recycling)
    U_L = f32(Q @ U_B)
    keep = U_L.shape[1] if p.recycle_extra < 0 else min(U_L.shape[1], info.k + p.recycle_extra)
    new = State(it=it, y=y.copy(), Q=U_L[:, :keep] if keep > 0 else None, eps_thr=eps_thr, eps_min=eps_min)
    if rel < p.tol or (p.mae_tol > 0 and info.mae < p.mae_tol):
        info.stopped = True
        return new, info
    delta32 = float(np.float32(p.delta))
    new.y = f32(y + delta32 * res)
    return new, info


# ----------------------------------------------------------------------------------------------
# BF16 basis with the exact projector onto its span
# ----------------------------------------------------------------------------------------------

def bf16(x):
    """Round to the nearest bfloat16, ties to even, through float32 (finite values)."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def projected_energy(Qh, W):
    """(L, ||B_o||_F^2) for the stored basis Q^ and W = Y^T Q^: L = chol(Q^T Q^), B_o = L^{-1} W^T."""
    L = np.linalg.cholesky(Qh.T @ Qh)
    Bo = np.linalg.solve(L, W.T)
    return L, float(np.sum(Bo * Bo))


def r4svd_bf16(Y, normY, Qh, eps_thr, p, it, replay_blocks=None, info=None):
    if Qh is None:
        X = _sample_block(Y, p.seed, it, 0, p.t0, p.npow)
        Qh = bf16(_orthonormal_block(X, np.linalg.norm(X, axis=0)))
    W = f32(np.asarray(Y.T @ Qh))
    _, normB = projected_energy(Qh, W)
    eps = (normY - normB) / normY
    if eps_thr is None:
        eps_thr = p.eps_thr0 if p.eps_thr0 >= 0 else 0.5 * (1.0 + eps)
    info.eps_thr_used = eps_thr
    info.eps_hist.append(eps)
    blk = 0
    while p.mode != "rsvd":
        r = Qh.shape[1]
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
        for _ in range(2):
            X = f32(X - Qh @ (Qh.T @ X))
        Qn = _orthonormal_block(X, pre)
        if Qn.shape[1] == 0:
            info.exhausted = True
            break
        Qn = bf16(Qn)
        Qh = np.hstack([Qh, Qn])                      # appended after the stored columns
        W = np.hstack([W, f32(np.asarray(Y.T @ Qn))])
        _, normB = projected_energy(Qh, W)
        eps = (normY - normB) / normY
        info.eps_hist.append(eps)
    info.blocks = blk
    return Qh, W, normB, eps, eps_thr


def svt_step_bf16(prob, p, state, replay=None):
    """One iteration of Alg. 4 in the emulated BF16 form (float32 iterate and factors, bfloat16 basis,
    float64 Gram, Cholesky and projected SVD); state.Q is the stored basis Q^."""
    p = p.resolved(prob.m, prob.n)
    if p.recycle_extra >= 0:
        raise ValueError("the BF16 form recycles the whole stored basis (no truncated recycling)")
    it = state.it + 1
    info = StepInfo(it=it)
    a = f32(prob.a)
    y = f32(state.y)
    Y = prob.sparse(y)
    normY = float(y @ y)
    Q0 = None if state.Q is None or p.mode != "r4svd" else bf16(state.Q)
    Qh, W, normB, eps, eps_thr = r4svd_bf16(Y, normY, Q0, state.eps_thr, p, it,
                                            replay_blocks=None if replay is None else replay[0], info=info)
    info.r, info.eps, info.normY, info.normB, info.Q, info.W = Qh.shape[1], eps, normY, normB, Qh, W

    L, _ = projected_energy(Qh, W)
    Bo = np.linalg.solve(L, W.T)                       # B_o = L^{-1} W^T = Q_o^T Y
    U_B, s, VBt = np.linalg.svd(Bo, full_matrices=Bo.shape[0] > Bo.shape[1])
    K = np.flatnonzero(s > p.tau)
    if p.mode == "rsvd":
        K = K[K < p.rank]
    info.sigma, info.k = s, int(K.size)
    LiT_U = np.linalg.solve(L.T, U_B[:, K])            # L^{-T} U_K
    Ut = f32(Qh @ (LiT_U * (s[K] - p.tau)))
    Vt = f32(W @ (LiT_U / s[K]))
    info.U, info.s_minus_tau, info.V = Qh @ LiT_U, s[K] - p.tau, VBt[K].T
    x = f32(np.einsum("ij,ij->i", Ut[prob.rows], Vt[prob.cols])) if K.size else np.zeros_like(a)
    res = f32(a - x)
    rel = float(np.linalg.norm(res)) / float(np.linalg.norm(a))
    info.x, info.rel = x, rel
    info.mae = float(np.mean(np.abs(res)))

    eps_min = state.eps_min
    target = eps_min * (1.0 - p.eta)
    info.anneal_margin = (rel - target) / eps_min if math.isfinite(eps_min) else -math.inf
    annealed = (rel >= target) if replay is None else bool(replay[1])
    if annealed:
        eps_thr = p.beta * eps_thr
    else:
        eps_min = rel
    info.annealed = annealed

    new = State(it=it, y=y.copy(), Q=Qh, eps_thr=eps_thr, eps_min=eps_min)
    if rel < p.tol or (p.mae_tol > 0 and info.mae < p.mae_tol):
        info.stopped = True
        return new, info
    delta32 = float(np.float32(p.delta))
    new.y = f32(y + delta32 * res)
    return new, info
