"""Reverse-mode derivative of T unrolled SVT iterations (test infrastructure only).

Convention (frozen basis): iteration i maps Y_i to X_i = Q_i D_tau(Q_i^T Y_i) with the basis
Q_i of the forward run and every discrete decision (kicking count k0, growth blocks,
annealing, the thresholded set K) held fixed; the dual update Y_{i+1} = Y_i + delta
P_Lambda(A - X_i) (Eq. 4) and the kicking start Y_1 = k0 delta P_Lambda(A) (Alg. 4
initialisation) are differentiated exactly.  The loss is a function of X_T on a held-out set
H; its gradient g_H = dL/dX_T on H is the input.

The derivative of the singular value thresholding map B -> U f(S) V^T with f(s) = (s - tau)_+
is the one of spectral functions of rectangular matrices (Lewis and Sendov; used for the SVT
operator by Candes, Sing-Long and Trzasko, 2013): with M = U^T Bbar V in the full SVD basis,
  Cbar_ij = (a_ij + b_ij)/2 M_ij + (a_ij - b_ij)/2 M_ji,  i != j <= r,
  Cbar_ii = f'(s_i) M_ii,   Cbar_ij = f(s_i)/s_i M_ij,  j > r,
  a_ij = (f_i - f_j)/(s_i - s_j),  b_ij = (f_i + f_j)/(s_i + s_j),
and the adjoint is U Cbar V^T.  dX/dtau = -Q U_K V_K^T.  This module writes that out with a
full numpy SVD per iteration.

grad_exact drops the frozen basis: it differentiates the unrolled iteration as R4SVD computes it
(Alg. 2-3 with every discrete decision held fixed), including how the basis depends on the
iterates.  With P_i the orthogonal projector onto span(Q_i), iteration i computes X_i =
D_tau(P_i Y_i), and the projector is built by appending sampled blocks (Alg. 3): starting from the
recycled P_{i-1} (the empty projector before the first iteration), each block gives
Z = (I - P) Y_i Omega and P <- P + Z (Z^T Z)^{-1} Z^T.  The reverse sweep carries the cotangent of
the recycled projector from iteration to iteration.  For Pz = Z (Z^T Z)^{-1} Z^T the adjoint in Z
of <Pbar, Pz> is (I - Pz)(Pbar + Pbar^T) Z (Z^T Z)^{-1}.
"""
import numpy as np

from .philox import omega_block
from .svt import Params, Problem, dense, initial_state, svt_step


def forward_record(prob, p, T, replay=None):
    """Run T iterations of the oracle; return the bases Q_i (as used by R4SVD in iteration i),
    the iterates y_i, the decisions and k0."""
    state, k0 = initial_state(prob, p)
    ys, Qs, decisions = [], [], []
    for i in range(T):
        ys.append(state.y.copy())
        rp = None if replay is None else replay[i]
        state, info = svt_step(prob, p, state, rp)
        Qs.append(info.Q.copy())
        decisions.append((info.blocks, info.annealed))
        if info.stopped and i < T - 1:
            raise ValueError("the forward run converged before T iterations; use a smaller T")
    return dict(ys=ys, Qs=Qs, decisions=decisions, k0=k0, final_info=info)


def frozen_x(prob, Q, y, tau):
    """X = Q D_tau(Q^T Y) as a dense matrix (the frozen-basis map of one iteration)."""
    B = Q.T @ dense(prob.m, prob.n, prob.rows, prob.cols, y)
    U, s, Vt = np.linalg.svd(B, full_matrices=False)
    K = s > tau
    return Q @ ((U[:, K] * (s[K] - tau)) @ Vt[K])


def frozen_forward(prob, a, tau, delta, k0, Qs, hr, hc):
    """T iterations of the frozen-basis map from Y_1 = k0 delta a; returns X_T on (hr, hc)."""
    y = k0 * delta * np.asarray(a, dtype=np.float64)
    X = None
    for i, Q in enumerate(Qs):
        X = frozen_x(prob, Q, y, tau)
        if i + 1 < len(Qs):
            y = y + delta * (a - X[prob.rows, prob.cols])
    return X[hr, hc]


def svt_vjp(Q, Y, tau, Xbar):
    """Adjoint of Y -> Q D_tau(Q^T Y) at Y (dense), applied to the cotangent Xbar (dense m x n).
    Returns (Ybar dense, tau_bar).  The coefficients Cbar of the module docstring are formed for
    all (i, j) at once (array expressions of the same case split)."""
    B = Q.T @ Y
    r, n = B.shape
    U, s, Vt = np.linalg.svd(B, full_matrices=True)  # U r x r, Vt n x n
    V = Vt.T
    ns = min(r, n)
    sig = s[:ns]
    f = np.maximum(sig - tau, 0.0)
    fp = (sig > tau).astype(float)
    Bbar = Q.T @ Xbar
    M = U.T @ Bbar @ V  # r x n
    Cbar = np.zeros_like(M)
    # the leading ns x ns block: divided differences of f over the singular values
    si, sj = sig[:, None], sig[None, :]
    fi, fj = f[:, None], f[None, :]
    same = si == sj
    with np.errstate(divide="ignore", invalid="ignore"):
        a = np.where(same, np.broadcast_to(fp[:, None], same.shape), (fi - fj) / np.where(same, 1.0, si - sj))
        pos = (si + sj) > 0
        b = np.where(pos, (fi + fj) / np.where(pos, si + sj, 1.0), 0.0)
    Ms = M[:ns, :ns]
    C = 0.5 * (a + b) * Ms + 0.5 * (a - b) * Ms.T
    np.fill_diagonal(C, fp * np.diag(Ms))
    Cbar[:ns, :ns] = C
    with np.errstate(divide="ignore", invalid="ignore"):
        fs = np.where(sig > 0, f / np.where(sig > 0, sig, 1.0), 0.0)
    if n > ns:   # right complement of the row space (n > r)
        Cbar[:ns, ns:] = fs[:, None] * M[:ns, ns:]
    if r > ns:   # left complement of the column space (r > n)
        Cbar[ns:, :ns] = fs[None, :] * M[ns:, :ns]
    Ybar = Q @ (U @ Cbar @ V.T)
    tau_bar = -float(np.sum(np.diag(Ms)[sig > tau]))
    return Ybar, tau_bar


def grad(prob, p, rec, hr, hc, gx_h):
    """dL/dtau, dL/ddelta, dL/da on Lambda for L with dL/dX_T = gx_h on (hr, hc), frozen basis."""
    a = prob.a
    tau, delta, k0 = p.tau, p.delta, rec["k0"]
    Qs = rec["Qs"]
    T = len(Qs)
    # recompute the y_i of the frozen forward (identical to the recorded ones)
    ys = [k0 * delta * a.copy()]
    xs = []
    for i in range(T):
        X = frozen_x(prob, Qs[i], ys[i], tau)
        xs.append(X[prob.rows, prob.cols])
        if i + 1 < T:
            ys.append(ys[i] + delta * (a - xs[i]))
    Xbar = np.zeros((prob.m, prob.n))
    np.add.at(Xbar, (hr, hc), gx_h)
    a_bar = np.zeros_like(a)
    d_bar = 0.0
    t_bar = 0.0
    ybar = None
    for i in range(T - 1, -1, -1):
        if i < T - 1:
            # y_{i+1} = y_i + delta (a - x_i)
            a_bar += delta * ybar
            d_bar += float(ybar @ (a - xs[i]))
            Xbar = np.zeros((prob.m, prob.n))
            Xbar[prob.rows, prob.cols] = -delta * ybar
        Yd = dense(prob.m, prob.n, prob.rows, prob.cols, ys[i])
        Ybar_d, tb = svt_vjp(Qs[i], Yd, tau, Xbar)
        t_bar += tb
        yb_i = Ybar_d[prob.rows, prob.cols]
        ybar = yb_i if i == T - 1 else ybar + yb_i
    # y_1 = k0 delta a
    a_bar += k0 * delta * ybar
    d_bar += k0 * float(ybar @ a)
    return t_bar, d_bar, a_bar


def _block_plan(prob, p, rec):
    """(blk, width) of the sampled blocks appended in each iteration: the t-block (blk 0) in the
    first one, then the growth blocks of Alg. 3 (width min(dt, r_max - r)).  Raises when the run
    dropped columns (the basis widths then differ from the plan)."""
    pr = p.resolved(prob.m, prob.n)
    if pr.mode != "r4svd" or pr.npow != 0:
        raise ValueError("grad_exact covers R4SVD without power iterations")
    plan, r = [], 0
    for i, (blocks, _) in enumerate(rec["decisions"]):
        cur = []
        if i == 0:
            cur.append((0, pr.t0))
            r = pr.t0
        for b in range(1, blocks + 1):
            w = min(pr.dt, pr.r_max - r)
            cur.append((b, w))
            r += w
        if r != rec["Qs"][i].shape[1]:
            raise ValueError(f"iteration {i + 1}: the basis width {rec['Qs'][i].shape[1]} differs from the plan {r}")
        plan.append(cur)
    return plan


def grad_exact(prob, p, rec, hr, hc, gx_h):
    """dL/dtau, dL/ddelta, dL/da through the unrolled R4SVD iteration itself (basis included), with
    the decisions of the recorded run held fixed; dL/dX_T = gx_h on (hr, hc)."""
    a, m, n = prob.a, prob.m, prob.n
    tau, delta, k0 = p.tau, p.delta, rec["k0"]
    T = len(rec["Qs"])
    plan = _block_plan(prob, p, rec)
    eye = np.eye(m)
    # forward: iterates, projectors, and the blocks (Z, Omega, projector before the block)
    ys, Ps, blocks, xs = [k0 * delta * a.copy()], [], [], []
    P = np.zeros((m, m))
    for i in range(T):
        Yd = dense(m, n, prob.rows, prob.cols, ys[i])
        cur = []
        for blk, w in plan[i]:
            Om = omega_block(p.seed, i + 1, blk, n, w)
            Z = (eye - P) @ (Yd @ Om)
            Qz, Rz = np.linalg.qr(Z)
            cur.append((Om, Z, Qz, Rz, P.copy()))
            P = P + Qz @ Qz.T
        Ps.append(P.copy())
        blocks.append(cur)
        X = d_tau_dense(P @ Yd, tau)
        xs.append(X[prob.rows, prob.cols])
        if i + 1 < T:
            ys.append(ys[i] + delta * (a - xs[i]))
    # reverse
    Xbar = np.zeros((m, n))
    np.add.at(Xbar, (hr, hc), gx_h)
    a_bar, d_bar, t_bar = np.zeros_like(a), 0.0, 0.0
    Pbar = np.zeros((m, m))
    ybar = None
    for i in range(T - 1, -1, -1):
        if i < T - 1:
            a_bar += delta * ybar
            d_bar += float(ybar @ (a - xs[i]))
            Xbar = np.zeros((m, n))
            Xbar[prob.rows, prob.cols] = -delta * ybar
        Yd = dense(m, n, prob.rows, prob.cols, ys[i])
        Mbar, tb = svt_vjp(eye, Ps[i] @ Yd, tau, Xbar)   # X_i = D_tau(M), M = P_i Y_i
        t_bar += tb
        Ybar = Ps[i] @ Mbar
        Pbar = Pbar + Mbar @ Yd.T
        for Om, Z, Qz, Rz, Pb in reversed(blocks[i]):
            Pz = Qz @ Qz.T
            Zbar = (eye - Pz) @ (Pbar + Pbar.T) @ np.linalg.solve(Rz, Qz.T).T   # (I - Pz)(Pbar + Pbar^T) Z (Z^T Z)^{-1}
            Ybar = Ybar + ((eye - Pb) @ Zbar) @ Om.T
            Pbar = Pbar - Zbar @ (Yd @ Om).T
        yb_i = Ybar[prob.rows, prob.cols]
        ybar = yb_i if i == T - 1 else ybar + yb_i
    a_bar += k0 * delta * ybar
    d_bar += k0 * float(ybar @ a)
    return t_bar, d_bar, a_bar


def d_tau_dense(M, tau):
    """D_tau of a dense matrix (Eq. 5) by a full SVD."""
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    K = s > tau
    return (U[:, K] * (s[K] - tau)) @ Vt[K]
