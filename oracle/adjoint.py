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
full numpy SVD (small problems only).
"""
import numpy as np

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
    Returns (Ybar dense, tau_bar)."""
    B = Q.T @ Y
    r, n = B.shape
    U, s, Vt = np.linalg.svd(B, full_matrices=True)  # U r x r, Vt n x n
    V = Vt.T
    ns = min(r, n)
    sig = np.zeros(r)
    sig[:ns] = s
    f = np.maximum(sig - tau, 0.0)
    fp = (sig > tau).astype(float)
    Bbar = Q.T @ Xbar
    M = U.T @ Bbar @ V  # r x n
    Cbar = np.zeros_like(M)
    for i in range(r):
        for j in range(n):
            if i < ns and j < ns:
                if i == j:
                    Cbar[i, j] = fp[i] * M[i, j]
                    continue
                si, sj, fi, fj = sig[i], sig[j], f[i], f[j]
                a = (fi - fj) / (si - sj) if si != sj else fp[i]
                b = (fi + fj) / (si + sj) if si + sj > 0 else 0.0
                Cbar[i, j] = 0.5 * (a + b) * M[i, j] + 0.5 * (a - b) * M[j, i]
            elif i < ns:   # right complement of the row space (n > r)
                Cbar[i, j] = f[i] / sig[i] * M[i, j] if sig[i] > 0 else 0.0
            elif j < ns:   # left complement of the column space (r > n)
                Cbar[i, j] = f[j] / sig[j] * M[i, j] if sig[j] > 0 else 0.0
    Ybar = Q @ (U @ Cbar @ V.T)
    tau_bar = -float(sum(M[i, i] for i in range(ns) if sig[i] > tau))
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
