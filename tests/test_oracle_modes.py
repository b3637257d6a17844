"""Pins of the oracle's operator variants: R3SVD in every iteration (no recycling), the
fixed-rank randomized SVD of Alg. 1, truncated recycling, and the sample MAE of Sec. 3 with its
stop rule.  Each pin checks a property that the paper or the mathematics fixes, not a retyped
formula.
"""
from dataclasses import replace

import numpy as np

import svt_workloads as W
from oracle import Params, Problem, d_tau, dense, initial_state, svt_run, svt_step


def _prob(w):
    return Problem(w.m, w.n, w.rows, w.cols, w.a)


def _range_residual(Y, Q):
    """Largest component of the columns of Q outside range(Y)."""
    U, s, _ = np.linalg.svd(Y, full_matrices=False)
    U = U[:, s > 1e-12 * s[0]]
    return float(np.abs(Q - U @ (U.T @ Q)).max())


def test_r3svd_basis_lies_in_the_range_of_the_current_iterate():
    """Without recycling every basis is built from products with the current Y (Alg. 2), so it lies
    in range(Y); a recycled basis (Alg. 3) carries directions of earlier iterates and does not."""
    w = W.tiny_dense(40, 12, 2, 0.5, seed=81)
    prob = _prob(w)
    for mode, expect_inside in (("r3svd", True), ("r4svd", False)):
        p = Params(tau=w.tau, delta=w.delta, seed=81, t0=4, dt=3, mode=mode)
        state, _ = initial_state(prob, p)
        worst = 0.0
        for i in range(5):
            Y = dense(prob.m, prob.n, prob.rows, prob.cols, state.y)
            state, info = svt_step(prob, p, state)
            if i >= 1:
                worst = max(worst, _range_residual(Y, info.Q))
        if expect_inside:
            assert worst <= 1e-10, (mode, worst)
        else:
            assert worst > 1e-6, (mode, worst)


def test_r3svd_first_iteration_equals_r4svd():
    w = W.tiny_dense(50, 40, 3, 0.4, seed=82)
    prob = _prob(w)
    p4 = Params(tau=w.tau, delta=w.delta, seed=82)
    _, i4 = svt_step(prob, p4, initial_state(prob, p4)[0])
    _, i3 = svt_step(prob, replace(p4, mode="r3svd"), initial_state(prob, p4)[0])
    assert np.array_equal(i4.x, i3.x) and i4.r == i3.r and i4.k == i3.k


def test_r3svd_reduces_to_exact_svt():
    """eps_thr = 0 on a square problem: the fresh basis spans R^m each time, so every iterate is
    SVT with an exact D_tau (Eq. 4-5)."""
    w = W.tiny_dense(14, 14, 2, 0.6, seed=83)
    prob = _prob(w)
    p = Params(tau=w.tau, delta=w.delta, seed=83, t0=4, dt=3, eps_thr0=0.0, mode="r3svd")
    state, _ = initial_state(prob, p)
    for _ in range(6):
        y = state.y.copy()
        state, info = svt_step(prob, p, state)
        ref = d_tau(dense(prob.m, prob.n, prob.rows, prob.cols, y), p.tau)[prob.rows, prob.cols]
        assert np.abs(info.x - ref).max() <= 1e-10 * max(np.abs(ref).max(), 1.0)


def _full_problem(rank, seed, m=18, n=15):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, rank)) @ rng.standard_normal((rank, n))
    rows, cols = np.divmod(np.arange(m * n), n)
    return Problem(m, n, rows, cols, A[rows, cols]), A


def test_rsvd_is_exact_when_the_sample_spans_the_range():
    """Alg. 1 with rank + p at least rank(Y): range(Y Omega) = range(Y) (Gaussian Omega), so the
    projected SVD is the exact SVD of Y; with Lambda = everything, X = D_tau(Y) restricted to the
    `rank` leading triplets."""
    prob, A = _full_problem(6, 84)
    s_all = np.linalg.svd(A, compute_uv=False)
    tau = 0.5 * s_all[5]                            # all six singular values of Y = A sit above tau
    for rank, over in ((6, 2), (3, 4)):
        p = Params(tau=tau, delta=1.0, seed=84, k0=1, mode="rsvd", rank=rank, oversample=over)
        state, _ = initial_state(prob, p)
        _, info = svt_step(prob, p, state)
        U, s, Vt = np.linalg.svd(A, full_matrices=False)
        ref = (U[:, :rank] * (s[:rank] - tau)) @ Vt[:rank]
        assert info.k == rank
        assert info.r == min(rank + over, 6)          # columns beyond rank(Y) = 6 are dependent and drop (S5)
        assert np.abs(info.x - ref[prob.rows, prob.cols]).max() <= 1e-10 * np.abs(ref).max()


def test_truncated_recycling():
    """recycle_extra >= r keeps the whole basis (the R4SVD trajectory bit for bit); recycle_extra = e
    keeps exactly the k + e leading left singular vectors of B (U_L of Alg. 3)."""
    w = W.tiny_dense(60, 45, 3, 0.4, seed=85)
    prob = _prob(w)
    p = Params(tau=w.tau, delta=w.delta, seed=85, maxit=8)
    _, full, k0 = svt_run(prob, p, keep_infos=True)
    _, big, _ = svt_run(prob, replace(p, recycle_extra=10_000), keep_infos=True)
    for a, b in zip(full, big):
        assert np.array_equal(a.x, b.x) and a.r == b.r
    pt = replace(p, recycle_extra=2)
    state, _ = initial_state(prob, pt)
    for _ in range(6):
        state, info = svt_step(prob, pt, state)
        keep = min(info.r, info.k + 2)
        assert state.Q.shape[1] == keep
        B = info.Q.T @ dense(prob.m, prob.n, prob.rows, prob.cols, state.y if info.stopped else
                             state.y - pt.delta * (prob.a - info.x))
        Ub, sb, _ = np.linalg.svd(B, full_matrices=False)
        top = info.Q @ Ub[:, :keep]
        # same span as the keep leading left singular vectors (principal angles ~ 0)
        cos = np.linalg.svd(top.T @ state.Q, compute_uv=False)
        assert np.abs(cos - 1.0).max() <= 1e-10


def test_sample_mae_and_its_stop_rule():
    """With tau above every singular value X = 0, so the sample MAE of Sec. 3 is mean |a|; it never
    exceeds the RMS residual; the MAE stop rule fires exactly when the MAE is below mae_tol."""
    w = W.tiny_dense(30, 25, 2, 0.5, seed=86)
    prob = _prob(w)
    p = Params(tau=1e9, delta=w.delta, seed=86, k0=1, tol=0.0)
    state, _ = initial_state(prob, p)
    _, info = svt_step(prob, p, state)
    assert info.k == 0 and info.mae == np.mean(np.abs(prob.a))
    p = Params(tau=w.tau, delta=w.delta, seed=86, tol=0.0, maxit=12)
    _, infos, _ = svt_run(prob, p, keep_infos=True)
    for inf in infos:
        assert inf.mae <= inf.rel * prob.norm_a / np.sqrt(prob.a.size) * (1 + 1e-12)
    target = infos[5].mae * 1.000001
    _, infos2, _ = svt_run(prob, replace(p, mae_tol=target), keep_infos=True)
    first = next(i for i, inf in enumerate(infos) if inf.mae < target)
    assert len(infos2) == first + 1 and infos2[-1].stopped
