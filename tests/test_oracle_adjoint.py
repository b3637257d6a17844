"""Pins of the oracle's reverse-mode derivatives on the CPU.

Frozen-basis convention (grad):
- central finite differences of an independent frozen-basis forward (h = 1e-6, float64)
- torch autograd through an exact SVD for the one-iteration map with a basis spanning R^m

Exact derivative of the unrolled iteration (grad_exact, basis construction included):
- central finite differences (h = 1e-6, float64) of the oracle's own SVT iteration (svt_step,
  R4SVD bases recomputed from the perturbed iterates, the recorded decisions replayed)
"""
import numpy as np
import pytest

import svt_workloads as W
from oracle import Params, Problem, initial_state, svt_step
from oracle.adjoint import forward_record, frozen_forward, grad, grad_exact, svt_vjp


def _setup(T=6, seed=71):
    w = W.tiny_dense(36, 30, 2, 0.5, seed=seed)
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=seed, t0=3, dt=4)
    rec = forward_record(prob, p, T)
    rng = np.random.default_rng(seed)
    free = np.setdiff1d(np.arange(w.m * w.n), w.rows.astype(np.int64) * w.n + w.cols)
    h = np.sort(rng.choice(free, 40, replace=False))
    hr, hc = h // w.n, h % w.n
    g = rng.standard_normal(h.size)
    return w, prob, p, rec, hr, hc, g


def test_frozen_forward_reproduces_the_run():
    w, prob, p, rec, hr, hc, g = _setup()
    x_frozen = frozen_forward(prob, prob.a, p.tau, p.delta, rec["k0"], rec["Qs"], w.rows, w.cols)
    np.testing.assert_allclose(x_frozen, rec["final_info"].x, rtol=0, atol=1e-10 * np.abs(rec["final_info"].x).max())


def test_adjoint_matches_central_differences():
    w, prob, p, rec, hr, hc, g = _setup()
    tb, db, ab = grad(prob, p, rec, hr, hc, g)

    def L(a, tau, delta):
        return float(g @ frozen_forward(prob, a, tau, delta, rec["k0"], rec["Qs"], hr, hc))

    h = 1e-6
    fd_tau = (L(prob.a, p.tau * (1 + h), p.delta) - L(prob.a, p.tau * (1 - h), p.delta)) / (2 * h * p.tau)
    fd_delta = (L(prob.a, p.tau, p.delta * (1 + h)) - L(prob.a, p.tau, p.delta * (1 - h))) / (2 * h * p.delta)
    assert abs(tb - fd_tau) <= 1e-6 * max(abs(fd_tau), 1e-3 * abs(L(prob.a, p.tau, p.delta)))
    assert abs(db - fd_delta) <= 1e-6 * max(abs(fd_delta), 1e-3 * abs(L(prob.a, p.tau, p.delta)))
    rng = np.random.default_rng(5)
    scale = np.abs(prob.a).max()
    for _ in range(3):
        v = rng.standard_normal(prob.a.size)
        fd = (L(prob.a + h * scale * v, p.tau, p.delta) - L(prob.a - h * scale * v, p.tau, p.delta)) / (2 * h * scale)
        assert abs(ab @ v - fd) <= 1e-6 * max(abs(fd), np.linalg.norm(ab) * 1e-3)
    for c in rng.choice(prob.a.size, 5, replace=False):
        e = np.zeros_like(prob.a)
        e[c] = 1.0
        fd = (L(prob.a + h * scale * e, p.tau, p.delta) - L(prob.a - h * scale * e, p.tau, p.delta)) / (2 * h * scale)
        assert abs(ab[c] - fd) <= 1e-5 * max(abs(fd), np.abs(ab).max() * 1e-3)


def test_svt_vjp_matches_torch_autograd_exact_svt():
    """With Q spanning R^m the frozen-basis map is exact SVT; torch differentiates an SVD independently."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    m, n = 9, 7
    Y = rng.standard_normal((m, n)) * 3.0
    tau = 2.5
    Q = np.linalg.qr(rng.standard_normal((m, m)))[0]
    Xbar = rng.standard_normal((m, n))
    Ybar, tb = svt_vjp(Q, Y, tau, Xbar)

    Yt = torch.tensor(Y, dtype=torch.float64, requires_grad=True)
    tt = torch.tensor(tau, dtype=torch.float64, requires_grad=True)
    U, S, Vh = torch.linalg.svd(Yt, full_matrices=False)
    X = U @ torch.diag(torch.clamp(S - tt, min=0.0)) @ Vh
    (X * torch.tensor(Xbar)).sum().backward()
    np.testing.assert_allclose(Ybar, Yt.grad.numpy(), rtol=0, atol=1e-10 * np.abs(Ybar).max())
    assert abs(tb - tt.grad.item()) <= 1e-10 * max(1.0, abs(tb))


EXACT_CASES = [
    # (m, n, rank, frac, seed, extra params, T): growth blocks in late and in every iteration
    (90, 70, 3, 0.4, 31, {}, 8),
    (60, 50, 4, 0.5, 77, {"t0": 3, "dt": 5, "eps_thr0": 0.05}, 6),
    (36, 30, 2, 0.5, 71, {"t0": 3, "dt": 4}, 6),
]


def _real_loss(w, prob, p, rec, hr, hc, g, T):
    """L = <g, X_T on H> of T steps of the oracle itself with the recorded decisions replayed."""
    def L(tau, delta, a):
        pp = Params(**{**p.__dict__, "tau": tau, "delta": delta, "k0": rec["k0"]})
        pr = Problem(w.m, w.n, w.rows, w.cols, a)
        st, _ = initial_state(pr, pp)
        for i in range(T):
            st, info = svt_step(pr, pp, st, rec["decisions"][i])
        X = (info.U * info.s_minus_tau) @ info.V.T if info.k > 0 else np.zeros((w.m, w.n))
        return float(g @ X[hr, hc])
    return L


@pytest.mark.parametrize("m,n,rank,frac,seed,extra,T", EXACT_CASES)
def test_exact_adjoint_matches_differences_of_the_real_iteration(m, n, rank, frac, seed, extra, T):
    w = W.tiny_dense(m, n, rank, frac, seed=seed)
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=seed, tol=0.0, **extra)
    rec = forward_record(prob, p, T)
    rng = np.random.default_rng(seed + 1000)
    free = np.setdiff1d(np.arange(m * n), w.rows.astype(np.int64) * n + w.cols)
    hsel = np.sort(rng.choice(free, 40, replace=False))
    hr, hc = hsel // n, hsel % n
    g = rng.standard_normal(hsel.size)
    te, de, ae = grad_exact(prob, p, rec, hr, hc, g)
    L = _real_loss(w, prob, p, rec, hr, hc, g, T)
    h = 1e-6
    ft = (L(p.tau * (1 + h), p.delta, prob.a) - L(p.tau * (1 - h), p.delta, prob.a)) / (2 * h * p.tau)
    fd = (L(p.tau, p.delta * (1 + h), prob.a) - L(p.tau, p.delta * (1 - h), prob.a)) / (2 * h * p.delta)
    assert abs(te - ft) <= 1e-6 * abs(ft), (te, ft)
    assert abs(de - fd) <= 1e-6 * abs(fd), (de, fd)
    scale = np.abs(prob.a).max()
    for v in np.random.default_rng(3).standard_normal((2, prob.a.size)):
        fa = (L(p.tau, p.delta, prob.a + h * scale * v) - L(p.tau, p.delta, prob.a - h * scale * v)) / (2 * h * scale)
        assert abs(ae @ v - fa) <= 1e-6 * max(abs(fa), 1e-3 * np.linalg.norm(ae)), (ae @ v, fa)


def test_frozen_basis_misses_the_basis_dependence():
    """Where growth blocks are sampled from the iterate, the frozen-basis gradient is not the
    derivative of the iteration (it drops d span(Q_i) / d Y); the exact one is.  Without growth
    after a first block that only depends on Y_1 = k0 delta a (the second case), the two agree
    in tau and delta."""
    out = []
    for (m, n, rank, frac, seed, extra, T) in EXACT_CASES[:1] + EXACT_CASES[2:]:
        w = W.tiny_dense(m, n, rank, frac, seed=seed)
        prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
        p = Params(tau=w.tau, delta=w.delta, seed=seed, tol=0.0, **extra)
        rec = forward_record(prob, p, T)
        rng = np.random.default_rng(seed + 1000)
        free = np.setdiff1d(np.arange(m * n), w.rows.astype(np.int64) * n + w.cols)
        hsel = np.sort(rng.choice(free, 40, replace=False))
        g = rng.standard_normal(hsel.size)
        tf, df, _ = grad(prob, p, rec, hsel // n, hsel % n, g)
        te, de, _ = grad_exact(prob, p, rec, hsel // n, hsel % n, g)
        out.append((abs(tf - te) / abs(te), abs(df - de) / abs(de)))
    assert out[0][0] > 0.1 and out[0][1] > 0.1      # 90 x 70: a growth block in iteration 8
    assert out[1][0] < 1e-8 and out[1][1] < 1e-8    # 36 x 30: the basis is the first block's
