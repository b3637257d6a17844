"""Pins of the oracle's reverse-mode derivative (frozen-basis convention) on the CPU.

- central finite differences of an independent frozen-basis forward (h = 1e-6, float64)
- torch autograd through an exact SVD for the one-iteration map with a basis spanning R^m
"""
import numpy as np
import pytest

import svt_workloads as W
from oracle import Params, Problem
from oracle.adjoint import forward_record, frozen_forward, grad, svt_vjp


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
