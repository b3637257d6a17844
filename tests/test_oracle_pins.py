"""Pins of the FP64 oracle against facts fixed by the paper and by linear algebra (CPU only).

Each test names the passage of Li & Yu it pins.  None of them re-types the
oracle's formula: they check closed forms built without an SVD, invariants,
special cases that reduce to exact SVT, brute force on tiny inputs, and
published known-answer vectors.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.stats as st

import svt_workloads as W
from oracle import (Params, Problem, State, d_tau, dense, initial_state, kicking_k0, philox4x64_10,
                    philox4x64_10_array, r4svd, spectral_norm, svt_exact_run, svt_exact_step, svt_run, svt_step)
from oracle.philox import omega_block, omega_block_scalar
from oracle.svt import StepInfo

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _orth(rng, m, k):
    q, _ = np.linalg.qr(rng.standard_normal((m, k)))
    return q


def _planted_dense(rng, m, n, s):
    """Y = U diag(s) V^T with orthonormal U, V drawn independently of any SVD routine."""
    k = len(s)
    U, V = _orth(rng, m, k), _orth(rng, n, k)
    return U, V, (U * s) @ V.T


# ---------------------------------------------------------------------------- RNG (Omega stream)

def test_philox_known_answers():
    """Philox4x64-10 against the published Random123 known-answer vectors."""
    with open(os.path.join(GOLDEN, "philox4x64_10_kat.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert philox4x64_10(v[0:4], v[4:6]) == tuple(v[6:10])
        arr = philox4x64_10_array([v[0]], [v[1]], [v[2]], [v[3]], v[4], v[5])
        assert tuple(int(a[0]) for a in arr) == tuple(v[6:10])


def test_philox_matches_numpy_bitgen():
    """numpy's Philox bit generator increments its counter before each block; output at c+1 equals ours at c+1."""
    for key, c in [((123, 456), 5), ((2**63 + 7, 1), 2**40), ((0, 0), 0)]:
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array([c, 0, 0, 0], dtype=np.uint64))
        raw = bg.random_raw(8)
        assert philox4x64_10((c + 1, 0, 0, 0), key) == tuple(int(x) for x in raw[:4])
        assert philox4x64_10((c + 2, 0, 0, 0), key) == tuple(int(x) for x in raw[4:])


def test_omega_block_is_standard_gaussian_and_layout_stable():
    z = omega_block(9, 3, 1, 4000, 10)
    assert z.shape == (4000, 10)
    # Kolmogorov-Smirnov against N(0,1): a dropped sqrt(-2 ln u) factor or a wrong angle fails this.
    assert st.kstest(z.ravel(), "norm").pvalue > 1e-3
    # columns are independent (no cos/sin pairing artefact)
    c = np.corrcoef(z.T)
    assert np.abs(c - np.eye(10)).max() < 0.06
    # the vectorised form equals the element-by-element form; widths share a prefix
    zs = omega_block_scalar(9, 3, 1, 40, 10)
    np.testing.assert_allclose(z[:40], zs, rtol=0, atol=1e-15)
    np.testing.assert_array_equal(omega_block(9, 3, 1, 40, 7), z[:40, :7])
    # different (iteration, block) give different streams
    assert np.abs(omega_block(9, 3, 2, 40, 10) - z[:40]).min() > 0


# ---------------------------------------------------------------------------- Eq. 5 and its properties

def test_d_tau_closed_form_P1():
    """Eq. 5: D_tau(U diag(s) V^T) = U diag((s - tau)_+) V^T."""
    rng = np.random.default_rng(0)
    s = np.array([9.0, 7.5, 5.0, 3.01, 2.99, 1.0, 0.2])
    U, V, Y = _planted_dense(rng, 40, 30, s)
    tau = 3.0
    expect = (U * np.maximum(s - tau, 0.0)) @ V.T
    np.testing.assert_allclose(d_tau(Y, tau), expect, rtol=0, atol=1e-12 * np.abs(Y).max())


def test_d_tau_through_r4svd_full_observation_P1():
    """With Lambda = everything and eps_thr = 0 one R4SVD-based step yields exactly D_tau(Y) on Lambda."""
    rng = np.random.default_rng(1)
    m, n = 24, 18
    s = np.linspace(12.0, 0.5, 12)
    U, V, Y = _planted_dense(rng, m, n, s)
    rows, cols = np.divmod(np.arange(m * n), n)
    prob = Problem(m, n, rows, cols, np.ones(m * n))
    tau = 4.0
    p = Params(tau=tau, delta=1.0, eps_thr0=0.0, seed=3, t0=3, dt=4)
    _, info = svt_step(prob, p, State(it=0, y=Y[rows, cols]))
    expect = ((U * np.maximum(s - tau, 0)) @ V.T)[rows, cols]
    np.testing.assert_allclose(info.x, expect, rtol=0, atol=1e-12 * np.abs(Y).max())
    assert info.k == int((s > tau).sum())
    np.testing.assert_allclose(np.sort(info.sigma)[::-1][: len(s)], s, rtol=1e-12)


def test_prox_optimality_P2():
    """Eq. 3 / Eq. 5: D_tau is the prox of tau ||.||_*, so ||Y - X||_2 <= tau and U_K^T (Y - X) V_K = tau I."""
    rng = np.random.default_rng(2)
    Y = rng.standard_normal((30, 25)) * 3.0
    tau = 4.0
    X = d_tau(Y, tau)
    assert np.linalg.norm(Y - X, 2) <= tau * (1 + 1e-12)
    U, s, Vt = np.linalg.svd(Y, full_matrices=False)
    K = s > tau
    G = U[:, K].T @ (Y - X) @ Vt[K].T
    np.testing.assert_allclose(G, tau * np.eye(K.sum()), atol=1e-10)

    def obj(Z):
        return 0.5 * np.linalg.norm(Z - Y) ** 2 + tau * np.linalg.svd(Z, compute_uv=False).sum()
    f0 = obj(X)
    for _ in range(20):
        assert obj(X + 1e-3 * rng.standard_normal(X.shape)) >= f0 - 1e-12


def test_non_expansive_P3():
    rng = np.random.default_rng(3)
    for _ in range(10):
        Y1 = rng.standard_normal((20, 15)) * 2
        Y2 = Y1 + 0.3 * rng.standard_normal((20, 15))
        assert np.linalg.norm(d_tau(Y1, 2.5) - d_tau(Y2, 2.5)) <= np.linalg.norm(Y1 - Y2) * (1 + 1e-12)


# ---------------------------------------------------------------------------- QB energy identities (Eq. 8-11) and Alg. 3

def _random_sparse(rng, m, n, frac):
    Yd = rng.standard_normal((m, n)) * (rng.random((m, n)) < frac)
    Yd[:, :3] += np.outer(rng.standard_normal(m), np.ones(3)) * 5 * (rng.random((m, 3)) < frac)
    return sp.csr_matrix(Yd), Yd


@pytest.mark.parametrize("eps_thr,npow", [(0.5, 0), (0.2, 0), (0.05, 1), (0.0, 0)])
def test_qb_energy_and_stopping_P4_P5_P6_P7_P8(eps_thr, npow):
    rng = np.random.default_rng(4)
    m, n = 60, 45
    Y, Yd = _random_sparse(rng, m, n, 0.3)
    normY = float(np.sum(Yd * Yd))
    p = Params(tau=1.0, delta=1.0, t0=4, dt=5, npow=npow, seed=5).resolved(m, n)
    info = StepInfo(it=1)
    Q, Wt, normB, eps, thr = r4svd(Y, normY, None, eps_thr, p, 1, info=info)
    # P8 orthonormality
    assert np.abs(Q.T @ Q - np.eye(Q.shape[1])).max() < 1e-13
    # P5 incremental normB equals ||Q^T Y||_F^2 recomputed, and W = Y^T Q
    B = Q.T @ Yd
    np.testing.assert_allclose(Wt, B.T, atol=1e-12)
    assert abs(normB - np.sum(B * B)) <= 1e-12 * normY
    # P4 Eq. 10: ||Y - Q Q^T Y||^2 = ||Y||^2 - ||B||^2
    resid = np.sum((Yd - Q @ B) ** 2)
    assert abs(resid - (normY - normB)) <= 1e-12 * normY
    assert abs(eps - resid / normY) <= 1e-12
    # P6 Eq. 9: no rank-r approximation beats the truncated SVD
    s = np.linalg.svd(Yd, compute_uv=False)
    r = Q.shape[1]
    assert eps >= np.sum(s[r:] ** 2) / normY - 1e-12
    # P7 Alg. 3 stopping rule: precision reached, or the basis is full, or the range is exhausted
    assert eps <= thr or r >= p.r_max or info.exhausted
    if info.blocks > 0:
        assert info.eps_hist[-2] > thr
    if eps_thr == 0.0:
        # the basis captures all of Y (rank n here), by a full basis, exhaustion or eps hitting zero
        assert abs(eps) < 1e-12 and r >= n


def test_recycled_start_keeps_span_and_grows_orthogonally_P8():
    rng = np.random.default_rng(6)
    m, n = 50, 40
    Y, Yd = _random_sparse(rng, m, n, 0.4)
    normY = float(np.sum(Yd * Yd))
    Q0 = _orth(rng, m, 7)
    p = Params(tau=1.0, delta=1.0, t0=4, dt=6, seed=8).resolved(m, n)
    info = StepInfo(it=2)
    Q, Wt, normB, eps, thr = r4svd(Y, normY, Q0, 0.1, p, 2, info=info)
    assert np.abs(Q.T @ Q - np.eye(Q.shape[1])).max() < 1e-13
    # Alg. 3 keeps the recycled columns as the trailing block (Q <- [Q', Q])
    np.testing.assert_array_equal(Q[:, -7:], Q0)
    assert Q.shape[1] == 7 + 6 * info.blocks


def test_range_exhaustion_on_rank_deficient_input():
    """Rank-2 Y and a threshold that is never met: growth stops when no new direction survives projection (S5)."""
    rng = np.random.default_rng(7)
    m, n = 30, 20
    Yd = np.outer(rng.standard_normal(m), rng.standard_normal(n)) + np.outer(rng.standard_normal(m), rng.standard_normal(n))
    Y = sp.csr_matrix(Yd)
    p = Params(tau=1.0, delta=1.0, t0=1, dt=3, seed=1).resolved(m, n)
    info = StepInfo(it=1)
    Q, Wt, normB, eps, thr = r4svd(Y, float(np.sum(Yd * Yd)), None, -1.0, p, 1, info=info)
    assert info.exhausted
    assert Q.shape[1] == 2
    assert abs(eps) < 1e-12


# ---------------------------------------------------------------------------- Alg. 4 against exact SVT

def test_reduces_to_exact_svt_P9():
    """eps_thr = 0 on a small square problem: the basis reaches R^m each iteration, so every iterate equals SVT-full SVD."""
    w = W.tiny_dense(30, 30, 3, 0.5, seed=11)
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, eps_thr0=0.0, beta=1.0 - 1e-12, seed=2, maxit=25)
    state, k0 = initial_state(prob, p)
    y = state.y.copy()
    for _ in range(25):
        state, info = svt_step(prob, p, state)
        x_exact, res, rel, _ = svt_exact_step(prob, p, y)
        assert info.r == 30
        np.testing.assert_allclose(info.x, x_exact, rtol=0, atol=1e-11 * np.abs(x_exact).max())
        assert abs(info.rel - rel) <= 1e-11 * rel
        if info.stopped:
            break
        y = y + p.delta * res
        np.testing.assert_allclose(state.y, y, rtol=0, atol=1e-11 * np.abs(y).max())


def test_rotation_invariance_P10():
    """Only span(Q) matters: rotating the recycled basis leaves x, eps and r unchanged (reading S9)."""
    w = W.tiny_dense(40, 35, 3, 0.5, seed=12)
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=4)
    state, _ = initial_state(prob, p)
    for _ in range(6):
        state, _ = svt_step(prob, p, state)
    rng = np.random.default_rng(0)
    R = _orth(rng, state.Q.shape[1], state.Q.shape[1])
    s1, i1 = svt_step(prob, p, state)
    rot = State(it=state.it, y=state.y, Q=state.Q @ R, eps_thr=state.eps_thr, eps_min=state.eps_min)
    s2, i2 = svt_step(prob, p, rot)
    assert i1.r == i2.r and i1.k == i2.k and i1.blocks == i2.blocks
    np.testing.assert_allclose(i1.x, i2.x, rtol=0, atol=1e-11 * np.abs(i1.x).max())
    assert abs(i1.eps - i2.eps) < 1e-12


def test_kicking_P11():
    """Alg. 4 initialisation: D_tau(j delta P_Lambda A) vanishes for j < k0 and not at k0 (reading S14)."""
    w = W.tiny_dense(40, 30, 3, 0.4, seed=13)
    PA = dense(w.m, w.n, w.rows, w.cols, w.a)
    s1 = spectral_norm(w.m, w.n, w.rows, w.cols, w.a)
    np.testing.assert_allclose(s1, np.linalg.svd(PA, compute_uv=False)[0], rtol=1e-13)
    k0 = kicking_k0(w.tau, w.delta, s1)
    assert k0 >= 2
    for j in range(1, k0):
        assert np.abs(d_tau(j * w.delta * PA, w.tau)).max() == 0.0
    assert np.abs(d_tau(k0 * w.delta * PA, w.tau)).max() > 0.0


def test_approximation_bound_P12():
    """||D_tau(Y) - D_tau(Q Q^T Y)||_F <= sqrt(eps) ||Y||_F (non-expansiveness + Eq. 10)."""
    rng = np.random.default_rng(14)
    m, n = 50, 40
    Y, Yd = _random_sparse(rng, m, n, 0.5)
    normY = float(np.sum(Yd * Yd))
    for thr in (0.6, 0.3, 0.1):
        p = Params(tau=2.0, delta=1.0, t0=3, dt=4, seed=2).resolved(m, n)
        info = StepInfo(it=1)
        Q, Wt, normB, eps, _ = r4svd(Y, normY, None, thr, p, 1, info=info)
        lhs = np.linalg.norm(d_tau(Yd, 2.0) - d_tau(Q @ (Q.T @ Yd), 2.0))
        assert lhs <= math.sqrt(max(eps, 0.0) * normY) * (1 + 1e-10) + 1e-12


def test_step_matches_dense_definition_on_lambda():
    """x of one oracle step equals D_tau(Q Q^T Y) on Lambda, the quantity Alg. 3 + Eq. 5 define."""
    w = W.tiny_dense(45, 38, 3, 0.45, seed=15)
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=6)
    state, _ = initial_state(prob, p)
    for _ in range(4):
        prev = state
        state, info = svt_step(prob, p, state)
    Yd = dense(w.m, w.n, w.rows, w.cols, prev.y)
    Q = info.Q
    X = d_tau(Q @ (Q.T @ Yd), p.tau)
    np.testing.assert_allclose(info.x, X[w.rows, w.cols], rtol=0, atol=1e-11 * max(1.0, np.abs(X).max()))
    res = w.a - info.x
    np.testing.assert_allclose(state.y, prev.y + p.delta * res, rtol=0, atol=1e-12 * np.abs(prev.y).max())


def test_annealing_rule_eq14():
    """Eq. 13-14: the threshold shrinks by beta exactly when the residual fails to decrease."""
    w = W.tiny_dense(40, 40, 3, 0.35, seed=16)
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=7, maxit=80)
    state, infos, _ = svt_run(prob, p, keep_infos=True)
    best = math.inf
    thr = infos[0].eps_thr_used
    for inf in infos:
        assert inf.eps_thr_used == pytest.approx(thr, rel=1e-15)
        if inf.rel < best:
            assert not inf.annealed
            best = inf.rel
        else:
            assert inf.annealed
            thr *= p.beta
    assert any(i.annealed for i in infos)


def test_planted_recovery_P13():
    """A planted low-rank matrix is recovered: residual below tol, rank equal to the planted rank."""
    w = W.tiny_dense(80, 80, 3, 0.4, seed=17)
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=1, maxit=600)
    state, info, k0 = svt_run(prob, p)
    assert info.stopped and info.rel < 1e-4
    assert info.k == 3
    X = (info.U * info.s_minus_tau) @ info.V.T
    assert np.linalg.norm(X - w.A) / np.linalg.norm(w.A) < 2e-3
    _, Xe, hist = svt_exact_run(prob, p)
    assert np.linalg.norm(X - Xe) / np.linalg.norm(Xe) < 2e-3


def test_replay_forces_decisions():
    w = W.tiny_dense(40, 40, 3, 0.35, seed=18)
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=3, maxit=30)
    _, infos, _ = svt_run(prob, p, keep_infos=True)
    replay = [(i.blocks, i.annealed) for i in infos]
    _, infos2, _ = svt_run(prob, p, replay=replay, keep_infos=True)
    for a, b in zip(infos, infos2):
        assert a.blocks == b.blocks and a.annealed == b.annealed
        np.testing.assert_array_equal(a.x, b.x)


# ---------------------------------------------------------------------------- emulated reduced precision

def test_mixed_oracle_rounds_at_storage_points_and_tracks_fp64():
    """The emulated mixed form keeps Y, x and the residual float32-representable and stays within
    float32 error of the FP64 step from the same state (same decisions)."""
    from oracle.mixed import f32, svt_step_mixed
    w = W.tiny_dense(70, 60, 3, 0.45, seed=19)
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=4)
    state, _ = initial_state(prob, p)
    for _ in range(5):
        state, _ = svt_step(prob, p, state)
    st32 = State(it=state.it, y=f32(state.y), Q=f32(state.Q), eps_thr=state.eps_thr, eps_min=state.eps_min)
    new32, i32 = svt_step_mixed(prob, p, st32)
    new64, i64 = svt_step(prob, p, st32)
    assert np.array_equal(new32.y, f32(new32.y)) and np.array_equal(i32.x, f32(i32.x))
    assert i32.r == i64.r and i32.k == i64.k
    assert np.abs(i32.x - i64.x).max() <= 1e-5 * np.abs(i64.x).max()
    assert abs(i32.rel - i64.rel) <= 1e-5 * i64.rel
    assert np.abs(new32.y - new64.y).max() <= 1e-5 * np.abs(new64.y).max()
    # and the float32 rounding is really applied: the two forms are not bit-identical
    assert np.abs(i32.x - i64.x).max() > 0


@pytest.mark.parametrize("mode_kw", [dict(mode="r3svd"), dict(mode="rsvd", rank=4, oversample=6),
                                     dict(recycle_extra=2)])
def test_mixed_oracle_modes_track_fp64(mode_kw):
    """The emulated mixed form's operator variants (R3SVD every iteration, the fixed-rank RSVD of
    Alg. 1, truncated recycling) take the FP64 oracle's decisions and stay within float32 error of
    it over several iterations; the widths are those the variant fixes (t0 per R3SVD iteration,
    rank + oversample for RSVD, at most k + extra recycled)."""
    from oracle.mixed import f32, svt_step_mixed
    w = W.tiny_dense(80, 70, 4, 0.45, seed=23)
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=6, t0=8, **mode_kw)
    s64, k0 = initial_state(prob, p)
    s32 = State(it=0, y=f32(s64.y))
    for _ in range(8):
        s64n, i64 = svt_step(prob, p, s64)
        s32, i32 = svt_step_mixed(prob, p, s32, replay=(i64.blocks, i64.annealed))
        assert i32.r == i64.r and i32.k == i64.k
        assert np.abs(i32.x - i64.x).max() <= 2e-5 * max(np.abs(i64.x).max(), 1e-300)
        assert abs(i32.rel - i64.rel) <= 2e-5 * i64.rel
        assert np.array_equal(i32.x, f32(i32.x))
        if p.mode == "rsvd":
            assert i64.r == 10 and i64.k <= 4
        if p.mode == "r3svd":
            assert i64.blocks > 0 or i64.r == 8
        if p.recycle_extra >= 0 and s32.Q is not None:
            assert s32.Q.shape[1] <= i64.k + 2
        s64 = s64n


def test_spectral_norm_sparse_branch_matches_dense_svd():
    """||P_Lambda A||_2 of the kicking start on problems above 4e6 entries comes from ARPACK
    (scipy svds); on a 2100 x 2000 pattern (1% observed, the branch taken) it must equal the largest
    singular value of the dense matrix from LAPACK's full SVD (np.linalg.norm(., 2)), and the
    power-law shape of the ratings workload must not change that."""
    from oracle.svt import dense, spectral_norm
    rng = np.random.default_rng(29)
    m, n = 2100, 2000
    assert m * n > 4_000_000
    for heavy in (False, True):
        if heavy:   # a few dense columns and rows dominate, as with power-law degrees
            lin = np.concatenate([rng.choice(m * n, 40_000, replace=False),
                                  np.arange(m) * n + 3, 7 * n + np.arange(n)])
        else:
            lin = rng.choice(m * n, 42_000, replace=False)
        lin = np.unique(lin)
        rows, cols = lin // n, lin % n
        vals = rng.standard_normal(lin.size)
        s_sparse = spectral_norm(m, n, rows, cols, vals)
        s_dense = float(np.linalg.svd(dense(m, n, rows, cols, vals), compute_uv=False)[0])
        assert abs(s_sparse - s_dense) <= 1e-12 * s_dense, (heavy, s_sparse, s_dense)
