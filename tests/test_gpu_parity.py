"""GPU parity: the HIP path through the C-ABI against the FP64 oracle on the same seeded inputs.

Bar (FP64 form): every real-valued result within 1e-10 relative (max-abs error over
max-abs value); integers (r, k, growth blocks, decisions) exact.
"""
import math

import numpy as np
import pytest

import svt_workloads as W
from oracle import Params, Problem, State, initial_state, svt_run, svt_step
from oracle.svt import kicking_k0, spectral_norm
from paper_1704_05528_amd._capi import SVT_F_EIG_INEXACT

pytestmark = pytest.mark.gpu

TOL = 1e-10


def rel_err(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    if a.size == 0 and b.size == 0:
        return 0.0
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _problem(w):
    return Problem(w.m, w.n, w.rows, w.cols, w.a)


def _gpu(svt, w, k0, **kw):
    return svt.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, k0=k0, **kw)


def _compare_step(st, info, h, w, ctx):
    assert st.r == info.r, (ctx, "r", st.r, info.r)
    assert st.k == info.k, (ctx, "k", st.k, info.k)
    assert st.blocks == info.blocks, (ctx, "blocks", st.blocks, info.blocks)
    assert bool(st.annealed) == bool(info.annealed), (ctx, "annealed")
    assert bool(st.stopped) == bool(info.stopped), (ctx, "stopped")
    assert abs(st.eps - info.eps) <= TOL, (ctx, "eps", st.eps, info.eps)
    assert abs(st.rel_res - info.rel) <= TOL * info.rel, (ctx, "rel", st.rel_res, info.rel)
    x = h.sample(w.rows, w.cols)
    assert rel_err(x, info.x) <= TOL, (ctx, "x", rel_err(x, info.x))
    if info.k > 0:
        assert rel_err(st.sigma1, info.sigma[0]) <= TOL, (ctx, "sigma1")
        assert rel_err(st.sigmak, info.sigma[info.k - 1]) <= TOL, (ctx, "sigmak")


SHAPES = [
    # (m, n, rank, frac, seed, extra params)
    (90, 70, 3, 0.40, 31, {}),
    (70, 90, 3, 0.40, 32, {}),
    (130, 110, 4, 0.35, 33, {"dt": 7}),          # ragged sizes, basis grows past one eigen block
    (64, 64, 2, 0.5, 34, {"t0": 5, "npow": 1}),   # power iterations
    (150, 40, 3, 0.6, 35, {"eps_thr0": 0.3}),     # tall, explicit threshold
    (500, 400, 2, 0.04, 36, {"t0": 12}),          # 4% observed: gather path for Y^T Q
    (300, 250, 3, 0.15, 37, {}),                   # 15% observed: LDS-tiled Y^T Q
    (400, 300, 40, 0.5, 81, {"dt": 40}),          # k up to 58: eigensolver blocks and growth blocks over 32 columns
]
# 25% or more observed (the rows above with frac >= 0.25): Y^T Q on the matrix cores with a dense copy of Y


@pytest.mark.parametrize("m,n,rank,frac,seed,extra", SHAPES)
def test_free_run_with_replayed_decisions(gpu_lib, m, n, rank, frac, seed, extra):
    """Both sides run 25 iterations; the GPU replays the oracle's two discrete decisions so that
    rounding-level ties cannot split the trajectories; all results agree to 1e-10."""
    w = W.tiny_dense(m, n, rank, frac, seed=seed)
    prob = _problem(w)
    p = Params(tau=w.tau, delta=w.delta, seed=seed, maxit=25, **extra)
    _, infos, k0 = svt_run(prob, p, keep_infos=True)
    h = _gpu(gpu_lib, w, k0, seed=seed, maxit=25, **extra)
    h.set_replay([i.blocks for i in infos], [int(i.annealed) for i in infos])
    for info in infos:
        st = h.iterate(1)
        _compare_step(st, info, h, w, (m, n, info.it))
    s = h.get_state()
    assert s["iter"] == infos[-1].it


@pytest.mark.parametrize("m,n,rank,frac,c,seed", [(400, 320, 200, 0.6, 0.6, 91), (300, 260, 200, 0.7, 0.4, 92)])
def test_counts_beyond_the_block_solver(gpu_lib, m, n, rank, frac, c, seed):
    """A rank-200 planted matrix with a low threshold: k passes the 92 pairs the subspace solver's
    96-column block can hold within four iterations and climbs to 242-284 of a 253-336 column
    basis.  The projected SVD then diagonalises all of G (Jacobi over many workgroups, warm-started
    from the previous iteration's eigenvectors).  30 iterations with replayed decisions at 1e-10."""
    w = W.tiny_dense(m, n, rank, frac, seed=seed, tau=c * math.sqrt(m * n))
    prob = _problem(w)
    extra = {"dt": 40}
    p = Params(tau=w.tau, delta=w.delta, seed=seed, maxit=30, **extra)
    _, infos, k0 = svt_run(prob, p, keep_infos=True)
    assert max(i.k for i in infos) > 200
    h = _gpu(gpu_lib, w, k0, seed=seed, maxit=30, **extra)
    h.set_replay([i.blocks for i in infos], [int(i.annealed) for i in infos])
    for info in infos:
        print(f"iteration {info.it} r={info.r} k={info.k}", flush=True)
        st = h.iterate(1)
        assert not (st.flags & SVT_F_EIG_INEXACT), info.it
        _compare_step(st, info, h, w, ("wide k", info.it))
        if info.k > 0:
            kk, s, U, V = h.factors(info.k)
            assert rel_err(s, info.sigma[:info.k] - w.tau) <= TOL


def test_subspace_blocks_wider_than_256_on_a_wide_basis(gpu_lib):
    """A 1000-column basis with 144-161 values above tau: the subspace solver holds blocks of up to a
    third of the basis there, so iterations 3-6 run it with blocks of 292 and 324 columns (Rayleigh
    quotients on the many-workgroup Jacobi) instead of the full decomposition.  Six iterations with
    replayed decisions at 1e-10."""
    w = W.tiny_dense(1100, 1000, 160, 0.6, seed=93, tau=2.5 * math.sqrt(1100 * 1000))
    prob = _problem(w)
    extra = {"t0": 1000}
    p = Params(tau=w.tau, delta=w.delta, seed=93, maxit=6, **extra)
    _, infos, k0 = svt_run(prob, p, keep_infos=True)
    assert [i.r for i in infos] == [1000] * 6 and 127 <= infos[2].k <= 162
    h = _gpu(gpu_lib, w, k0, seed=93, maxit=6, **extra)
    h.set_replay([i.blocks for i in infos], [int(i.annealed) for i in infos])
    for info in infos:
        print(f"iteration {info.it} r={info.r} k={info.k}", flush=True)
        st = h.iterate(1)
        assert not (st.flags & SVT_F_EIG_INEXACT), info.it
        _compare_step(st, info, h, w, ("wide blocks", info.it))


@pytest.mark.parametrize("extra", [{"t0": 20}, {"t0": 6, "dt": 4}])
def test_heavy_columns_chunked_gather(gpu_lib, extra):
    """1% observed with three columns of 9000, 5000 and 2600 rows: Y^T Q takes the gather path
    with the long columns cut into chunks (16-wide and wider blocks), 20 iterations at 1e-10."""
    w = W.heavy_columns(30000, 60, 3, (9000, 5000, 2600), 40, seed=51, delta=1.2)
    prob = _problem(w)
    p = Params(tau=w.tau, delta=w.delta, seed=51, maxit=20, **extra)
    _, infos, k0 = svt_run(prob, p, keep_infos=True)
    h = _gpu(gpu_lib, w, k0, seed=51, maxit=20, **extra)
    h.set_replay([i.blocks for i in infos], [int(i.annealed) for i in infos])
    for info in infos:
        st = h.iterate(1)
        _compare_step(st, info, h, w, ("heavy", info.it))


def test_free_run_decisions_agree(gpu_lib):
    """Without replay the device takes the same discrete decisions while margins are clear."""
    w = W.tiny_dense(100, 80, 3, 0.4, seed=41)
    prob = _problem(w)
    p = Params(tau=w.tau, delta=w.delta, seed=3, maxit=40)
    _, infos, k0 = svt_run(prob, p, keep_infos=True)
    h = _gpu(gpu_lib, w, k0, seed=3, maxit=40)
    for info in infos:
        margins = [abs(g) for g in info.grow_margins] + [abs(info.anneal_margin)]
        st = h.iterate(1)
        if min(margins) < 1e-9:
            pytest.skip(f"near-tie decision at iteration {info.it}: replay test covers it")
        _compare_step(st, info, h, w, info.it)


def test_step_parity_from_oracle_state(gpu_lib):
    """Load the oracle's state after 15 iterations, run one step on both sides."""
    w = W.tiny_dense(120, 100, 4, 0.4, seed=42)
    prob = _problem(w)
    p = Params(tau=w.tau, delta=w.delta, seed=8, maxit=40)
    state, k0 = initial_state(prob, p)
    for _ in range(15):
        state, _ = svt_step(prob, p, state)
    h = _gpu(gpu_lib, w, k0, seed=8)
    h.set_state(state.y, state.Q, state.eps_thr, state.eps_min, state.it)
    nxt, info = svt_step(prob, p, state)
    st = h.iterate(1)
    _compare_step(st, info, h, w, "step")
    s = h.get_state()
    assert rel_err(s["y"], nxt.y) <= TOL
    # the device keeps an unrotated basis: compare projectors
    Pg = s["Q"] @ s["Q"].T
    Po = nxt.Q @ nxt.Q.T
    assert np.abs(Pg - Po).max() <= 1e-10


def test_wide_basis_tiled_gram(gpu_lib):
    """A 1100-column basis on 36400 columns of Y (rows * r above the cut-over): the Gram matrix
    W^T W comes from the 64 x 64 LDS-tiled kernel.  One step from a given state on both sides
    (k = 9, with clear gaps at the threshold: in a dense part of the spectrum a cold-started
    subspace iteration can stop at its product cap, which SVT_F_EIG_INEXACT reports)."""
    m, n, r = 1200, 36400, 1100
    w = W.tiny_dense(m, n, 5, 0.01, seed=61, delta=1.2)
    prob = _problem(w)
    p = Params(tau=w.tau, delta=w.delta, seed=61, maxit=10, r_max=m)
    rng = np.random.default_rng(62)
    Q0, _ = np.linalg.qr(rng.standard_normal((m, r)))
    k0 = kicking_k0(w.tau, w.delta, spectral_norm(m, n, w.rows, w.cols, w.a))
    state = State(it=4, y=1.2 * k0 * w.delta * w.a, Q=Q0, eps_thr=0.99, eps_min=math.inf)
    nxt, info = svt_step(prob, p, state)
    assert info.blocks == 0 and info.r == r
    h = _gpu(gpu_lib, w, k0, seed=61, maxit=10, r_max=m)
    h.set_state(state.y, state.Q, state.eps_thr, state.eps_min, state.it)
    st = h.iterate(1)
    assert info.k > 4 and not (st.flags & SVT_F_EIG_INEXACT)
    _compare_step(st, info, h, w, "wide gram")
    s = h.get_state()
    assert rel_err(s["y"], nxt.y) <= TOL
    Pg = s["Q"] @ s["Q"].T
    Po = nxt.Q @ nxt.Q.T
    assert np.abs(Pg - Po).max() <= 1e-10


@pytest.mark.parametrize("m,r", [(600, 450), (700, 537)])
def test_wide_basis_gram_32_tiles(gpu_lib, m, r):
    """A basis of several hundred columns on 997 columns of Y: the Gram matrix W^T W comes from the
    32 x 32-tile kernel (537 columns leave a ragged tile, 997 rows a partial last k-step).  One step
    from a given state on both sides (k = 5, the planted rank, with a clear gap below it)."""
    n = 997
    w = W.tiny_dense(m, n, 5, 0.3, seed=63, delta=1.2)
    prob = _problem(w)
    p = Params(tau=w.tau, delta=w.delta, seed=63, maxit=10, r_max=m)
    rng = np.random.default_rng(64)
    Q0, _ = np.linalg.qr(rng.standard_normal((m, r)))
    k0 = kicking_k0(w.tau, w.delta, spectral_norm(m, n, w.rows, w.cols, w.a))
    state = State(it=4, y=2.0 * k0 * w.delta * w.a, Q=Q0, eps_thr=0.99, eps_min=math.inf)
    nxt, info = svt_step(prob, p, state)
    assert info.blocks == 0 and info.r == r and info.k == 5
    h = _gpu(gpu_lib, w, k0, seed=63, maxit=10, r_max=m)
    h.set_state(state.y, state.Q, state.eps_thr, state.eps_min, state.it)
    st = h.iterate(1)
    assert not (st.flags & SVT_F_EIG_INEXACT)
    _compare_step(st, info, h, w, "gram 32")
    s = h.get_state()
    assert rel_err(s["y"], nxt.y) <= TOL
    assert np.abs(s["Q"] @ s["Q"].T - nxt.Q @ nxt.Q.T).max() <= 1e-10


def test_state_roundtrip_and_orthonormal_basis(gpu_lib):
    w = W.tiny_dense(80, 60, 3, 0.5, seed=43)
    prob = _problem(w)
    p = Params(tau=w.tau, delta=w.delta, seed=4)
    _, k0 = initial_state(prob, p)
    h = _gpu(gpu_lib, w, k0, seed=4)
    h.iterate(8)
    s = h.get_state()
    Q = s["Q"]
    assert np.abs(Q.T @ Q - np.eye(Q.shape[1])).max() < 1e-13
    h2 = _gpu(gpu_lib, w, k0, seed=4)
    h2.set_state(s["y"], Q, s["eps_thr"], s["eps_min"], s["iter"])
    s2 = h2.get_state()
    np.testing.assert_array_equal(s2["y"], s["y"])
    np.testing.assert_array_equal(s2["Q"], Q)
    a = h.iterate(1)
    b = h2.iterate(1)
    assert a.r == b.r and a.k == b.k and a.rel_res == b.rel_res


def test_factors_are_thresholded_svd(gpu_lib):
    """svt_factors returns orthonormal U, V and s = sigma - tau > 0 with X = U diag(s) V^T (Eq. 5)."""
    w = W.tiny_dense(90, 75, 3, 0.45, seed=44)
    prob = _problem(w)
    p = Params(tau=w.tau, delta=w.delta, seed=6)
    state, k0 = initial_state(prob, p)
    for _ in range(10):
        state, info = svt_step(prob, p, state)
    h = _gpu(gpu_lib, w, k0, seed=6)
    h.iterate(10)
    k, s, U, V = h.factors()
    assert k == info.k and k > 0
    assert (s > 0).all()
    np.testing.assert_allclose(s, info.s_minus_tau, rtol=TOL)
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-12
    assert np.abs(V.T @ V - np.eye(k)).max() < 1e-12
    X = (U * s) @ V.T
    Xo = (info.U * info.s_minus_tau) @ info.V.T
    assert rel_err(X, Xo) <= TOL
    qi, qj = np.divmod(np.arange(w.m * w.n), w.n)
    assert rel_err(h.sample(qi, qj), X.ravel()) <= 1e-12


def test_r4svd_step_leaves_state_unchanged(gpu_lib):
    w = W.tiny_dense(70, 70, 3, 0.4, seed=45)
    prob = _problem(w)
    p = Params(tau=w.tau, delta=w.delta, seed=2)
    _, k0 = initial_state(prob, p)
    h = _gpu(gpu_lib, w, k0, seed=2)
    h.iterate(5)
    before = h.get_state()
    st = h.r4svd_step()
    after = h.get_state()
    np.testing.assert_array_equal(before["y"], after["y"])
    assert before["r"] == after["r"] and before["iter"] == after["iter"]
    nxt = h.iterate(1)
    assert nxt.r == st.r and nxt.k == st.k


def test_run_twice_bitwise_identical(gpu_lib):
    """Deterministic reductions: two handles on the same input give bit-identical trajectories."""
    w = W.tiny_dense(110, 90, 3, 0.4, seed=46)
    _, k0 = initial_state(_problem(w), Params(tau=w.tau, delta=w.delta))
    outs = []
    for _ in range(2):
        h = _gpu(gpu_lib, w, k0, seed=9)
        st = h.iterate(20)
        outs.append((st.rel_res, st.r, h.get_state()["y"]))
    assert outs[0][0] == outs[1][0] and outs[0][1] == outs[1][1]
    np.testing.assert_array_equal(outs[0][2], outs[1][2])


@pytest.mark.parametrize("frac", [0.4, 0.15])
def test_calls_between_steps_leave_trajectory_unchanged(gpu_lib, frac):
    """R4SVD enqueues the next step's leading work (dense copy, W = Y^T Q, ||W||^2) at the end of a step.  Steps
    taken one call at a time, with reads and single-phase replays between them (which drop or keep that work),
    must follow the trajectory of one call taking them all, bit for bit (dense-copy and gather paths)."""
    w = W.tiny_dense(160, 140, 5, frac, seed=48)
    _, k0 = initial_state(_problem(w), Params(tau=w.tau, delta=w.delta))
    ref = _gpu(gpu_lib, w, k0, seed=9, tol=1e-13)  # no stop within the 16 steps
    st_ref = ref.iterate(16)
    h = _gpu(gpu_lib, w, k0, seed=9, tol=1e-13)
    qi, qj = w.rows[:50], w.cols[:50]
    for it in range(16):
        st = h.iterate(1)
        if it % 4 == 0:
            h.sample(qi, qj)
            h.get_state()
        if it % 4 == 1:
            h.time_phase("spmm_t", reps=2)
        if it % 4 == 2:
            h.time_phase("gram", reps=2)
            h.time_phase("sddmm", reps=2)
        if it % 4 == 3 and h.get_state()["r"] > 0:
            h.factors()
    assert st.iter == st_ref.iter and st.rel_res == st_ref.rel_res and st.r == st_ref.r
    a, b = ref.get_state(), h.get_state()
    np.testing.assert_array_equal(a["y"], b["y"])
    np.testing.assert_array_equal(a["Q"], b["Q"])


def test_rmax_and_range_exhaustion_flags(gpu_lib):
    import paper_1704_05528_amd as svt
    w = W.tiny_dense(60, 50, 3, 0.5, seed=47)
    _, k0 = initial_state(_problem(w), Params(tau=w.tau, delta=w.delta))
    h = _gpu(gpu_lib, w, k0, seed=1, r_max=12, t0=4, dt=5, eps_thr0=0.0)
    st = h.iterate(1)
    assert st.r == 12 and (st.flags & svt.SVT_F_RMAX_HIT)
    # rank-2 data fully observed: growth runs out of directions
    rng = np.random.default_rng(0)
    A = np.outer(rng.standard_normal(20), rng.standard_normal(15)) + np.outer(rng.standard_normal(20), rng.standard_normal(15))
    qi, qj = np.divmod(np.arange(300), 15)
    h2 = svt.svt_init(20, 15, qi, qj, A.ravel(), tau=1e-3, delta=1.0, k0=1, t0=1, dt=3, eps_thr0=0.0, seed=2)
    st2 = h2.iterate(1)
    assert st2.r == 2 or (st2.flags & svt.SVT_F_EXHAUSTED)


def test_empty_rows_and_columns(gpu_lib):
    """Rows and columns without observations (and a single-entry column) follow the oracle."""
    w = W.tiny_dense(80, 70, 3, 0.4, seed=48)
    keep = (w.rows % 7 != 3) & (w.cols % 9 != 4)
    keep |= (w.cols == 4) & (w.rows == w.rows[w.cols == 4].min())
    w.rows, w.cols, w.a = w.rows[keep], w.cols[keep], w.a[keep]
    prob = _problem(w)
    p = Params(tau=w.tau, delta=w.delta, seed=5, maxit=12)
    _, infos, k0 = svt_run(prob, p, keep_infos=True)
    h = _gpu(gpu_lib, w, k0, seed=5, maxit=12)
    h.set_replay([i.blocks for i in infos], [int(i.annealed) for i in infos])
    for info in infos:
        _compare_step(h.iterate(1), info, h, w, info.it)


def test_kicking_count_matches_spectral_norm(gpu_lib):
    """The device computes ||P_Lambda A||_2 by power iteration; the kicked Y^(0) matches the oracle's."""
    w = W.tiny_dense(100, 90, 3, 0.3, seed=49)
    prob = _problem(w)
    p = Params(tau=w.tau, delta=w.delta)
    state, k0 = initial_state(prob, p)
    h = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta)
    np.testing.assert_allclose(h.get_state()["y"], state.y, rtol=1e-14)


def test_planted_1000_first_iterations(gpu_lib):
    """The 1000 x 1000 rank-10 problem at 20% sampling: first 6 iterations against the oracle."""
    w = W.planted()
    prob = _problem(w)
    p = Params(tau=w.tau, delta=w.delta, seed=11, maxit=6)
    _, infos, k0 = svt_run(prob, p, keep_infos=True)
    h = _gpu(gpu_lib, w, k0, seed=11, maxit=6)
    h.set_replay([i.blocks for i in infos], [int(i.annealed) for i in infos])
    for info in infos:
        _compare_step(h.iterate(1), info, h, w, info.it)


def test_image_workload_wide_basis_step(gpu_lib):
    """Image workload (1024^2, 50% observed) from a state with a 300-column basis: one step on both
    sides exercises the warm-started block eigensolver at full size."""
    w = W.image()
    prob = _problem(w)
    rng = np.random.default_rng(7)
    Q, _ = np.linalg.qr(rng.standard_normal((w.m, 300)))
    y = 3.0 * w.delta * w.a + 0.05 * rng.standard_normal(w.nnz)
    st0 = State(it=7, y=y, Q=Q, eps_thr=0.2, eps_min=0.05)
    p = Params(tau=w.tau, delta=w.delta, seed=12)
    _, info = svt_step(prob, p, st0)
    h = _gpu(gpu_lib, w, 2, seed=12)
    h.set_state(y, Q, 0.2, 0.05, 7)
    st = h.iterate(1)
    _compare_step(st, info, h, w, "image")


def test_image_workload_bench_configuration(gpu_lib):
    """The benchmark's own configuration: image workload from Y^(0) with Omega seed 11 through the
    warm-up into the timed window (45 iterations, basis 51 -> ~300 columns), every step against
    the oracle (decisions replayed)."""
    w = W.image()
    prob = _problem(w)
    p = Params(tau=w.tau, delta=w.delta, seed=11, maxit=45)
    _, infos, k0 = svt_run(prob, p, keep_infos=True)
    h = _gpu(gpu_lib, w, k0, seed=11, maxit=45)
    h.set_replay([i.blocks for i in infos], [int(i.annealed) for i in infos])
    for info in infos:
        _compare_step(h.iterate(1), info, h, w, ("image", info.it))


def test_tall_products_with_many_tiles(gpu_lib):
    """40000 x 200 at 5% observed, rank 20: the factor products Q C over 40000 rows have more than
    2048 16 x 16 tiles and run as the 64 x 32 workgroup variant (k_rowmul_tall); 8 iterations,
    every step against the oracle."""
    w = W.tiny_dense(40000, 200, 20, 0.05, seed=93)
    prob = _problem(w)
    p = Params(tau=w.tau, delta=w.delta, seed=93, maxit=8)
    _, infos, k0 = svt_run(prob, p, keep_infos=True)
    assert max(i.k for i in infos) >= 17  # two column tiles of the factors: 2500 x 2 tiles
    h = _gpu(gpu_lib, w, k0, seed=93, maxit=8)
    h.set_replay([i.blocks for i in infos], [int(i.annealed) for i in infos])
    for info in infos:
        _compare_step(h.iterate(1), info, h, w, ("tall", info.it))


def test_ratings_workload_first_iterations(gpu_lib):
    """Recommendation shape (6040 x 3706, 900,188 power-law training entries, 4% observed: the
    gather kernels), tau and delta by the rule of Sec. 3, r_max = 1024: first 6 iterations,
    including a round of growth blocks, against the oracle."""
    w = W.ratings()
    prob = _problem(w)
    p = Params(tau=w.tau, delta=w.delta, seed=11, maxit=6, r_max=1024)
    _, infos, k0 = svt_run(prob, p, keep_infos=True)
    h = _gpu(gpu_lib, w, k0, seed=11, maxit=6, r_max=1024)
    h.set_replay([i.blocks for i in infos], [int(i.annealed) for i in infos])
    for info in infos:
        _compare_step(h.iterate(1), info, h, w, ("ratings", info.it))


def test_planted_step_with_the_basis_filling_the_space(gpu_lib):
    """The planted 1000 x 1000 rank-10 problem late in its run: the oracle's state once the basis
    holds all m = 1000 columns (tests/golden/make_planted_late_state.py, oracle only).  The device
    starts from it (basis = identity, the same span) and takes one step: a 1000-column Gram, its
    eigenpairs above tau and the sampled update, against the oracle's next step at 1e-10."""
    import os
    ref = np.load(os.path.join(os.path.dirname(__file__), "golden", "planted_late_state.npz"))
    w = W.planted()
    h = _gpu(gpu_lib, w, int(ref["k0"]), seed=int(ref["seed"]), maxit=2000)
    h.set_state(ref["y"], np.eye(w.m), float(ref["eps_thr"]), float(ref["eps_min"]), int(ref["it"]))
    h.set_replay([int(ref["blocks"])], [int(ref["annealed"])])
    st = h.iterate(1)
    print(f"late planted step: iteration {st.iter} r={st.r} k={st.k} rel={st.rel_res:.6e}", flush=True)
    assert st.r == int(ref["r"]) == w.m and st.k == int(ref["k"])
    assert abs(st.rel_res - float(ref["rel"])) <= TOL * float(ref["rel"])
    x = h.sample(w.rows[ref["x_sample_pos"]], w.cols[ref["x_sample_pos"]])
    assert rel_err(x, ref["x_sample"]) <= TOL
    kk, s, U, V = h.factors()
    assert rel_err(s + w.tau, ref["sigma_k"]) <= TOL
    if not st.stopped:
        assert rel_err(h.get_state()["y"][ref["x_sample_pos"]], ref["y_next_sample"]) <= TOL


@pytest.mark.parametrize("name", ["planted", "ratings"])
def test_device_kicking_count(gpu_lib, name):
    """k0 = ceil(tau / (delta ||P_Lambda A||_2)) from the device's own power iteration, against the
    oracle's spectral norm (dense SVD for the planted problem, ARPACK for the ratings shape)."""
    w = W.planted() if name == "planted" else W.ratings()
    if name == "ratings":
        w.delta = 1.9
    sig = spectral_norm(w.m, w.n, w.rows, w.cols, w.a)
    ratio = w.tau / (w.delta * sig)
    if abs(ratio - round(ratio)) < 1e-9:
        pytest.skip("tau / (delta sigma_1) within 1e-9 of an integer")
    k0 = kicking_k0(w.tau, w.delta, sig)
    h = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, seed=1)
    y0 = h.get_state()["y"]
    nz = np.abs(w.a) > 0
    k_dev = np.unique(np.rint(y0[nz] / (w.delta * w.a[nz])).astype(int))
    print(f"{name}: ratio {ratio:.6f} oracle k0 {k0} device {k_dev}", flush=True)
    assert k_dev.tolist() == [k0]
