"""GPU parity of the BF16 form (bfloat16 basis with the exact projector onto its span, float32
iterate and factors, float64 Gram / Cholesky / eigen-solver) against the emulated BF16 oracle
(oracle.mixed.svt_step_bf16), and its error against the FP64 oracle.

Bars:
- one step from an oracle state: values within 1e-5 relative of the emulated oracle (float32
  accumulation-order noise, as for the float32 form), integers (r, k, growth blocks) exact;
- free runs with the oracle's decisions replayed: the relative residual within 1e-4 relative of
  the emulated run at every step.  Longer runs drift further apart than single steps because the
  device (CholeskyQR2) and the oracle (Householder QR) orthonormalise growth blocks with float32
  results a few units in 1e-7 apart, and the rare entry that sits at a bfloat16 rounding tie then
  rounds to neighbouring bfloat16 values on the two sides; x after the image window is checked
  at 2e-3 relative for that reason;
- against the FP64 oracle the same step stays within 5e-3 relative in x (the rounded basis spans
  a slightly different space) and 5e-4 in the residual.
"""
import numpy as np
import pytest

import svt_workloads as W
from oracle import Params, Problem, State, initial_state, svt_step
from oracle.mixed import bf16, f32, svt_step_bf16

pytestmark = pytest.mark.gpu

TOL_STEP = 1e-5
TOL_RUN = 1e-4
TOL_FP64_X, TOL_FP64_RES = 5e-3, 5e-4


def rel_err(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _oracle_state(prob, p, steps, step=svt_step):
    state, k0 = initial_state(prob, p)
    for _ in range(steps):
        state, _ = step(prob, p, state)
    return state, k0


@pytest.mark.parametrize("m,n,rank,frac,seed,steps", [(90, 70, 3, 0.4, 61, 6), (130, 110, 4, 0.35, 62, 14),
                                                      (200, 150, 3, 0.3, 63, 25)])
def test_bf16_step_against_emulated_and_fp64_oracle(gpu_lib, m, n, rank, frac, seed, steps):
    w = W.tiny_dense(m, n, rank, frac, seed=seed)
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=seed)
    s64, k0 = _oracle_state(prob, p, steps)
    st = State(it=s64.it, y=f32(s64.y), Q=bf16(s64.Q), eps_thr=s64.eps_thr, eps_min=s64.eps_min)
    nxt, info = svt_step_bf16(prob, p, st)
    _, info64 = svt_step(prob, p, s64)
    h = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, k0=k0, seed=seed,
                         precision=gpu_lib.SVT_BF16)
    h.set_state(st.y, st.Q, st.eps_thr, st.eps_min, st.it)
    d = h.iterate(1)
    x = h.sample(w.rows, w.cols)
    assert (d.r, d.k, d.blocks) == (info.r, info.k, info.blocks)
    assert rel_err(x, info.x) <= TOL_STEP
    assert abs(d.rel_res - info.rel) <= TOL_STEP * info.rel
    assert abs(d.eps - info.eps) <= 1e-6
    assert rel_err(h.get_state()["y"], nxt.y) <= TOL_STEP
    assert rel_err(x, info64.x) <= TOL_FP64_X
    assert abs(d.rel_res - info64.rel) <= TOL_FP64_RES * info64.rel
    h.close()


def test_bf16_free_run_with_replay_tracks_emulated_oracle(gpu_lib):
    w = W.tiny_dense(120, 100, 3, 0.4, seed=64)
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=3, maxit=40)
    state, k0 = initial_state(prob, p)
    infos = []
    for _ in range(40):
        state, info = svt_step_bf16(prob, p, state)
        infos.append(info)
    h = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, k0=k0, seed=3, maxit=40,
                         precision=gpu_lib.SVT_BF16)
    h.set_replay([i.blocks for i in infos], [int(i.annealed) for i in infos])
    for info in infos:
        d = h.iterate(1)
        assert (d.r, d.k) == (info.r, info.k)
        assert abs(d.rel_res - info.rel) <= TOL_RUN * info.rel
    # the stored basis is bfloat16 and not orthonormal: the correction is doing the work
    Q = h.get_state()["Q"]
    np.testing.assert_array_equal(Q, bf16(Q))
    assert np.abs(Q.T @ Q - np.eye(Q.shape[1])).max() > 1e-4
    h.close()


def test_bf16_image_size_step_and_window(gpu_lib):
    """The image-recovery workload (1024 x 1024, 50% observed): one step from the emulated oracle's
    state after 20 iterations at the 1e-5 bar, and the first 25 iterations with the oracle's
    decisions replayed at the free-run bars."""
    w = W.image()
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=11)
    state, k0 = initial_state(prob, p)
    infos = []
    for i in range(25):
        if i == 20:
            s20 = state
        state, info = svt_step_bf16(prob, p, state)
        infos.append(info)
    rng = np.random.default_rng(0)
    sel = rng.choice(w.nnz, 20000, replace=False)
    # one step from the oracle's state after 20 iterations
    h = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, k0=k0, seed=11,
                         precision=gpu_lib.SVT_BF16)
    h.set_state(s20.y, s20.Q, s20.eps_thr, s20.eps_min, s20.it)
    h.set_replay([infos[20].blocks], [int(infos[20].annealed)])
    d = h.iterate(1)
    assert (d.r, d.k) == (infos[20].r, infos[20].k)
    assert abs(d.rel_res - infos[20].rel) <= TOL_STEP * infos[20].rel
    assert rel_err(h.sample(w.rows[sel], w.cols[sel]), infos[20].x[sel]) <= TOL_STEP
    h.close()
    # the window from Y^(0)
    h = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, k0=k0, seed=11,
                         precision=gpu_lib.SVT_BF16)
    h.set_replay([i.blocks for i in infos], [int(i.annealed) for i in infos])
    for info in infos:
        d = h.iterate(1)
        assert (d.r, d.k) == (info.r, info.k)
        assert abs(d.rel_res - info.rel) <= TOL_RUN * info.rel
    assert rel_err(h.sample(w.rows[sel], w.cols[sel]), infos[-1].x[sel]) <= 2e-3
    h.close()


def test_bf16_planted_reaches_tolerance_like_fp64(gpu_lib):
    """The planted 1000 x 1000 rank-10 problem reaches relative residual 1e-4 in the BF16 form within
    a few iterations of the FP64 form's count, and the error percentage of Eq. 10 stays above float32
    noise on the way (the corrected energy never exceeds ||Y||^2)."""
    w = W.planted()
    its = {}
    for prec in (gpu_lib.SVT_FP64, gpu_lib.SVT_BF16):
        h = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, seed=11, maxit=1000, tol=w.tol,
                             precision=prec)
        d = h.iterate(1000)
        assert d.stopped and d.rel_res < 1e-4
        its[prec] = d.iter
        if prec == gpu_lib.SVT_BF16:
            assert min(x.eps for x in h.history()) >= -1e-6
        h.close()
    assert abs(its[gpu_lib.SVT_BF16] - its[gpu_lib.SVT_FP64]) <= max(5, its[gpu_lib.SVT_FP64] // 20)


@pytest.mark.parametrize("mode_kw", [dict(mode=1), dict(mode=2, rank=4, oversample=6)])
def test_bf16_operator_variants_against_emulated_oracle(gpu_lib, mode_kw):
    """R3SVD from a fresh t-block every iteration and the fixed-rank randomized SVD of Alg. 1 in the
    BF16 form: the bases are rebuilt (and their inverse Cholesky factors with them) every iteration."""
    w = W.tiny_dense(80, 70, 4, 0.45, seed=23)
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    omode = {1: "r3svd", 2: "rsvd"}[mode_kw["mode"]]
    p = Params(tau=w.tau, delta=w.delta, seed=6, t0=8, mode=omode,
               **{k: v for k, v in mode_kw.items() if k != "mode"})
    state, k0 = initial_state(prob, p)
    infos = []
    for _ in range(8):
        state, info = svt_step_bf16(prob, p, state)
        infos.append(info)
    h = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, k0=k0, seed=6, t0=8,
                         precision=gpu_lib.SVT_BF16, **mode_kw)
    h.set_replay([i.blocks for i in infos], [int(i.annealed) for i in infos])
    for info in infos:
        d = h.iterate(1)
        assert (d.r, d.k) == (info.r, info.k)
        assert abs(d.rel_res - info.rel) <= TOL_RUN * info.rel
    h.close()


def test_bf16_checkpoint_resumes_bit_for_bit(gpu_lib):
    w = W.tiny_dense(150, 120, 4, 0.4, seed=65)
    kw = dict(tau=w.tau, delta=w.delta, seed=9, maxit=100, tol=0.0, precision=gpu_lib.SVT_BF16)
    h1 = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, **kw)
    h1.iterate(7)
    blob = h1.checkpoint()
    h1.iterate(6)
    h2 = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, **kw)
    h2.restore(blob)
    h2.iterate(6)
    np.testing.assert_array_equal(h2.sample(w.rows, w.cols), h1.sample(w.rows, w.cols))
    h1.close()
    h2.close()


def test_bf16_refusals(gpu_lib):
    w = W.tiny_dense(60, 50, 2, 0.5, seed=66)
    with pytest.raises(gpu_lib.SVTError) as e:
        gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, precision=gpu_lib.SVT_BF16,
                         recycle_extra=2)
    assert e.value.status == gpu_lib.SVT_E_INVALID_ARG
    h = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, precision=gpu_lib.SVT_BF16,
                         tol=0.0)
    h.iterate(3)
    with pytest.raises(gpu_lib.SVTError) as e:
        h.grad(3, 0, [0], [1], [1.0])
    assert e.value.status == gpu_lib.SVT_E_STATE
    h.close()
