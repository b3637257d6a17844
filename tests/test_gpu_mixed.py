"""GPU parity of the mixed form (float32 storage and sparse accumulation, float64 Gram / Cholesky /
eigen-solver / norms) against the emulated-precision oracle, and its error against the FP64 oracle.

Bars: against the emulated oracle, values within 2e-5 relative (float32 accumulation-order noise,
about sqrt(row length) x 6e-8, amplified by the conditioning of the step); against the FP64
oracle the same step stays within 1e-4 relative; integers (r, k, blocks) exact.
"""
import math

import numpy as np
import pytest

import svt_workloads as W
from oracle import Params, Problem, State, initial_state, svt_run, svt_step
from oracle.mixed import f32, svt_step_mixed
from oracle.svt import kicking_k0, spectral_norm

pytestmark = pytest.mark.gpu

TOL_EMU = 2e-5
TOL_FP64 = 1e-4


def rel_err(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _state_after(prob, p, steps):
    state, k0 = initial_state(prob, p)
    for _ in range(steps):
        state, _ = svt_step(prob, p, state)
    return state, k0


@pytest.mark.parametrize("m,n,rank,frac,seed,steps", [(90, 70, 3, 0.4, 61, 6), (130, 110, 4, 0.35, 62, 14),
                                                      (200, 150, 3, 0.3, 63, 25)])
def test_mixed_step_against_emulated_and_fp64_oracle(gpu_lib, m, n, rank, frac, seed, steps):
    w = W.tiny_dense(m, n, rank, frac, seed=seed)
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=seed)
    s64, k0 = _state_after(prob, p, steps)
    st32 = State(it=s64.it, y=f32(s64.y), Q=f32(s64.Q), eps_thr=s64.eps_thr, eps_min=s64.eps_min)
    nxt_emu, info_emu = svt_step_mixed(prob, p, st32)
    _, info_64 = svt_step(prob, p, st32)
    h = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, k0=k0, seed=seed,
                         precision=gpu_lib.SVT_MIXED)
    h.set_state(st32.y, st32.Q, st32.eps_thr, st32.eps_min, st32.it)
    st = h.iterate(1)
    x = h.sample(w.rows, w.cols)
    assert st.r == info_emu.r and st.k == info_emu.k and st.blocks == info_emu.blocks
    assert rel_err(x, info_emu.x) <= TOL_EMU, rel_err(x, info_emu.x)
    assert abs(st.rel_res - info_emu.rel) <= TOL_EMU * info_emu.rel
    assert abs(st.eps - info_emu.eps) <= 1e-6
    assert rel_err(h.get_state()["y"], nxt_emu.y) <= TOL_EMU
    # stated error of the mixed form against the FP64 step from the same state
    assert rel_err(x, info_64.x) <= TOL_FP64
    assert abs(st.rel_res - info_64.rel) <= TOL_FP64 * info_64.rel


def test_mixed_free_run_with_replay_tracks_fp64(gpu_lib):
    """30 iterations of the mixed form with the FP64 oracle's decisions replayed: the residual
    trajectory stays within 1e-4 relative of the FP64 one."""
    w = W.tiny_dense(120, 100, 3, 0.4, seed=64)
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=3, maxit=30)
    _, infos, k0 = svt_run(prob, p, keep_infos=True)
    h = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, k0=k0, seed=3, maxit=30,
                         precision=gpu_lib.SVT_MIXED)
    h.set_replay([i.blocks for i in infos], [int(i.annealed) for i in infos])
    worst = 0.0
    for info in infos:
        st = h.iterate(1)
        assert st.r == info.r and st.k == info.k
        worst = max(worst, abs(st.rel_res - info.rel) / info.rel)
    assert worst <= TOL_FP64, worst


def test_mixed_planted_reaches_tolerance(gpu_lib):
    """The mixed form reaches relative residual 1e-4 on a planted problem (float32 storage is far
    below the tolerance)."""
    w = W.tiny_dense(150, 150, 3, 0.4, seed=65)
    h = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, seed=1, maxit=800,
                         precision=gpu_lib.SVT_MIXED)
    st = h.iterate(800)
    assert st.stopped and st.rel_res < 1e-4
    k, s, U, V = h.factors()
    X = (U * s) @ V.T
    assert np.linalg.norm(X - w.A) / np.linalg.norm(w.A) < 2e-3


@pytest.mark.parametrize("m,n,frac,seed", [(100, 90, 0.3, 49), (160, 120, 0.5, 64)])
def test_mixed_kicking_start_matches_oracle(gpu_lib, m, n, frac, seed):
    """The mixed form computes ||P_Lambda A||_2 by a float32 power iteration that stops at float
    precision; the kicking count k0 is an integer, so Y^(0) = k0 delta a matches the FP64 oracle to
    float32 rounding."""
    w = W.tiny_dense(m, n, 3, frac, seed=seed)
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    state, k0 = initial_state(prob, Params(tau=w.tau, delta=w.delta))
    h = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, precision=gpu_lib.SVT_MIXED)
    np.testing.assert_allclose(h.get_state()["y"], state.y, rtol=3e-7)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_diverging_step_size_stops_with_numeric_error(gpu_lib, precision):
    """A step size far above the stable bound makes Y grow without limit; once the iterate leaves
    the storage type's range the call must stop with SVT_E_NUMERIC (the mixed form's float iterate
    overflows long before the residual sums in double do)."""
    from paper_1704_05528_amd._capi import SVT_E_NUMERIC, SVTError
    w = W.tiny_dense(60, 50, 3, 0.5, seed=71, delta=40.0)
    prec = gpu_lib.SVT_MIXED if precision == "mixed" else gpu_lib.SVT_FP64
    h = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, seed=71, maxit=5000,
                         precision=prec)
    with pytest.raises(SVTError) as ei:
        h.iterate(5000)
    assert ei.value.status == SVT_E_NUMERIC, ei.value


@pytest.mark.parametrize("extra", [{"t0": 20}, {"t0": 6, "dt": 4}])
def test_mixed_step_heavy_columns_chunked_gather(gpu_lib, extra):
    """The mixed form on a 1%-observed pattern with three columns of 9000, 5000 and 2600 rows: W = Y^T Q
    on the gather path with the long columns in chunks (float partial rows added in order), wide and
    narrow blocks, one step from a state after eight FP64 steps, against the emulated oracle."""
    w = W.heavy_columns(30000, 60, 3, (9000, 5000, 2600), 40, seed=51, delta=1.2)
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=51, **extra)
    s64, k0 = _state_after(prob, p, 8)
    st32 = State(it=s64.it, y=f32(s64.y), Q=f32(s64.Q), eps_thr=s64.eps_thr, eps_min=s64.eps_min)
    nxt_emu, info_emu = svt_step_mixed(prob, p, st32)
    h = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, k0=k0, seed=51,
                         precision=gpu_lib.SVT_MIXED, **extra)
    h.set_state(st32.y, st32.Q, st32.eps_thr, st32.eps_min, st32.it)
    st = h.iterate(1)
    x = h.sample(w.rows, w.cols)
    assert info_emu.k > 0
    assert st.r == info_emu.r and st.k == info_emu.k and st.blocks == info_emu.blocks
    assert rel_err(x, info_emu.x) <= TOL_EMU, rel_err(x, info_emu.x)
    assert abs(st.rel_res - info_emu.rel) <= TOL_EMU * info_emu.rel
    assert rel_err(h.get_state()["y"], nxt_emu.y) <= TOL_EMU


def test_mixed_step_wide_basis_gram_32_tiles(gpu_lib):
    """The mixed form with a 537-column basis on 997 columns of Y: the float W gives its FP64 Gram
    matrix through the 32 x 32-tile kernel.  One step from a given state against the emulated oracle."""
    m, n, r = 700, 997, 537
    w = W.tiny_dense(m, n, 5, 0.3, seed=63, delta=1.2)
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=63, maxit=10, r_max=m)
    rng = np.random.default_rng(64)
    Q0, _ = np.linalg.qr(rng.standard_normal((m, r)))
    k0 = kicking_k0(w.tau, w.delta, spectral_norm(m, n, w.rows, w.cols, w.a))
    st32 = State(it=4, y=f32(2.0 * k0 * w.delta * w.a), Q=f32(Q0), eps_thr=0.99, eps_min=math.inf)
    nxt_emu, info_emu = svt_step_mixed(prob, p, st32)
    h = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, k0=k0, seed=63, maxit=10, r_max=m,
                         precision=gpu_lib.SVT_MIXED)
    h.set_state(st32.y, st32.Q, st32.eps_thr, st32.eps_min, st32.it)
    st = h.iterate(1)
    x = h.sample(w.rows, w.cols)
    assert info_emu.k == 5 and info_emu.blocks == 0
    assert st.r == info_emu.r and st.k == info_emu.k and st.blocks == info_emu.blocks
    assert rel_err(x, info_emu.x) <= TOL_EMU, rel_err(x, info_emu.x)
    assert abs(st.rel_res - info_emu.rel) <= TOL_EMU * info_emu.rel
    assert rel_err(h.get_state()["y"], nxt_emu.y) <= TOL_EMU


def test_mixed_form_image_size_over_the_benchmark_window(gpu_lib):
    """The reduced-precision form at the image workload's full size (1024 x 1024, 524,288 observed)
    over iterations 1-25, the window the default benchmark command times.  Step parity: each
    iteration starts the device from the emulated oracle's state and replays its two decisions;
    x on Lambda, the residual and the next Y agree at the emulated bar, integers exactly."""
    w = W.image()
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=11, maxit=30)
    s64, k0 = initial_state(prob, p)
    s32 = State(it=0, y=f32(s64.y))
    h = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, k0=k0, seed=11,
                         precision=gpu_lib.SVT_MIXED, maxit=30)
    for it in range(1, 26):
        nxt, info = svt_step_mixed(prob, p, s32)
        h.set_state(s32.y, s32.Q, math.nan if s32.eps_thr is None else s32.eps_thr, s32.eps_min, s32.it)
        h.set_replay([info.blocks], [int(info.annealed)])
        st = h.iterate(1)
        x = h.sample(w.rows, w.cols)
        print(f"iteration {it}: r={info.r} k={info.k} err={rel_err(x, info.x):.2e}", flush=True)
        assert st.r == info.r and st.k == info.k and st.blocks == info.blocks, it
        assert rel_err(x, info.x) <= TOL_EMU, (it, rel_err(x, info.x))
        assert abs(st.rel_res - info.rel) <= TOL_EMU * info.rel, it
        assert rel_err(h.get_state()["y"], nxt.y) <= TOL_EMU, it
        s32 = nxt
