"""GPU parity of the device reverse sweep (svt_grad) against the FP64 oracle's adjoints: the exact
derivative of the unrolled iteration (oracle grad_exact, pinned to central differences of the
oracle's own iteration) and the frozen-basis one (oracle grad, pinned to central differences of a
frozen-basis forward and to torch autograd through an exact SVD), both on the CPU.

Bar: dtau, ddelta and dL/dA within 1e-8 relative (max-abs error over max-abs value).  The
gradient divides by gaps s_i - s_j between singular values, so the 1e-10 bar of the forward
values grows by the inverse relative gap; 1e-8 leaves a factor of 100 for it on these problems.
"""
import numpy as np
import pytest

import svt_workloads as W
from oracle import Params, Problem
from oracle.adjoint import forward_record, grad, grad_exact

pytestmark = pytest.mark.gpu

TOL = 1e-8

CASES = [
    # (m, n, rank, frac, seed, extra params, T)
    (36, 30, 2, 0.5, 71, {"t0": 3, "dt": 4}, 6),
    (90, 70, 3, 0.4, 31, {}, 8),                   # a growth block and an annealing step at the end
    (80, 60, 6, 0.5, 73, {"t0": 40, "dt": 8}, 5),  # 40-column basis, k = 6
    (500, 400, 2, 0.04, 36, {"t0": 12}, 8),        # 4% observed, basis grows 12 -> 52
    (120, 110, 5, 0.5, 74, {"t0": 90, "dt": 12, "eps_thr0": 1e-6}, 5),  # 120-column basis: many-workgroup
    # Jacobi; the basis passes rank Y = 110, so columns drop and only the frozen-basis sweep applies
]
# bases wider than 96 columns with many singular values above tau: (m, n, rank, frac, seed, extra, T, tau/sqrt(mn))
WIDE_K = [(140, 120, 40, 0.6, 75, {"t0": 100, "dt": 10}, 6, 1.2)]


def rel_err(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _setup(svt, m, n, rank, frac, seed, extra, T, nh=40, tau=None):
    w = W.tiny_dense(m, n, rank, frac, seed=seed, tau=tau)
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=seed, **extra)
    rec = forward_record(prob, p, T)
    rng = np.random.default_rng(seed + 1000)
    free = np.setdiff1d(np.arange(m * n), w.rows.astype(np.int64) * n + w.cols)
    hsel = np.sort(rng.choice(free, min(nh, free.size), replace=False))
    hr, hc = (hsel // n).astype(np.int32), (hsel % n).astype(np.int32)
    g = rng.standard_normal(hsel.size)
    h = svt.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, k0=rec["k0"], seed=seed,
                     maxit=T + 5, tol=0.0, **extra)
    h.set_replay([b for b, _ in rec["decisions"]], [int(a) for _, a in rec["decisions"]])
    st = h.iterate(T)
    assert st.iter == T
    return w, prob, p, rec, hr, hc, g, h


@pytest.mark.parametrize("convention", ["exact", "frozen"])
@pytest.mark.parametrize("m,n,rank,frac,seed,extra,T", CASES)
def test_grad_matches_oracle(gpu_lib, m, n, rank, frac, seed, extra, T, convention):
    w, prob, p, rec, hr, hc, g, h = _setup(gpu_lib, m, n, rank, frac, seed, extra, T)
    print(f"case m={m} n={n} T={T} r={[q.shape[1] for q in rec['Qs']]} {convention}", flush=True)
    frozen = convention == "frozen"
    try:
        tb, db, ab = (grad if frozen else grad_exact)(prob, p, rec, hr, hc, g)
    except ValueError:
        # the run dropped columns (the basis reached rank Y): the exact sweep is not defined there
        # and the device refuses it
        assert not frozen
        with pytest.raises(gpu_lib.SVTError) as e:
            h.grad(T, 0, hr, hc, g)
        assert e.value.status == gpu_lib.SVT_E_STATE
        return
    gt, gd, ga = h.grad(T, 0, hr, hc, g, frozen_basis=frozen)
    assert abs(gt - tb) <= TOL * max(abs(tb), 1e-12), ("dtau", gt, tb)
    assert abs(gd - db) <= TOL * max(abs(db), 1e-12), ("ddelta", gd, db)
    assert rel_err(ga, ab) <= TOL, ("da", rel_err(ga, ab))


@pytest.mark.parametrize("convention", ["exact", "frozen"])
@pytest.mark.parametrize("m,n,rank,frac,seed,extra,T,c", WIDE_K)
def test_grad_wide_basis_many_values_above_tau(gpu_lib, m, n, rank, frac, seed, extra, T, c, convention):
    """A 100-column basis with 74 singular values above tau: every Gram is diagonalised by the
    many-workgroup Jacobi, and the coefficient block spans 2 k + r = 248 columns."""
    w, prob, p, rec, hr, hc, g, h = _setup(gpu_lib, m, n, rank, frac, seed, extra, T,
                                           tau=c * np.sqrt(m * n))
    print(f"case m={m} n={n} T={T} r={[q.shape[1] for q in rec['Qs']]} k={rec['final_info'].k}", flush=True)
    frozen = convention == "frozen"
    tb, db, ab = (grad if frozen else grad_exact)(prob, p, rec, hr, hc, g)
    gt, gd, ga = h.grad(T, 0, hr, hc, g, frozen_basis=frozen)
    assert abs(gt - tb) <= TOL * max(abs(tb), 1e-12), ("dtau", gt, tb)
    assert abs(gd - db) <= TOL * max(abs(db), 1e-12), ("ddelta", gd, db)
    assert rel_err(ga, ab) <= TOL, ("da", rel_err(ga, ab))


def test_checkpoint_interval_does_not_change_the_result(gpu_lib):
    """The recompute replays the same launches on the same values, so every interval gives the
    bit-identical gradient; the handle's own state is untouched by the call."""
    w, prob, p, rec, hr, hc, g, h = _setup(gpu_lib, 90, 70, 3, 0.4, 31, {}, 8)
    before = h.get_state()
    ref = h.grad(8, 1, hr, hc, g)
    for ck in (0, 2, 3, 8, 50):
        out = h.grad(8, ck, hr, hc, g)
        assert out[0] == ref[0] and out[1] == ref[1], ck
        assert np.array_equal(out[2], ref[2]), ck
    after = h.get_state()
    assert np.array_equal(before["y"], after["y"]) and before["r"] == after["r"]
    # a prefix of the run: T smaller than the iterations done
    tb, db, ab = grad_exact(prob, p, dict(rec, Qs=rec["Qs"][:5], decisions=rec["decisions"][:5]), hr, hc, g)
    gt, gd, ga = h.grad(5, 0, hr, hc, g)
    assert abs(gt - tb) <= TOL * abs(tb) and abs(gd - db) <= TOL * abs(db)
    assert rel_err(ga, ab) <= TOL


def test_repeated_held_out_entries_add_up(gpu_lib):
    w, prob, p, rec, hr, hc, g, h = _setup(gpu_lib, 36, 30, 2, 0.5, 71, {"t0": 3, "dt": 4}, 6, nh=10)
    one = h.grad(6, 0, hr, hc, g)
    two = h.grad(6, 0, np.concatenate([hr, hr]), np.concatenate([hc, hc]), np.concatenate([g, g]))
    assert abs(two[0] - 2 * one[0]) <= 1e-12 * abs(one[0])
    assert rel_err(two[2], 2 * one[2]) <= 1e-12
    zero = h.grad(6, 0, hr[:0], hc[:0], g[:0])
    assert zero[0] == 0.0 and zero[1] == 0.0 and not zero[2].any()


def test_grad_error_paths(gpu_lib):
    svt = gpu_lib
    w, prob, p, rec, hr, hc, g, h = _setup(svt, 36, 30, 2, 0.5, 71, {"t0": 3, "dt": 4}, 6, nh=10)
    with pytest.raises(svt.SVTError) as e:
        h.grad(7, 0, hr, hc, g)
    assert e.value.status == svt.SVT_E_STATE
    with pytest.raises(svt.SVTError) as e:
        h.grad(0, 0, hr, hc, g)
    assert e.value.status == svt.SVT_E_INVALID_ARG
    bad = hr.copy()
    bad[0] = w.m
    with pytest.raises(svt.SVTError) as e:
        h.grad(6, 0, bad, hc, g)
    assert e.value.status == svt.SVT_E_INVALID_ARG
    s = h.get_state()
    h.set_state(s["y"], s["Q"], s["eps_thr"], s["eps_min"], s["iter"])
    with pytest.raises(svt.SVTError) as e:
        h.grad(6, 0, hr, hc, g)
    assert e.value.status == svt.SVT_E_STATE
    hm = svt.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, k0=rec["k0"], seed=71, t0=3, dt=4,
                      precision=svt.SVT_MIXED, tol=0.0)
    hm.iterate(2)
    with pytest.raises(svt.SVTError) as e:
        hm.grad(2, 0, hr, hc, g)
    assert e.value.status == svt.SVT_E_STATE
    # power iterations: the exact sweep refuses, the frozen-basis one runs
    hp = svt.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, k0=rec["k0"], seed=71, t0=3, dt=4,
                      npow=1, tol=0.0)
    hp.iterate(3)
    with pytest.raises(svt.SVTError) as e:
        hp.grad(3, 0, hr, hc, g)
    assert e.value.status == svt.SVT_E_STATE
    hp.grad(3, 0, hr, hc, g, frozen_basis=True)
    # unknown flag bits
    import ctypes as C
    from paper_1704_05528_amd import _capi
    out = (C.c_double(), C.c_double(), np.zeros(w.nnz))
    st = svt.load().svt_grad(h._h, 6, 0, 0, None, None, None, 4, C.byref(out[0]), C.byref(out[1]),
                             out[2].ctypes.data_as(C.POINTER(C.c_double)))
    assert st == _capi.SVT_E_INVALID_ARG


def test_autograd_function(gpu_lib):
    """torch.autograd through SVTHeldOut gives the oracle's gradient of a held-out loss."""
    import torch

    from paper_1704_05528_amd.autograd import svt_heldout
    m, n, seed, T = 90, 70, 31, 6
    w = W.tiny_dense(m, n, 3, 0.4, seed=seed)
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=seed)
    rec = forward_record(prob, p, T)
    rng = np.random.default_rng(7)
    free = np.setdiff1d(np.arange(m * n), w.rows.astype(np.int64) * n + w.cols)
    hsel = np.sort(rng.choice(free, 50, replace=False))
    hr, hc = (hsel // n).astype(np.int32), (hsel % n).astype(np.int32)
    target = rng.standard_normal(hsel.size)
    # dL/dX_T on H = x - target, with x the oracle's X_T on H
    xo = rec["final_info"]
    from oracle.adjoint import frozen_forward
    x_or = frozen_forward(prob, prob.a, p.tau, p.delta, rec["k0"], rec["Qs"], hr, hc)
    for frozen, oracle_grad in ((False, grad_exact), (True, grad)):
        a = torch.tensor(w.a, dtype=torch.float64, requires_grad=True)
        tau = torch.tensor(w.tau, dtype=torch.float64, requires_grad=True)
        delta = torch.tensor(w.delta, dtype=torch.float64, requires_grad=True)
        x = svt_heldout(a, tau, delta, m, n, w.rows, w.cols, hr, hc, T, frozen_basis=frozen, seed=seed,
                        k0=rec["k0"])
        loss = 0.5 * ((x - torch.from_numpy(target)) ** 2).sum()
        loss.backward()
        assert rel_err(x.detach().numpy(), x_or) <= 1e-10
        tb, db, ab = oracle_grad(prob, p, rec, hr, hc, x_or - target)
        assert abs(tau.grad.item() - tb) <= TOL * abs(tb), frozen
        assert abs(delta.grad.item() - db) <= TOL * abs(db), frozen
        assert rel_err(a.grad.numpy(), ab) <= TOL, frozen
    assert xo.it == T


def test_image_derivative_workload_T50_checkpoint10(gpu_lib):
    """The derivative workload at full size: the 1024 x 1024 image, 50 unrolled iterations,
    checkpoints every 10, RMSE on the 52,428 held-out pixels.  Reference values come from the FP64
    oracle (tests/golden/make_image_adjoint.py): its exact and frozen-basis reverse sweeps on a seeded
    sample of 4096 observed positions (and the norm and sum of dL/da), central differences of its own
    iteration (exact) and of the frozen-basis forward (frozen).  The device replays the oracle's
    decisions; its X_T on H must agree to 1e-10 and the gradients to 1e-8; against the differences
    the bar is 1e-6 (truncation and rounding of a relative step of 1e-6)."""
    import os
    svt = gpu_lib
    ref = np.load(os.path.join(os.path.dirname(__file__), "golden", "image_adjoint_T50.npz"))
    T = int(ref["T"])
    w = W.image_adjoint()
    print(f"image derivative workload: T={T} ckpt=10 |H|={w.held_rows.size}", flush=True)
    h = svt.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, k0=int(ref["k0"]),
                     seed=int(ref["seed"]), maxit=T + 5, tol=0.0)
    h.set_replay(ref["blocks"], ref["annealed"])
    st = h.iterate(T)
    assert st.iter == T and [x.r for x in h.history()] == list(ref["r"])
    x = h.sample(w.held_rows, w.held_cols)
    assert rel_err(x[ref["h_sample"]], ref["x_h_sample"]) <= 1e-10
    L0 = float(np.sqrt(np.mean((x - w.held_a) ** 2)))
    g = (x - w.held_a) / (x.size * L0)
    rng_dirs = np.random.default_rng(int(ref["fd_real_dir_seed"])).standard_normal((2, w.nnz))
    for frozen in (False, True):
        dt_, dd_, da_ = h.grad(T, 10, w.held_rows, w.held_cols, g, frozen_basis=frozen)
        pre = "" if frozen else "exact_"
        assert abs(dt_ - float(ref[pre + "dtau"])) <= TOL * abs(float(ref[pre + "dtau"])), (frozen, dt_)
        assert abs(dd_ - float(ref[pre + "ddelta"])) <= TOL * abs(float(ref[pre + "ddelta"])), (frozen, dd_)
        assert rel_err(da_[ref["da_sample_pos"]], ref[pre + "da_sample"]) <= TOL, frozen
        assert abs(np.linalg.norm(da_) - float(ref[pre + "da_norm"])) <= TOL * float(ref[pre + "da_norm"])
        if frozen:
            fd_t, fd_d = float(ref["fd_tau"]), float(ref["fd_delta"])
            dirs = np.random.default_rng(int(ref["fd_dir_seed"])).standard_normal((3, w.nnz))
            fd_v = ref["fd_dir"]
        else:
            fd_t, fd_d = float(ref["fd_real_tau"]), float(ref["fd_real_delta"])
            dirs, fd_v = rng_dirs, ref["fd_real_dir"]
        assert abs(dt_ - fd_t) <= 1e-6 * abs(fd_t), (frozen, dt_, fd_t)
        assert abs(dd_ - fd_d) <= 1e-6 * abs(fd_d), (frozen, dd_, fd_d)
        for v, fd in zip(dirs, fd_v):
            assert abs(da_ @ v - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.linalg.norm(da_)), (frozen, da_ @ v, fd)
