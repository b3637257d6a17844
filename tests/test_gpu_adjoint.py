"""GPU parity of the device reverse sweep (svt_grad, frozen-basis convention) against the FP64
oracle's adjoint, which is itself pinned to central finite differences and to torch autograd
through an exact SVD on the CPU.

Bar: dtau, ddelta and dL/dA within 1e-8 relative (max-abs error over max-abs value).  The
gradient divides by gaps s_i - s_j between singular values, so the 1e-10 bar of the forward
values grows by the inverse relative gap; 1e-8 leaves a factor of 100 for it on these problems.
"""
import numpy as np
import pytest

import svt_workloads as W
from oracle import Params, Problem
from oracle.adjoint import forward_record, grad

pytestmark = pytest.mark.gpu

TOL = 1e-8

CASES = [
    # (m, n, rank, frac, seed, extra params, T)
    (36, 30, 2, 0.5, 71, {"t0": 3, "dt": 4}, 6),
    (90, 70, 3, 0.4, 31, {}, 8),                   # a growth block and an annealing step at the end
    (80, 60, 6, 0.5, 73, {"t0": 40, "dt": 8}, 5),  # 40-column basis, k = 6
    (500, 400, 2, 0.04, 36, {"t0": 12}, 8),        # 4% observed, basis grows 12 -> 52
    (120, 110, 5, 0.5, 74, {"t0": 90, "dt": 12, "eps_thr0": 1e-6}, 5),  # 120-column basis: many-workgroup Jacobi
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


@pytest.mark.parametrize("m,n,rank,frac,seed,extra,T", CASES)
def test_grad_matches_oracle(gpu_lib, m, n, rank, frac, seed, extra, T):
    w, prob, p, rec, hr, hc, g, h = _setup(gpu_lib, m, n, rank, frac, seed, extra, T)
    print(f"case m={m} n={n} T={T} r={[q.shape[1] for q in rec['Qs']]}", flush=True)
    tb, db, ab = grad(prob, p, rec, hr, hc, g)
    gt, gd, ga = h.grad(T, 0, hr, hc, g)
    assert abs(gt - tb) <= TOL * max(abs(tb), 1e-12), ("dtau", gt, tb)
    assert abs(gd - db) <= TOL * max(abs(db), 1e-12), ("ddelta", gd, db)
    assert rel_err(ga, ab) <= TOL, ("da", rel_err(ga, ab))


@pytest.mark.parametrize("m,n,rank,frac,seed,extra,T,c", WIDE_K)
def test_grad_wide_basis_many_values_above_tau(gpu_lib, m, n, rank, frac, seed, extra, T, c):
    """A 100-column basis with 74 singular values above tau: every Gram is diagonalised by the
    many-workgroup Jacobi, and the coefficient block spans 2 k + r = 248 columns."""
    w, prob, p, rec, hr, hc, g, h = _setup(gpu_lib, m, n, rank, frac, seed, extra, T,
                                           tau=c * np.sqrt(m * n))
    print(f"case m={m} n={n} T={T} r={[q.shape[1] for q in rec['Qs']]} k={rec['final_info'].k}", flush=True)
    tb, db, ab = grad(prob, p, rec, hr, hc, g)
    gt, gd, ga = h.grad(T, 0, hr, hc, g)
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
    tb, db, ab = grad(prob, p, dict(rec, Qs=rec["Qs"][:5]), hr, hc, g)
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
    a = torch.tensor(w.a, dtype=torch.float64, requires_grad=True)
    tau = torch.tensor(w.tau, dtype=torch.float64, requires_grad=True)
    delta = torch.tensor(w.delta, dtype=torch.float64, requires_grad=True)
    x = svt_heldout(a, tau, delta, m, n, w.rows, w.cols, hr, hc, T, seed=seed, k0=rec["k0"])
    loss = 0.5 * ((x - torch.from_numpy(target)) ** 2).sum()
    loss.backward()
    # dL/dX_T on H = x - target, with x the oracle's X_T on H
    xo = rec["final_info"]
    from oracle.adjoint import frozen_forward
    x_or = frozen_forward(prob, prob.a, p.tau, p.delta, rec["k0"], rec["Qs"], hr, hc)
    assert rel_err(x.detach().numpy(), x_or) <= 1e-10
    tb, db, ab = grad(prob, p, rec, hr, hc, x_or - target)
    assert abs(tau.grad.item() - tb) <= TOL * abs(tb)
    assert abs(delta.grad.item() - db) <= TOL * abs(db)
    assert rel_err(a.grad.numpy(), ab) <= TOL
    assert xo.it == T
