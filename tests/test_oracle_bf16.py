"""Pins of the emulated BF16 form of the oracle (CPU only).

- the rounding against torch's float32 -> bfloat16 conversion (round to nearest even) and against
  hand-checked ties
- the energy ||B_o||_F^2 = trace(L^{-1} W^T W L^{-T}) against the squared norm of the orthogonal
  projection of Y onto span(Q^), formed from an orthonormal basis of that span taken by an SVD
  (scipy.linalg.orth), so a wrong transpose or a dropped L^{-1} shows
- the step with an exactly representable orthonormal basis (coordinate vectors) equals the float32
  mixed step from the same state, where the projector correction is the identity
- whole runs: the error percentage of Eq. 10 never goes below float32 noise (the energy of the
  projection never exceeds ||Y||^2), and a planted problem reaches relative residual 1e-4 in about the FP64
  iteration count; without the correction (||W||^2 in place of ||B_o||^2) the energy does exceed
  ||Y||^2 on the same run
"""
import numpy as np
import pytest
import scipy.linalg as sla

import svt_workloads as W
from oracle import Params, Problem, State, initial_state, svt_step
from oracle.mixed import bf16, f32, projected_energy, svt_step_bf16, svt_step_mixed


def test_bf16_rounding_matches_torch_and_ties():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(4000) * 10.0 ** rng.integers(-6, 6, 4000),
                        [0.0, -0.0, 1.0, -1.0, 65504.0, 1e-30]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(bf16(x), ref)
    # ties go to the even mantissa: 1 + 2^-8 -> 1, 1 + 3 2^-8 -> 1 + 2^-6
    np.testing.assert_array_equal(bf16([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8)]),
                                  [1.0, 1 + 2.0 ** -6, -1.0])


def test_projected_energy_is_the_norm_of_the_orthogonal_projection():
    rng = np.random.default_rng(7)
    m, n, r = 60, 45, 12
    Q, _ = np.linalg.qr(rng.standard_normal((m, r)))
    Qh = bf16(Q)
    assert np.abs(Qh.T @ Qh - np.eye(r)).max() > 1e-4  # rounding really leaves the basis non-orthonormal
    Y = rng.standard_normal((m, n))
    L, e = projected_energy(Qh, Y.T @ Qh)
    O = sla.orth(Qh)  # orthonormal basis of span(Q^) from an SVD
    assert O.shape[1] == r
    ref = float(np.sum((O.T @ Y) ** 2))
    assert abs(e - ref) <= 1e-12 * ref
    # and L is the Cholesky factor of Q^T Q^ (lower, positive diagonal)
    np.testing.assert_allclose(L @ L.T, Qh.T @ Qh, rtol=0, atol=1e-14)
    assert np.allclose(L, np.tril(L)) and (np.diag(L) > 0).all()


def test_bf16_step_with_coordinate_basis_equals_mixed_step():
    w = W.tiny_dense(50, 40, 3, 0.5, seed=13)
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=3)
    s0, _ = initial_state(prob, p)
    rng = np.random.default_rng(2)
    Q = np.eye(w.m)[:, rng.choice(w.m, 20, replace=False)]  # exact in bfloat16 and orthonormal
    st = State(it=4, y=f32(s0.y), Q=Q, eps_thr=0.2, eps_min=np.inf)
    nb, ib = svt_step_bf16(prob, p, st, replay=(0, False))
    nm, im = svt_step_mixed(prob, p, st, replay=(0, False))
    assert ib.k == im.k and ib.r == im.r == 20
    assert abs(ib.normB - im.normB) <= 1e-12 * im.normB
    np.testing.assert_allclose(ib.x, im.x, rtol=0, atol=1e-6 * np.abs(im.x).max())
    np.testing.assert_allclose(nb.y, nm.y, rtol=0, atol=1e-6 * np.abs(nm.y).max())


def _run(step, prob, p, T):
    state, _ = initial_state(prob, p)
    out = []
    for _ in range(T):
        state, info = step(prob, p, state)
        out.append(info)
        if info.stopped:
            break
    return out


def test_bf16_runs_keep_the_energy_identity_and_converge():
    w = W.tiny_dense(120, 100, 4, 0.4, seed=31)
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=8, maxit=400, tol=1e-4)
    r64 = _run(svt_step, prob, p, 400)
    rb = _run(svt_step_bf16, prob, p, 400)
    assert r64[-1].stopped and rb[-1].stopped
    assert len(rb) <= int(1.25 * len(r64)) + 5
    # float32 noise only (W is stored in float32): once the basis spans R^m, ||B_o||^2 = ||Y||^2
    assert min(min(i.eps_hist) for i in rb) >= -1e-6
    # the uncorrected energy of the same stored bases exceeds ||Y||^2 by far more than that
    over = max(float(np.sum(i.W * i.W)) / i.normY for i in rb)
    assert over > 1.0 + 5e-6
    # and the stored basis really is bfloat16 and not orthonormal
    Qh = rb[-1].Q
    np.testing.assert_array_equal(Qh, bf16(Qh))
    assert np.abs(Qh.T @ Qh - np.eye(Qh.shape[1])).max() > 1e-4
