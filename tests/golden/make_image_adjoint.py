"""Writes image_adjoint_T50.npz: the oracle's reference values for the derivative workload.

The derivative workload is the 1024 x 1024 image-recovery matrix (50% observed) with a held-out
set H of 5% of the pixels drawn from the unobserved half; the loss is the RMSE of X_T on H after
T = 50 unrolled SVT iterations.  Everything here comes from the FP64 oracle (oracle/ only):

  * the discrete decisions of the oracle's run (growth blocks and annealing per iteration, and the
    kicking count), so the device can replay them;
  * X_T on a seeded sample of H (forward parity);
  * the exact reverse sweep through the unrolled iteration (basis construction included) and the
    frozen-basis one: dL/dtau, dL/ddelta, dL/da on a seeded sample of 4096 observed positions, and
    the norm and sum of dL/da;
  * central finite differences (relative step 1e-6, float64) of the frozen-basis forward in tau,
    delta and three seeded random directions of a;
  * central finite differences of the oracle's real unrolled iteration (bases recomputed from the
    perturbed iterates, decisions replayed) in tau, delta and two seeded random directions of a:
    the derivative the exact sweep computes and the frozen-basis convention approximates.

Run from the repository root:  python tests/golden/make_image_adjoint.py   (several minutes)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import svt_workloads as W  # noqa: E402
from oracle import Params, Problem, initial_state, svt_step  # noqa: E402
from oracle.adjoint import forward_record, frozen_forward, grad, grad_exact  # noqa: E402

T = 50
SEED = 11          # Omega stream key
H_STEP = 1e-6      # relative step of the central differences
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "image_adjoint_T50.npz")


def rmse(x, ref):
    return float(np.sqrt(np.mean((x - ref) ** 2)))


def real_x_on_h(prob, p, k0, replay, hr, hc, a=None):
    """X_T on H from T steps of the oracle (R4SVD bases recomputed) with replayed decisions."""
    pp = Params(**{**p.__dict__, "k0": k0})
    if a is not None:
        prob = Problem(prob.m, prob.n, prob.rows, prob.cols, a)
    state, _ = initial_state(prob, pp)
    info = None
    for i in range(T):
        state, info = svt_step(prob, pp, state, replay[i])
    X = (info.U * info.s_minus_tau) @ info.V.T if info.k > 0 else np.zeros((prob.m, prob.n))
    return X[hr, hc]


def main():
    t0 = time.time()
    w = W.image_adjoint()
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=SEED, maxit=T + 5, tol=0.0)
    rec = forward_record(prob, p, T)
    hr, hc, ah = w.held_rows.astype(np.int64), w.held_cols.astype(np.int64), w.held_a
    info = rec["final_info"]
    X_T = (info.U * info.s_minus_tau) @ info.V.T
    x_h = X_T[hr, hc]
    L0 = rmse(x_h, ah)
    g = (x_h - ah) / (x_h.size * L0)
    print(f"forward {time.time() - t0:.0f} s, r = {[q.shape[1] for q in rec['Qs']][::10]}, RMSE {L0:.6e}", flush=True)
    tb, db, ab = grad(prob, p, rec, hr, hc, g)
    print(f"frozen-basis adjoint {time.time() - t0:.0f} s: dtau {tb:.6e} ddelta {db:.6e}", flush=True)
    te, de, ae = grad_exact(prob, p, rec, hr, hc, g)
    print(f"exact adjoint {time.time() - t0:.0f} s: dtau {te:.6e} ddelta {de:.6e}", flush=True)

    def L_frozen(a, tau, delta):
        return rmse(frozen_forward(prob, a, tau, delta, rec["k0"], rec["Qs"], hr, hc), ah)

    h = H_STEP
    fd_tau = (L_frozen(prob.a, p.tau * (1 + h), p.delta) - L_frozen(prob.a, p.tau * (1 - h), p.delta)) / (2 * h * p.tau)
    fd_delta = (L_frozen(prob.a, p.tau, p.delta * (1 + h)) - L_frozen(prob.a, p.tau, p.delta * (1 - h))) / (2 * h * p.delta)
    rng = np.random.default_rng(2024)
    scale = float(np.abs(prob.a).max())
    dirs = rng.standard_normal((3, prob.a.size))
    fd_dir = []
    for v in dirs:
        fd_dir.append((L_frozen(prob.a + h * scale * v, p.tau, p.delta)
                       - L_frozen(prob.a - h * scale * v, p.tau, p.delta)) / (2 * h * scale))
    print(f"frozen differences {time.time() - t0:.0f} s", flush=True)
    replay = [(b, a) for b, a in rec["decisions"]]
    fd_real_tau = (rmse(real_x_on_h(prob, Params(**{**p.__dict__, "tau": p.tau * (1 + h)}), rec["k0"], replay, hr, hc), ah)
                   - rmse(real_x_on_h(prob, Params(**{**p.__dict__, "tau": p.tau * (1 - h)}), rec["k0"], replay, hr, hc), ah)
                   ) / (2 * h * p.tau)
    fd_real_delta = (rmse(real_x_on_h(prob, Params(**{**p.__dict__, "delta": p.delta * (1 + h)}), rec["k0"], replay, hr, hc), ah)
                     - rmse(real_x_on_h(prob, Params(**{**p.__dict__, "delta": p.delta * (1 - h)}), rec["k0"], replay, hr, hc), ah)
                     ) / (2 * h * p.delta)
    dirs_real = np.random.default_rng(2025).standard_normal((2, prob.a.size))
    fd_real_dir = []
    for v in dirs_real:
        fd_real_dir.append((rmse(real_x_on_h(prob, p, rec["k0"], replay, hr, hc, prob.a + h * scale * v), ah)
                            - rmse(real_x_on_h(prob, p, rec["k0"], replay, hr, hc, prob.a - h * scale * v), ah))
                           / (2 * h * scale))
    print(f"real-iteration differences {time.time() - t0:.0f} s", flush=True)
    sample = np.sort(np.random.default_rng(7).choice(prob.a.size, 4096, replace=False))
    hsample = np.sort(np.random.default_rng(8).choice(hr.size, 2048, replace=False))
    np.savez_compressed(
        OUT, T=T, seed=SEED, k0=rec["k0"], blocks=np.array([b for b, _ in rec["decisions"]], np.int32),
        annealed=np.array([int(a) for _, a in rec["decisions"]], np.int32),
        r=np.array([q.shape[1] for q in rec["Qs"]], np.int32), k_last=info.k, rmse=L0,
        h_sample=hsample, x_h_sample=x_h[hsample],
        dtau=tb, ddelta=db, da_sample_pos=sample, da_sample=ab[sample], da_norm=float(np.linalg.norm(ab)),
        da_sum=float(ab.sum()), fd_step=h, fd_tau=fd_tau, fd_delta=fd_delta, fd_dir_seed=2024,
        fd_dir=np.array(fd_dir), fd_real_tau=fd_real_tau, fd_real_delta=fd_real_delta,
        exact_dtau=te, exact_ddelta=de, exact_da_sample=ae[sample], exact_da_norm=float(np.linalg.norm(ae)),
        exact_da_sum=float(ae.sum()), fd_real_dir_seed=2025, fd_real_dir=np.array(fd_real_dir),
        exact_dir_dots=np.array([float(ae @ v) for v in dirs_real]))
    print(f"wrote {OUT} after {time.time() - t0:.0f} s", flush=True)
    print(f"frozen: dtau {tb:.9e} fd {fd_tau:.9e}; ddelta {db:.9e} fd {fd_delta:.9e}; "
          f"dirs {[float(ab @ v) for v in dirs]} fd {fd_dir}")
    print(f"exact: dtau {te:.9e} real fd {fd_real_tau:.9e}; ddelta {de:.9e} real fd {fd_real_delta:.9e}; "
          f"dirs {[float(ae @ v) for v in dirs_real]} real fd {fd_real_dir}")


if __name__ == "__main__":
    main()
