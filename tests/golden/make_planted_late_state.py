"""Writes planted_late_state.npz: an oracle state of the planted 1000 x 1000 rank-10 problem once its
basis has grown to all m = 1000 columns, and the oracle's next step from it.

Once r = m the recycled basis spans R^m, so the state is Y on Lambda plus the thresholds (any
orthonormal basis of R^m, e.g. the identity, gives the same next step).  The oracle (oracle/ only)
runs from the kicking start with Omega seed 11 until r = 1000; the file holds that state and, for
the following step, x on Lambda at a seeded sample of 20,000 positions, the relative residual,
k and the singular values above tau.

Run from the repository root:  python tests/golden/make_planted_late_state.py   (a few minutes)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import svt_workloads as W  # noqa: E402
from oracle import Params, Problem, State, initial_state, svt_step  # noqa: E402

SEED = 11
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "planted_late_state.npz")


def main():
    t0 = time.time()
    w = W.planted()
    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, seed=SEED, tol=w.tol, maxit=1000)
    state, k0 = initial_state(prob, p)
    info = None
    while True:
        state, info = svt_step(prob, p, state)
        if info.stopped:
            raise RuntimeError("converged before the basis filled R^m")
        if info.r == w.m:
            break
    print(f"r = m after iteration {state.it} ({time.time() - t0:.0f} s), rel {info.rel:.4e}", flush=True)
    # the next step from this state, with the basis replaced by the identity (same span)
    start = State(it=state.it, y=state.y.copy(), Q=np.eye(w.m), eps_thr=state.eps_thr, eps_min=state.eps_min)
    nxt, ni = svt_step(prob, p, start)
    sample = np.sort(np.random.default_rng(12).choice(prob.a.size, 20_000, replace=False))
    np.savez_compressed(OUT, seed=SEED, k0=k0, it=state.it, y=state.y, eps_thr=state.eps_thr,
                        eps_min=state.eps_min, x_sample_pos=sample, x_sample=ni.x[sample], rel=ni.rel, k=ni.k,
                        r=ni.r, blocks=ni.blocks, annealed=int(ni.annealed), sigma_k=ni.sigma[:ni.k],
                        y_next_sample=nxt.y[sample])
    print(f"wrote {OUT} ({time.time() - t0:.0f} s): next step k={ni.k} rel={ni.rel:.6e}", flush=True)


if __name__ == "__main__":
    main()
