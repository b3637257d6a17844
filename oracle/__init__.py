"""FP64 CPU oracle of SVT with recycling rank-revealing randomized SVD.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The device library
never calls it, and it shares no code with the device library.

Modules
  philox  -- Philox4x64-10 + Box-Muller Gaussian blocks (the Omega stream)
  svt     -- exact D_tau (Eq. 5), SVT with full SVD, R3SVD/R4SVD (Alg. 2, 3),
             Fast SVT (Alg. 4) with decision trace and replay
  mixed   -- the reduced-precision form with explicit rounding points
  adjoint -- reverse-mode derivative of the unrolled iteration (frozen basis)

Parity status: every function is pinned by tests/test_oracle_pins.py except
the match with the paper's whole-run numbers (images and MovieLens are not
available): parity unpinned for those.
"""
from .philox import omega_block, philox4x64_10, philox4x64_10_array
from .svt import (Params, Problem, State, StepInfo, d_tau, dense, initial_state, kicking_k0, r4svd,
                  spectral_norm, svt_exact_run, svt_exact_step, svt_run, svt_step)
