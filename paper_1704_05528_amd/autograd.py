"""torch.autograd face of svt_grad: X_T on a held-out set as a differentiable function of the
observed values, tau and delta (the exact derivative of the unrolled iteration by default, the
frozen-basis one with frozen_basis=True).

    x_h = svt_heldout(a, tau, delta, m, n, rows, cols, hi, hj, T=20, seed=3)
    loss = ((x_h - target) ** 2).sum()
    loss.backward()          # a.grad, tau.grad, delta.grad from the device reverse sweep

The forward pass runs T iterations of Alg. 4 on the GPU and samples X_T on H; the backward pass
calls svt_grad on the same handle.  When a is a GPU tensor every array crosses the boundary as a
device pointer and X_T(H) and dL/da stay on the GPU; a CPU tensor goes through host memory.  Only
argument marshalling happens here.
"""
import numpy as np
import torch

from .svt import SVT


class SVTHeldOut(torch.autograd.Function):
    """(a, tau, delta) -> X_T(H) after T unrolled iterations, float64 (on a's device)."""

    @staticmethod
    def forward(ctx, a, tau, delta, m, n, rows, cols, hi, hj, T, ckpt, params, frozen_basis):
        dev = a.is_cuda
        if dev:
            def idx(v):
                return torch.as_tensor(v, dtype=torch.int32, device=a.device).contiguous()
            vals = a.detach().contiguous()
            if vals.dtype not in (torch.float64, torch.float32):
                vals = vals.to(torch.float64)
            rows, cols, hi, hj = idx(rows), idx(cols), idx(hi), idx(hj)
        else:
            vals = a.detach().to(torch.float64).numpy()
            hi = np.ascontiguousarray(hi, dtype=np.int32)
            hj = np.ascontiguousarray(hj, dtype=np.int32)
        h = SVT(m, n, rows, cols, vals, tau=float(tau), delta=float(delta), precision=0, **params)
        st = h.iterate(T)
        if st.iter != T:
            h.close()
            raise RuntimeError(f"the run stopped after {st.iter} of {T} iterations (converged or maxit)")
        x = h.sample(hi, hj)
        ctx.h, ctx.T, ctx.ckpt, ctx.hi, ctx.hj, ctx.frozen = h, int(T), int(ckpt), hi, hj, bool(frozen_basis)
        ctx.a_dtype, ctx.dev = a.dtype, dev
        return x if dev else torch.from_numpy(x)

    @staticmethod
    def backward(ctx, gx):
        h = ctx.h
        g = gx.detach().to(torch.float64).contiguous() if ctx.dev else gx.detach().to("cpu", torch.float64).numpy()
        dtau, ddelta, da = h.grad(ctx.T, ctx.ckpt, ctx.hi, ctx.hj, g, frozen_basis=ctx.frozen)
        h.close()
        need = ctx.needs_input_grad
        ga = None
        if need[0]:
            ga = (da if ctx.dev else torch.from_numpy(da)).to(ctx.a_dtype)
        gt = torch.tensor(dtau, dtype=torch.float64) if need[1] else None
        gd = torch.tensor(ddelta, dtype=torch.float64) if need[2] else None
        return (ga, gt, gd, None, None, None, None, None, None, None, None, None, None)


def svt_heldout(a, tau, delta, m, n, rows, cols, hi, hj, T, ckpt=0, frozen_basis=False, **params):
    """X_T on (hi, hj) after T iterations; differentiable in a (observed values), tau and delta.
    params go to svt_init (seed, t0, dt, k0, ...); maxit is raised to at least T."""
    params = dict(params)
    params["maxit"] = max(int(params.get("maxit", 0)), int(T))
    params["tol"] = params.get("tol", 0.0)
    return SVTHeldOut.apply(a, tau, delta, int(m), int(n), rows, cols, hi, hj, int(T), int(ckpt), params,
                            bool(frozen_basis))
