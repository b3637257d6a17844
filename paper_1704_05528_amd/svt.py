"""Python face of the C-ABI: the same calls as include/svt.h, numpy in and out.

    h = svt_init(m, n, rows, cols, vals, tau=..., delta=..., seed=...)
    stats = svt_iterate(h, 100)
    k, s, U, V = h.factors()

Inputs may also be torch tensors on the GPU (int32 indices, float64 or float32 values): they are
then handed to the library as device pointers, and sample(), grad() and factors(device=True)
answer with GPU tensors written on the handle's stream.  Only argument marshalling happens here;
every step of the iteration runs in libsvt.so on the GPU that is current when the handle is created.
"""
import ctypes as C
import math

import numpy as np

from ._capi import (SVTError, StepStats, check, default_params, load, SVT_E_INVALID_ARG, SVT_DTYPE_F32,
                    SVT_DTYPE_F64, SVT_GRAD_DEVICE_POINTERS, SVT_GRAD_FROZEN_BASIS)

_i32p, _f64p = C.POINTER(C.c_int32), C.POINTER(C.c_double)


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_i32p)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_f64p)


def _is_device(x):
    """True for a torch tensor in GPU memory (torch is imported by load() already)."""
    return type(x).__module__.startswith("torch") and getattr(x, "is_cuda", False)


def _dev(t, dtypes, name):
    """Device pointer of a contiguous GPU tensor of one of the given torch dtypes."""
    if not _is_device(t):
        raise SVTError(SVT_E_INVALID_ARG, f"{name}: expected a GPU tensor like the other device arguments")
    if t.dtype not in dtypes:
        raise SVTError(SVT_E_INVALID_ARG, f"{name}: dtype {t.dtype} is not one of {dtypes}")
    if not t.is_contiguous():
        raise SVTError(SVT_E_INVALID_ARG, f"{name}: the tensor must be contiguous")
    return t.data_ptr()


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(int(stream.cuda_stream))


class SVT:
    """One matrix-completion problem on the GPU (an svt_handle)."""

    def __init__(self, m, n, rows, cols, vals, stream=None, **params):
        L = load()
        self.m, self.n = int(m), int(n)
        if _is_device(vals):
            import torch
            rp = _dev(rows, (torch.int32,), "rows")
            cp = _dev(cols, (torch.int32,), "cols")
            vp = _dev(vals, (torch.float64, torch.float32), "vals")
            sizes = (rows.numel(), cols.numel(), vals.numel())
            dtype, on_dev = (SVT_DTYPE_F64 if vals.dtype == torch.float64 else SVT_DTYPE_F32), 1
            if stream is not None:  # the library reads them on its stream
                torch.cuda.current_stream().synchronize()
        else:
            rows, rp = _i32(rows)
            cols, cp = _i32(cols)
            vals, vp = _f64(vals)
            sizes = (rows.size, cols.size, vals.size)
            dtype, on_dev = SVT_DTYPE_F64, 0
        if not (sizes[0] == sizes[1] == sizes[2]):
            raise SVTError(SVT_E_INVALID_ARG, "rows, cols and vals differ in length")
        self.nnz = int(sizes[0])
        self.params = default_params(**params)
        h = C.c_void_p()
        check(L.svt_init(C.byref(h), self.m, self.n, self.nnz, rp, cp, vp, dtype, on_dev, C.byref(self.params),
                         _stream_handle(stream)), None)
        self._h = h
        self._stream = stream  # the library works on this stream until close(): keep it alive

    def close(self):
        if getattr(self, "_h", None):
            load().svt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- Alg. 3 / Alg. 4 ------------------------------------------------------------------------
    def r4svd_step(self):
        st = StepStats()
        check(load().r4svd_step(self._h, C.byref(st)), self._h)
        return st

    def iterate(self, max_steps=1):
        st = StepStats()
        check(load().svt_iterate(self._h, int(max_steps), C.byref(st)), self._h)
        return st

    def history(self, first=0, count=None):
        """Reports of the iterations run by iterate() on this handle, oldest first."""
        L = load()
        total = C.c_int64()
        check(L.svt_history(self._h, 0, 0, None, C.byref(total)), self._h)
        n = max(0, total.value - int(first)) if count is None else int(count)
        if n <= 0:
            return []
        arr = (StepStats * n)()
        check(L.svt_history(self._h, int(first), n, arr, None), self._h)
        return list(arr[:max(0, min(n, total.value - int(first)))])

    # -- outputs --------------------------------------------------------------------------------
    def factors(self, kcap=None, device=False):
        """(k, s, U, V) of the last X; device=True: GPU tensors on the current device."""
        L = load()
        k = C.c_int32()
        check(L.svt_factors(self._h, 0, C.byref(k), None, None, None, 0), self._h)
        kc = k.value if kcap is None else int(kcap)
        if device:
            import torch
            s, U, V = (torch.zeros(sh, dtype=torch.float64, device="cuda") for sh in (kc, (self.m, kc), (self.n, kc)))
            ptrs = [t.data_ptr() for t in (s, U, V)]
        else:
            s, U, V = np.zeros(kc), np.zeros((self.m, kc)), np.zeros((self.n, kc))
            ptrs = [t.ctypes.data for t in (s, U, V)]
        if kc > 0:
            self._order_after_torch(device)
            check(L.svt_factors(self._h, kc, C.byref(k), *ptrs, int(device)), self._h)
            if device:
                self._order_torch_after()
        return k.value, s, U, V

    def sample(self, qi, qj):
        """X of the last iteration on (qi, qj): numpy in, numpy out; GPU int32 tensors in, a GPU
        float64 tensor out (an index outside m x n gives NaN there)."""
        if _is_device(qi):
            import torch
            ip = _dev(qi, (torch.int32,), "qi")
            jp = _dev(qj, (torch.int32,), "qj")
            if qi.numel() != qj.numel():
                raise SVTError(SVT_E_INVALID_ARG, "qi and qj differ in length")
            out = torch.empty(qi.numel(), dtype=torch.float64, device=qi.device)
            self._order_after_torch(True)
            check(load().svt_sample(self._h, qi.numel(), ip, jp, out.data_ptr(), 1), self._h)
            self._order_torch_after()
            return out
        qi, ip = _i32(qi)
        qj, jp = _i32(qj)
        out = np.zeros(qi.size)
        check(load().svt_sample(self._h, qi.size, ip, jp, out.ctypes.data, 0), self._h)
        return out

    def _order_after_torch(self, device):
        """Device arguments written by torch on its current stream are complete before the library
        reads them on the handle's stream (torch's allocations and fills are asynchronous)."""
        if device and self._stream is not None:
            import torch
            torch.cuda.current_stream().synchronize()

    def _order_torch_after(self):
        """torch's current stream waits for what the library enqueued on the handle's stream."""
        if self._stream is None:
            return  # the legacy default stream orders itself with every blocking stream
        import torch
        if isinstance(self._stream, torch.cuda.Stream):
            torch.cuda.current_stream().wait_stream(self._stream)
        else:
            torch.cuda.synchronize()

    def mae(self, qi, qj, ref):
        """Mean |ref - X| over the entries (qi, qj) (the MAE of Eq. 15 on those entries)."""
        qi, ip = _i32(qi)
        qj, jp = _i32(qj)
        ref, rp = _f64(ref)
        out = C.c_double()
        check(load().svt_mae(self._h, qi.size, ip, jp, rp, C.byref(out)), self._h)
        return out.value

    def get_state(self):
        L = load()
        r = C.c_int32()
        it = C.c_int32()
        thr, emin = C.c_double(), C.c_double()
        y = np.zeros(self.nnz)
        check(L.svt_get_state(self._h, y.ctypes.data_as(_f64p), None, 0, C.byref(r), C.byref(thr), C.byref(emin),
                              C.byref(it)), self._h)
        Q = np.zeros((self.m, max(r.value, 1)))
        if r.value > 0:
            check(L.svt_get_state(self._h, None, Q.ctypes.data_as(_f64p), r.value, None, None, None, None), self._h)
        return dict(y=y, Q=Q[:, : r.value], r=r.value, eps_thr=thr.value, eps_min=emin.value, iter=it.value)

    def set_state(self, y, Q=None, eps_thr=math.nan, eps_min=math.inf, iter=0):
        y, yp = _f64(y)
        if Q is None or Q.size == 0:
            r, qp = 0, None
        else:
            Q, qp = _f64(Q)
            r = Q.shape[1]
        check(load().svt_set_state(self._h, yp, qp, r, float(eps_thr), float(eps_min), int(iter)), self._h)

    def checkpoint(self):
        """bytes of svt_checkpoint (restart point with the decision log)"""
        L = load()
        size = C.c_int64()
        check(L.svt_checkpoint(self._h, None, 0, C.byref(size)), self._h)
        buf = C.create_string_buffer(size.value)
        check(L.svt_checkpoint(self._h, buf, size.value, C.byref(size)), self._h)
        return buf.raw[: size.value]

    def restore(self, blob):
        check(load().svt_restore(self._h, bytes(blob), len(blob)), self._h)

    def set_replay(self, blocks, annealed):
        b, bp = _i32(blocks)
        a, ap = _i32(annealed)
        check(load().svt_set_replay(self._h, bp, ap, int(b.size)), self._h)

    def profile(self, enable=True, phases=None):
        """Start (reset) or stop the per-phase device timers; `phases` limits them to the named
        phases (names from PHASES), which keeps the event markers out of the other phases."""
        if phases is None or not enable:
            check(load().svt_profile(self._h, 1 if enable else 0), self._h)
            return
        from ._capi import PHASES
        mask = 0
        for ph in phases:
            mask |= 1 << PHASES.index(ph)
        check(load().svt_profile_phases(self._h, mask), self._h)

    def profile_read(self):
        """{phase: dict(ms, bytes, flops, launches)} accumulated since profile(True)."""
        from ._capi import PHASES
        nph = len(PHASES)
        ms, by, fl = np.zeros(nph), np.zeros(nph), np.zeros(nph)
        ln = np.zeros(nph, dtype=np.int64)
        check(load().svt_profile_read(self._h, ms.ctypes.data_as(_f64p), by.ctypes.data_as(_f64p),
                                      fl.ctypes.data_as(_f64p), ln.ctypes.data_as(C.POINTER(C.c_int64))), self._h)
        return {ph: dict(ms=float(ms[i]), bytes=float(by[i]), flops=float(fl[i]), launches=int(ln[i]))
                for i, ph in enumerate(PHASES)}

    def time_phase(self, phase, reps=50):
        """(ms per launch, algorithmic bytes, flops) of `reps` back-to-back launches of a single-kernel
        phase ("spmm_t", "gram", "sddmm" or "densify") on the last iteration's operands."""
        from ._capi import PHASES
        ms, by, fl = C.c_double(), C.c_double(), C.c_double()
        check(load().svt_time_phase(self._h, PHASES.index(phase), int(reps), C.byref(ms), C.byref(by), C.byref(fl)),
              self._h)
        return ms.value, by.value, fl.value

    def grad(self, T, ckpt, hi, hj, gx_h, frozen_basis=False):
        """dL/dtau, dL/ddelta, dL/da through T unrolled iterations (exact, or with frozen bases).
        GPU tensors for hi, hj (int32) and gx_h (float64) give da as a GPU tensor."""
        flags = SVT_GRAD_FROZEN_BASIS if frozen_basis else 0
        dtau, ddelta = C.c_double(), C.c_double()
        if _is_device(gx_h):
            import torch
            ip = _dev(hi, (torch.int32,), "hi")
            jp = _dev(hj, (torch.int32,), "hj")
            gp = _dev(gx_h, (torch.float64,), "gx_h")
            if not (hi.numel() == hj.numel() == gx_h.numel()):
                raise SVTError(SVT_E_INVALID_ARG, "hi, hj and gx_h differ in length")
            nh = hi.numel()
            da = torch.empty(self.nnz, dtype=torch.float64, device=gx_h.device)
            dp = da.data_ptr()
            flags |= SVT_GRAD_DEVICE_POINTERS
            self._order_after_torch(True)
        else:
            hi, ip = _i32(hi)
            hj, jp = _i32(hj)
            g, gp = _f64(gx_h)
            nh = hi.size
            da = np.zeros(self.nnz)
            dp = da.ctypes.data
        check(load().svt_grad(self._h, int(T), int(ckpt), nh, ip, jp, gp, flags, C.byref(dtau), C.byref(ddelta), dp),
              self._h)
        return dtau.value, ddelta.value, da


# Same names as the C-ABI -------------------------------------------------------------------------
def svt_init(m, n, rows, cols, vals, stream=None, **params):
    return SVT(m, n, rows, cols, vals, stream=stream, **params)


def r4svd_step(h):
    return h.r4svd_step()


def svt_iterate(h, max_steps=1):
    return h.iterate(max_steps)


def svt_grad(h, T, ckpt, hi, hj, gx_h, frozen_basis=False):
    return h.grad(T, ckpt, hi, hj, gx_h, frozen_basis=frozen_basis)
