"""Python face of the C-ABI: the same calls as include/svt.h, numpy in and out.

    h = svt_init(m, n, rows, cols, vals, tau=..., delta=..., seed=...)
    stats = svt_iterate(h, 100)
    k, s, U, V = h.factors()

Only argument marshalling happens here; every step of the iteration runs in
libsvt.so on the GPU that is current when the handle is created.
"""
import ctypes as C
import math

import numpy as np

from ._capi import SVTError, StepStats, check, default_params, load, SVT_E_INVALID_ARG

_i32p, _f64p = C.POINTER(C.c_int32), C.POINTER(C.c_double)


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_i32p)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_f64p)


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
        rows, rp = _i32(rows)
        cols, cp = _i32(cols)
        vals, vp = _f64(vals)
        if not (rows.size == cols.size == vals.size):
            raise SVTError(SVT_E_INVALID_ARG, "rows, cols and vals differ in length")
        self.nnz = int(rows.size)
        self.params = default_params(**params)
        h = C.c_void_p()
        check(L.svt_init(C.byref(h), self.m, self.n, self.nnz, rp, cp, vp, C.byref(self.params),
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
    def factors(self, kcap=None):
        L = load()
        k = C.c_int32()
        check(L.svt_factors(self._h, 0, C.byref(k), None, None, None), self._h)
        kc = k.value if kcap is None else int(kcap)
        s = np.zeros(kc)
        U = np.zeros((self.m, kc))
        V = np.zeros((self.n, kc))
        if kc > 0:
            check(L.svt_factors(self._h, kc, C.byref(k), s.ctypes.data_as(_f64p), U.ctypes.data_as(_f64p),
                                V.ctypes.data_as(_f64p)), self._h)
        return k.value, s, U, V

    def sample(self, qi, qj):
        qi, ip = _i32(qi)
        qj, jp = _i32(qj)
        out = np.zeros(qi.size)
        check(load().svt_sample(self._h, qi.size, ip, jp, out.ctypes.data_as(_f64p)), self._h)
        return out

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
        """dL/dtau, dL/ddelta, dL/da through T unrolled iterations (exact, or with frozen bases)."""
        from ._capi import SVT_GRAD_FROZEN_BASIS
        hi, ip = _i32(hi)
        hj, jp = _i32(hj)
        g, gp = _f64(gx_h)
        dtau, ddelta = C.c_double(), C.c_double()
        da = np.zeros(self.nnz)
        flags = SVT_GRAD_FROZEN_BASIS if frozen_basis else 0
        check(load().svt_grad(self._h, int(T), int(ckpt), hi.size, ip, jp, gp, flags, C.byref(dtau),
                              C.byref(ddelta), da.ctypes.data_as(_f64p)), self._h)
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
