"""The host-side validation of the C-ABI under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): a host-only build of the library (no device code) with both sanitizers, loaded by a
child Python process with the clang ASan runtime preloaded, takes every invalid-argument path of
svt_init (host and float32 inputs, bad sizes, out-of-range and duplicate indices, non-finite values,
bad parameters), the NULL-handle paths of the other calls, and one valid svt_init, which on a
machine without a GPU fails at its first device allocation and must release what it built."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import ctypes as C, sys
import numpy as np
sys.path.insert(0, ROOT)
from paper_1704_05528_amd._capi import Params, SVT_DTYPE_F32, SVT_DTYPE_F64, SVT_E_INVALID_ARG
L = C.CDLL(LIB)
L.svt_default_params.argtypes = [C.POINTER(Params)]
L.svt_default_params.restype = None
L.svt_init.argtypes = [C.POINTER(C.c_void_p), C.c_int64, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                       C.c_int32, C.c_int32, C.POINTER(Params), C.c_void_p]
L.svt_last_error.argtypes = [C.c_void_p]
L.svt_last_error.restype = C.c_char_p
L.svt_destroy.argtypes = [C.c_void_p]
L.svt_destroy.restype = None

def init(m, n, rows, cols, vals, dtype=SVT_DTYPE_F64, dev=0, **kw):
    p = Params()
    L.svt_default_params(C.byref(p))
    p.tau, p.delta = 1.0, 1.0
    for k, v in kw.items():
        setattr(p, k, v)
    r = np.ascontiguousarray(rows, dtype=np.int32)
    c = np.ascontiguousarray(cols, dtype=np.int32)
    v = np.ascontiguousarray(vals, dtype=np.float32 if dtype == SVT_DTYPE_F32 else np.float64)
    h = C.c_void_p()
    st = L.svt_init(C.byref(h), m, n, r.size, r.ctypes.data, c.ctypes.data, v.ctypes.data, dtype, dev, C.byref(p), None)
    msg = L.svt_last_error(None)
    assert msg is not None
    if h.value:
        L.svt_destroy(h)
    return st

bad = [
    ((0, 3, [0], [0], [1.0]), {}),
    ((3, 3, [0, 3], [0, 1], [1.0, 2.0]), {}),
    ((3, 3, [0, 1], [0, -1], [1.0, 2.0]), {}),
    ((3, 3, [1, 1], [2, 2], [1.0, 2.0]), {}),
    ((3, 3, [0, 1], [0, 1], [1.0, float("nan")]), {}),
    ((3, 3, [0, 1], [0, 1], [1.0, float("inf")]), {"dtype": SVT_DTYPE_F32}),
    ((3, 3, [1, 1], [2, 2], [1.0, 2.0]), {"dtype": SVT_DTYPE_F32}),
    ((3, 3, [0], [0], [1.0]), {"dtype": 9}),
    ((3, 3, [0], [0], [1.0]), {"dev": 2}),
    ((3, 3, [0], [0], [1.0]), {"tau": 0.0}),
    ((3, 3, [0], [0], [1.0]), {"delta": -1.0}),
    ((3, 3, [0], [0], [1.0]), {"beta": 1.5}),
    ((3, 3, [0], [0], [1.0]), {"eta": 1.0}),
    ((3, 3, [0], [0], [1.0]), {"npow": -1}),
    ((3, 3, [0], [0], [1.0]), {"precision": 5}),
    ((3, 3, [0], [0], [1.0]), {"precision": 2, "recycle_extra": 1}),
    ((2, 2, [0, 0, 1, 1, 0], [0, 1, 0, 1, 1], [1.0, 2.0, 3.0, 4.0, 5.0]), {}),
]
for args, kw in bad:
    assert init(*args, **kw) == SVT_E_INVALID_ARG, (args, kw)
# NULL handles
for call, n in (("svt_iterate", 3), ("r4svd_step", 2), ("svt_history", 5), ("svt_factors", 7), ("svt_sample", 6),
                ("svt_grad", 11), ("svt_checkpoint", 4), ("svt_restore", 3), ("svt_mae", 6), ("svt_mae_device", 6)):
    f = getattr(L, call)
    f.restype = C.c_int
    assert f(*([None] * n)) == SVT_E_INVALID_ARG, call
L.svt_destroy(None)
# a valid problem: set-up runs on the host, then the first device allocation fails without a GPU
rng = np.random.default_rng(1)
idx = rng.choice(60 * 50, 900, replace=False)
st = init(60, 50, idx // 50, idx % 50, rng.standard_normal(900))  # SVT_E_HIP without a GPU, SVT_OK with one
print("sanitized host paths ok", st)
'''


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_host_validation_under_asan_and_ubsan(tmp_path):
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("the clang ASan runtime is not installed")
    from host_sanitized_build import build_host_sanitized
    lib = build_host_sanitized(str(tmp_path / "libsvt_host_sanitized.so"))
    syms = subprocess.run(["nm", "-D", "--undefined-only", lib], stdout=subprocess.PIPE).stdout.decode()
    assert "__asan_" in syms and "__ubsan_" in syms  # the host code really is instrumented
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    code = f"ROOT = {ROOT!r}\nLIB = {lib!r}\n" + CHILD
    r = subprocess.run([sys.executable, "-c", code], env=env, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                       timeout=600)
    err = r.stderr.decode(errors="replace")
    assert r.returncode == 0, err[-4000:]
    assert "AddressSanitizer" not in err and "runtime error:" not in err, err[-4000:]
    assert "sanitized host paths ok" in r.stdout.decode()
