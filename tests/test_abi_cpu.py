"""The C-ABI library loads, exports every declared symbol, and rejects bad arguments on the host (no GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1704_05528_amd as svt
from paper_1704_05528_amd import _capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "svt.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("svt_", "r4svd_"))))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ["svt_init", "r4svd_step", "svt_iterate", "svt_grad"]:
        assert required in names
    assert sorted(_capi.EXPORTS) == names


def test_library_exports_every_declared_symbol():
    L = svt.load()
    for name in _declared_functions():
        assert hasattr(L, name), name
        assert C.cast(getattr(L, name), C.c_void_p).value


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of svt_params and svt_step_stats against the header as a C compiler lays
    it out: size and the offset of every field (gcc on include/svt.h)."""
    import os
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "svt.h"', "int main(void) {"]
    for cname, py in (("svt_params", _capi.Params), ("svt_step_stats", _capi.StepStats)):
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'printf("{cname}.{field} %zu\\n", offsetof({cname}, {field}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", inc, str(src), "-o", str(exe)], check=True)
    out = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                              text=True).stdout.split("\n") if line)
    for cname, py in (("svt_params", _capi.Params), ("svt_step_stats", _capi.StepStats)):
        assert int(out[cname]) == C.sizeof(py), cname
        for field, _ in py._fields_:
            assert int(out[f"{cname}.{field}"]) == getattr(py, field).offset, (cname, field)


def test_default_params():
    p = svt.default_params()
    assert p.tol == 1e-4 and p.beta == 0.95 and p.dt == 10 and p.maxit == 500
    assert p.k0 == -1 and p.eps_thr0 < 0 and p.precision == svt.SVT_FP64 and p.t0 == 0
    assert p.mode == svt.SVT_MODE_R4SVD and p.recycle_extra == -1 and p.oversample == 10 and p.mae_tol == 0.0


def _init(m, n, rows, cols, vals, vals_dtype=_capi.SVT_DTYPE_F64, ptr_is_device=0, **kw):
    params = svt.default_params(**kw)
    h = C.c_void_p()
    r = np.ascontiguousarray(rows, dtype=np.int32)
    c = np.ascontiguousarray(cols, dtype=np.int32)
    v = np.ascontiguousarray(vals, dtype=np.float32 if vals_dtype == _capi.SVT_DTYPE_F32 else np.float64)
    L = svt.load()
    st = L.svt_init(C.byref(h), m, n, r.size, r.ctypes.data, c.ctypes.data, v.ctypes.data, vals_dtype, ptr_is_device,
                    C.byref(params), None)
    return st, h, L.svt_last_error(None).decode()


GOOD = dict(tau=1.0, delta=1.0)


@pytest.mark.parametrize("case,args,kw", [
    ("m zero", (0, 3, [0], [0], [1.0]), GOOD),
    ("row out of range", (3, 3, [0, 3], [0, 1], [1.0, 2.0]), GOOD),
    ("negative col", (3, 3, [0, 1], [0, -1], [1.0, 2.0]), GOOD),
    ("duplicate", (3, 3, [1, 1], [2, 2], [1.0, 2.0]), GOOD),
    ("nan value", (3, 3, [0, 1], [0, 1], [1.0, float("nan")]), GOOD),
    ("tau", (3, 3, [0], [0], [1.0]), dict(tau=0.0, delta=1.0)),
    ("delta", (3, 3, [0], [0], [1.0]), dict(tau=1.0, delta=-2.0)),
    ("beta", (3, 3, [0], [0], [1.0]), dict(tau=1.0, delta=1.0, beta=1.0)),
    ("eta", (3, 3, [0], [0], [1.0]), dict(tau=1.0, delta=1.0, eta=1.0)),
    ("npow", (3, 3, [0], [0], [1.0]), dict(tau=1.0, delta=1.0, npow=-1)),
    ("vals_dtype", (3, 3, [0], [0], [1.0]), dict(tau=1.0, delta=1.0, vals_dtype=7)),
    ("ptr_is_device", (3, 3, [0], [0], [1.0]), dict(tau=1.0, delta=1.0, ptr_is_device=2)),
    ("nan float32 value", (3, 3, [0, 1], [0, 1], [1.0, float("nan")]),
     dict(tau=1.0, delta=1.0, vals_dtype=_capi.SVT_DTYPE_F32)),
    ("float32 duplicate", (3, 3, [1, 1], [2, 2], [1.0, 2.0]), dict(tau=1.0, delta=1.0, vals_dtype=_capi.SVT_DTYPE_F32)),
    ("precision", (3, 3, [0], [0], [1.0]), dict(tau=1.0, delta=1.0, precision=3)),
    ("bf16 truncated recycling", (3, 3, [0], [0], [1.0]),
     dict(tau=1.0, delta=1.0, precision=_capi.SVT_BF16, recycle_extra=2)),
])
def test_init_rejects_bad_arguments_on_host(case, args, kw):
    st, h, msg = _init(*args, **kw)
    assert st == svt.SVTError(-1, "").status == _capi.SVT_E_INVALID_ARG, case
    assert not h.value
    assert msg


def test_null_handles_are_rejected():
    L = svt.load()
    assert L.svt_iterate(None, 1, None) == _capi.SVT_E_INVALID_ARG
    assert L.r4svd_step(None, None) == _capi.SVT_E_INVALID_ARG
    assert L.svt_grad(None, 1, 1, 0, None, None, None, 0, None, None, None) == _capi.SVT_E_INVALID_ARG
    assert L.svt_factors(None, 0, None, None, None, None, 0) == _capi.SVT_E_INVALID_ARG
    assert L.svt_sample(None, 0, None, None, None, 1) == _capi.SVT_E_INVALID_ARG
    assert L.svt_history(None, 0, 0, None, None) == _capi.SVT_E_INVALID_ARG
    L.svt_destroy(None)
