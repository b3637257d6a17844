"""Instrumentation through the C-ABI: per-phase timers limited by a phase mask, and the
iteration history.  The phase counters are host-side bookkeeping around device events."""
import pytest

import svt_workloads as W

pytestmark = pytest.mark.gpu


def _handle(svt, seed=21, **kw):
    w = W.tiny_dense(120, 90, 4, 0.5, seed=seed)
    return svt.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, seed=seed, maxit=20, **kw)


def test_phase_mask_records_only_selected_phases(gpu_lib):
    h = _handle(gpu_lib)
    h.iterate(2)
    h.profile(True, phases=["gram", "sddmm"])
    h.iterate(3)
    p = h.profile_read()
    assert p["gram"]["launches"] == 3 and p["sddmm"]["launches"] == 3
    assert p["gram"]["ms"] > 0.0 and p["sddmm"]["ms"] > 0.0
    for ph in ("spmm_t", "grow", "eig", "factors", "reduce", "densify"):
        assert p[ph]["launches"] == 0 and p[ph]["ms"] == 0.0, ph
    h.profile(True)  # every phase, counters reset
    h.iterate(2)
    q = h.profile_read()
    assert q["gram"]["launches"] == 2 and q["eig"]["launches"] >= 2 and q["reduce"]["launches"] > 0
    h.profile(False)
    h.iterate(1)
    assert h.profile_read()["gram"]["launches"] == 2  # stopped: nothing more recorded
    assert len(h.history()) == 8


def test_phase_mask_rejects_unknown_bits(gpu_lib):
    import paper_1704_05528_amd._capi as capi
    h = _handle(gpu_lib, seed=22)
    L = capi.load()
    assert L.svt_profile_phases(h._h, 1 << 20) == capi.SVT_E_INVALID_ARG
    assert L.svt_profile_phases(h._h, 0) == capi.SVT_OK
