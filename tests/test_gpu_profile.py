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


def test_time_phase_replays_without_changing_the_iteration(gpu_lib):
    """Back-to-back replays of the single-kernel phases report positive per-launch times and the
    phase timers' work counts, and leave the iteration bitwise unchanged."""
    a, b = _handle(gpu_lib, seed=23), _handle(gpu_lib, seed=23)
    a.iterate(3)
    b.iterate(3)
    b.profile(True, phases=["spmm_t", "gram", "sddmm", "densify"])
    b.iterate(1)
    counted = b.profile_read()
    b.profile(False)
    a.iterate(1)
    grew = b.history()[-1].blocks > 0  # W = Y^T Q ran on the basis before this iteration's growth
    for ph in ("spmm_t", "gram", "sddmm", "densify"):
        ms, by, fl = a.time_phase(ph, reps=5)
        assert ms > 0.0, ph
        if ph == "spmm_t" and grew:
            r = b.history()[-1].r
            assert fl == 2.0 * a.nnz * r
        elif ph == "densify":
            # the previous step's update wrote the dense copy: no refresh inside the step
            assert counted[ph]["launches"] == 0 and by > 0.0
        else:
            assert by == counted[ph]["bytes"] and fl == counted[ph]["flops"], ph
    sa, sb = a.iterate(2), b.iterate(2)
    assert (sa.r, sa.k, sa.blocks) == (sb.r, sb.k, sb.blocks)
    assert sa.rel_res == sb.rel_res and sa.normB == sb.normB
    assert (a.sample([0, 5, 7], [1, 2, 3]) == b.sample([0, 5, 7], [1, 2, 3])).all()


def test_time_phase_rejects_bad_requests(gpu_lib):
    from paper_1704_05528_amd import SVTError
    import paper_1704_05528_amd._capi as capi
    h = _handle(gpu_lib, seed=24)
    with pytest.raises(SVTError) as e:
        h.time_phase("gram")  # no iteration yet
    assert e.value.status == capi.SVT_E_STATE
    h.iterate(1)
    with pytest.raises(SVTError) as e:
        h.time_phase("eig")  # not a single-kernel phase
    assert e.value.status == capi.SVT_E_INVALID_ARG
    with pytest.raises(SVTError) as e:
        h.time_phase("gram", reps=0)
    assert e.value.status == capi.SVT_E_INVALID_ARG
    w = W.tiny_dense(120, 90, 4, 0.15, seed=25)  # sparse enough to have no dense copy of Y
    s = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, seed=25, maxit=5)
    s.iterate(1)
    with pytest.raises(SVTError) as e:
        s.time_phase("densify")
    assert e.value.status == capi.SVT_E_STATE
