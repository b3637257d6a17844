"""Checkpoint and restore through the C-ABI: a handle restored from svt_checkpoint continues bit for
bit as the checkpointed handle does (step reports, Y, samples of X), in the FP64 and the mixed form
and with the projected SVD in full-decomposition mode; svt_grad works across a restore; a blob of
another problem is refused and leaves the handle as it was."""
import numpy as np
import pytest

import svt_workloads as W

pytestmark = pytest.mark.gpu


def _fields(st):
    return [getattr(st, f) for f, _ in st._fields_]


@pytest.mark.parametrize("case", ["fp64", "mixed", "wide_k"])
def test_restore_continues_bit_for_bit(gpu_lib, case):
    svt = gpu_lib
    if case == "wide_k":
        w = W.tiny_dense(300, 260, 200, 0.7, seed=92, tau=0.4 * np.sqrt(300 * 260))
        kw = dict(dt=40, seed=92)
    else:
        w = W.tiny_dense(130, 110, 4, 0.35, seed=33)
        kw = dict(dt=7, seed=33, precision=svt.SVT_MIXED if case == "mixed" else svt.SVT_FP64)
    h1 = svt.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, maxit=200, tol=0.0, **kw)
    h1.iterate(12)
    blob = h1.checkpoint()
    h1.iterate(10)
    ref_hist = [_fields(x) for x in h1.history()]
    ref_y = h1.get_state()["y"]
    ref_x = h1.sample(w.rows, w.cols)
    h2 = svt.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, maxit=200, tol=0.0, **kw)
    h2.restore(blob)
    h2.iterate(10)
    print(f"{case}: r={h2.history()[-1].r} k={h2.history()[-1].k}", flush=True)
    assert [_fields(x) for x in h2.history()] == ref_hist
    assert np.array_equal(h2.get_state()["y"], ref_y)
    assert np.array_equal(h2.sample(w.rows, w.cols), ref_x)


def test_grad_across_restore_and_bad_blobs(gpu_lib):
    svt = gpu_lib
    w = W.tiny_dense(90, 70, 3, 0.4, seed=31)
    kw = dict(seed=31, maxit=50, tol=0.0)
    h1 = svt.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, **kw)
    h1.iterate(8)
    blob = h1.checkpoint()
    rng = np.random.default_rng(5)
    hr = rng.integers(0, w.m, 30).astype(np.int32)
    hc = rng.integers(0, w.n, 30).astype(np.int32)
    g = rng.standard_normal(30)
    ref = h1.grad(8, 0, hr, hc, g)
    h2 = svt.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, **kw)
    h2.restore(blob)
    out = h2.grad(8, 0, hr, hc, g)
    assert out[0] == ref[0] and out[1] == ref[1] and np.array_equal(out[2], ref[2])
    # another problem's checkpoint is refused and leaves the handle unchanged
    w3 = W.tiny_dense(60, 50, 2, 0.5, seed=3)
    h3 = svt.svt_init(w3.m, w3.n, w3.rows, w3.cols, w3.a, tau=w3.tau, delta=w3.delta, seed=3)
    h3.iterate(2)
    before = h3.get_state()
    with pytest.raises(svt.SVTError) as e:
        h3.restore(blob)
    assert e.value.status == svt.SVT_E_INVALID_ARG
    with pytest.raises(svt.SVTError) as e:
        h3.restore(b"not a checkpoint at all")
    assert e.value.status == svt.SVT_E_INVALID_ARG
    after = h3.get_state()
    assert np.array_equal(before["y"], after["y"]) and before["iter"] == after["iter"]
