"""The device-pointer forms of the boundary against the host-pointer forms of the same calls.

svt_init with device rows, cols and values (float64, or float32 widened on input), svt_factors
into device matrices, svt_sample on device queries, and svt_grad with SVT_GRAD_DEVICE_POINTERS all
run the same kernels on the same inputs as the host forms, so their results must agree bit for
bit; the host forms are held to the oracle by the other parity tests.  Device queries outside
m x n give NaN at their places and leave the others intact.
"""
import ctypes as C

import numpy as np
import pytest

import svt_workloads as W

pytestmark = pytest.mark.gpu


def _w(seed=3):
    return W.tiny_dense(90, 70, 3, 0.4, seed=seed)


def _dev(torch, x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda").contiguous()


def _queries(w, nq=500, seed=9):
    rng = np.random.default_rng(seed)
    return rng.integers(0, w.m, nq).astype(np.int32), rng.integers(0, w.n, nq).astype(np.int32)


@pytest.mark.parametrize("stream_kind", ["default", "own"])
def test_device_init_factors_and_sample_equal_the_host_forms(gpu_lib, stream_kind):
    import torch
    w = _w()
    kw = dict(tau=w.tau, delta=w.delta, seed=5, maxit=40, tol=0.0)
    stream = torch.cuda.Stream() if stream_kind == "own" else None
    hh = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, **kw)
    hd = gpu_lib.svt_init(w.m, w.n, _dev(torch, w.rows, torch.int32), _dev(torch, w.cols, torch.int32),
                          _dev(torch, w.a, torch.float64), stream=stream, **kw)
    sh, sd = hh.iterate(12), hd.iterate(12)
    assert (sh.iter, sh.k, sh.r) == (sd.iter, sd.k, sd.r)
    assert sh.rel_res == sd.rel_res
    qi, qj = _queries(w)
    xh = hh.sample(qi, qj)
    xd = hd.sample(_dev(torch, qi, torch.int32), _dev(torch, qj, torch.int32))
    assert xd.is_cuda and xd.dtype == torch.float64
    np.testing.assert_array_equal(xd.cpu().numpy(), xh)
    kh, s_h, U_h, V_h = hh.factors()
    kd, s_d, U_d, V_d = hd.factors(device=True)
    assert kh == kd > 0 and U_d.is_cuda
    np.testing.assert_array_equal(s_d.cpu().numpy(), s_h)
    np.testing.assert_array_equal(U_d.cpu().numpy(), U_h)
    np.testing.assert_array_equal(V_d.cpu().numpy(), V_h)
    # a wider kcap leaves the extra device columns as they were (zeros from torch)
    _, s2, U2, V2 = hd.factors(kcap=kh + 3, device=True)
    assert torch.count_nonzero(U2[:, kh:]).item() == 0 and torch.count_nonzero(s2[kh:]).item() == 0
    np.testing.assert_array_equal(U2[:, :kh].cpu().numpy(), U_h)
    hh.close()
    hd.close()


def test_float32_values_are_widened_on_input(gpu_lib):
    import torch
    w = _w(seed=4)
    a32 = w.a.astype(np.float32)
    kw = dict(tau=w.tau, delta=w.delta, seed=6, maxit=40, tol=0.0)
    hh = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, a32.astype(np.float64), **kw)
    hd = gpu_lib.svt_init(w.m, w.n, _dev(torch, w.rows, torch.int32), _dev(torch, w.cols, torch.int32),
                          _dev(torch, a32, torch.float32), **kw)
    hh.iterate(8)
    hd.iterate(8)
    qi, qj = _queries(w, seed=10)
    np.testing.assert_array_equal(hd.sample(qi, qj), hh.sample(qi, qj))
    hh.close()
    hd.close()


def test_device_init_rejects_what_the_host_form_rejects(gpu_lib):
    import torch
    w = _w()
    rows = w.rows.copy()
    rows[7] = w.m  # out of range
    with pytest.raises(gpu_lib.SVTError) as e:
        gpu_lib.svt_init(w.m, w.n, _dev(torch, rows, torch.int32), _dev(torch, w.cols, torch.int32),
                         _dev(torch, w.a, torch.float64), tau=w.tau, delta=w.delta)
    assert e.value.status == gpu_lib.SVT_E_INVALID_ARG
    with pytest.raises(gpu_lib.SVTError):  # index tensors must be int32
        gpu_lib.svt_init(w.m, w.n, _dev(torch, w.rows, torch.int64), _dev(torch, w.cols, torch.int32),
                         _dev(torch, w.a, torch.float64), tau=w.tau, delta=w.delta)


def test_device_sample_marks_out_of_range_queries_with_nan(gpu_lib):
    import torch
    w = _w()
    h = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, seed=5)
    h.iterate(5)
    qi, qj = _queries(w, nq=300, seed=11)
    ref = h.sample(qi, qj)
    bad = np.array([3, 50, 51, 299])
    qi2, qj2 = qi.copy(), qj.copy()
    qi2[bad[0]], qj2[bad[1]], qi2[bad[2]], qj2[bad[3]] = -1, w.n, w.m + 5, -7
    x = h.sample(_dev(torch, qi2, torch.int32), _dev(torch, qj2, torch.int32)).cpu().numpy()
    assert np.isnan(x[bad]).all()
    keep = np.setdiff1d(np.arange(qi.size), bad)
    np.testing.assert_array_equal(x[keep], ref[keep])
    with pytest.raises(gpu_lib.SVTError) as e:  # the host form refuses them
        h.sample(qi2, qj2)
    assert e.value.status == gpu_lib.SVT_E_INVALID_ARG
    # nq = 0 is a no-op in both forms
    assert h.sample(_dev(torch, qi[:0], torch.int32), _dev(torch, qj[:0], torch.int32)).numel() == 0
    h.close()


@pytest.mark.parametrize("frozen", [False, True])
def test_device_grad_equals_the_host_form(gpu_lib, frozen):
    import torch
    w = _w(seed=31)
    T = 8
    kw = dict(tau=w.tau, delta=w.delta, seed=31, maxit=T + 2, tol=0.0)
    rng = np.random.default_rng(12)
    free = np.setdiff1d(np.arange(w.m * w.n), w.rows.astype(np.int64) * w.n + w.cols)
    hsel = np.sort(rng.choice(free, 60, replace=False))
    hi, hj = (hsel // w.n).astype(np.int32), (hsel % w.n).astype(np.int32)
    g = rng.standard_normal(hsel.size)
    h = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, **kw)
    h.iterate(T)
    th, dh, ah = h.grad(T, 0, hi, hj, g, frozen_basis=frozen)
    td, dd, ad = h.grad(T, 0, _dev(torch, hi, torch.int32), _dev(torch, hj, torch.int32),
                        _dev(torch, g, torch.float64), frozen_basis=frozen)
    assert ad.is_cuda
    assert (td, dd) == (th, dh)
    np.testing.assert_array_equal(ad.cpu().numpy(), ah)
    h.close()


def test_autograd_on_gpu_tensors_equals_the_cpu_path(gpu_lib):
    import torch
    from paper_1704_05528_amd.autograd import svt_heldout
    w = _w(seed=31)
    T = 6
    rng = np.random.default_rng(13)
    free = np.setdiff1d(np.arange(w.m * w.n), w.rows.astype(np.int64) * w.n + w.cols)
    hsel = np.sort(rng.choice(free, 50, replace=False))
    hi, hj = hsel // w.n, hsel % w.n
    target = rng.standard_normal(hsel.size)
    out = []
    for device in ("cpu", "cuda"):
        a = torch.tensor(w.a, dtype=torch.float64, device=device, requires_grad=True)
        tau = torch.tensor(w.tau, dtype=torch.float64, requires_grad=True)
        delta = torch.tensor(w.delta, dtype=torch.float64, requires_grad=True)
        x = svt_heldout(a, tau, delta, w.m, w.n, w.rows, w.cols, hi, hj, T=T, seed=31)
        assert x.device.type == device
        loss = ((x - torch.as_tensor(target, device=device)) ** 2).sum()
        loss.backward()
        out.append((x.detach().cpu().numpy(), a.grad.cpu().numpy(), tau.grad.item(), delta.grad.item()))
    np.testing.assert_array_equal(out[1][0], out[0][0])
    np.testing.assert_array_equal(out[1][1], out[0][1])
    assert out[1][2:] == out[0][2:]


def test_c_abi_device_calls_directly(gpu_lib):
    """The raw C calls with device pointers: svt_sample enqueues and returns; svt_factors with
    out_is_device writes the device matrices."""
    import torch
    L = gpu_lib.load()
    w = _w()
    h = gpu_lib.svt_init(w.m, w.n, w.rows, w.cols, w.a, tau=w.tau, delta=w.delta, seed=5)
    h.iterate(4)
    qi, qj = _queries(w, nq=64, seed=14)
    dqi, dqj = _dev(torch, qi, torch.int32), _dev(torch, qj, torch.int32)
    out = torch.full((64,), -1.0, dtype=torch.float64, device="cuda")
    assert L.svt_sample(h._h, 64, dqi.data_ptr(), dqj.data_ptr(), out.data_ptr(), 1) == 0
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), h.sample(qi, qj))
    assert L.svt_sample(h._h, 64, dqi.data_ptr(), dqj.data_ptr(), out.data_ptr(), 3) == gpu_lib.SVT_E_INVALID_ARG
    k = C.c_int32()
    assert L.svt_factors(h._h, 0, C.byref(k), None, None, None, 0) == 0
    U = torch.zeros((w.m, k.value), dtype=torch.float64, device="cuda")
    assert L.svt_factors(h._h, k.value, C.byref(k), None, U.data_ptr(), None, 1) == 0
    torch.cuda.synchronize()
    np.testing.assert_array_equal(U.cpu().numpy(), h.factors()[2])
    assert L.svt_factors(h._h, k.value, C.byref(k), None, U.data_ptr(), None, 2) == gpu_lib.SVT_E_INVALID_ARG
    h.close()
