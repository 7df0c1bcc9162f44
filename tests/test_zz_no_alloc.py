"""The no-allocation g2 entry point (xs_g2_rings_noalloc) through the C ABI against
xs_g2_rings on the same inputs: bit for bit, on two calls in a row (the second with
fewer frames, pixels and lags, so it runs on buffers the first call left behind), and
its refusal of a request larger than its fixed array."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2204_13241_amd import _lib, inputs

pytestmark = pytest.mark.gpu


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _g2(fn, I, q, edges, n_tau):
    lib = _lib.load()
    e = np.ascontiguousarray(edges, dtype=np.float64)
    R = e.shape[0] - 1
    g2 = torch.full((R, n_tau), -7.0, dtype=torch.float64, device=I.device)
    cnt = torch.full((R,), -7, dtype=torch.int32, device=I.device)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = getattr(lib, fn)(_p(I), I.shape[0], I.shape[1], _p(q), e.ctypes.data_as(ctypes.c_void_p), R,
                          int(n_tau), _p(g2), _p(cnt), s)
    assert rc == 0, lib.xs_last_error().decode()
    torch.cuda.synchronize()
    return g2.cpu().numpy(), cnt.cpu().numpy()


def _case(F, n_det, q_max, rings, n_tau, seed):
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(seed)
    q = torch.as_tensor(inputs.ewald_detector(n_det, q_max), dtype=torch.float64, device="cuda:0")
    I = torch.empty((F, q.shape[0]), dtype=torch.float64, device="cuda:0").exponential_(1.0, generator=gen)
    I[:, :7] = 0.0                       # dark pixels are left out of the ring means
    return I, q, inputs.ring_edges(rings, q_max)


def test_noalloc_g2_equals_g2_on_two_calls_in_a_row():
    # the trajectory shape (200 frames, 256 x 256 pixels, 32 rings, 100 lags), then a
    # smaller ragged one: 37 frames, 100 x 100 pixels, 7 rings, 11 lags
    for F, n_det, q_max, rings, n_tau, seed in ((200, 256, 1.5, 32, 100, 1), (37, 100, 1.5, 7, 11, 2)):
        print("noalloc g2: F=%d det=%d rings=%d tau=%d" % (F, n_det, rings, n_tau), flush=True)
        I, q, edges = _case(F, n_det, q_max, rings, n_tau, seed)
        a, ca = _g2("xs_g2_rings", I, q, edges, n_tau)
        b, cb = _g2("xs_g2_rings_noalloc", I, q, edges, n_tau)
        assert np.array_equal(ca, cb) and ca.sum() > 0
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_noalloc_g2_refuses_more_than_its_fixed_array():
    lib = _lib.load()
    q = torch.zeros((1 << 20, 3), dtype=torch.float64, device="cuda:0")
    I = torch.zeros((16, 1 << 20), dtype=torch.float64, device="cuda:0")
    e = np.linspace(0.0, 1.0, 3)
    g2 = torch.empty((2, 16), dtype=torch.float64, device="cuda:0")
    # 2^20 pixels x 16 lags x 8 bytes = 128 MiB > 64 MiB
    rc = lib.xs_g2_rings_noalloc(_p(I), 16, 1 << 20, _p(q), e.ctypes.data_as(ctypes.c_void_p), 2, 16, _p(g2),
                                 None, None)
    assert rc == _lib.XS_EINVAL
    assert "fixed scratch" in lib.xs_last_error().decode()
