"""The allocation-free distance-QMC entry point (fastsum_distance_qmc_noalloc,
workspace in a static device array) against the allocating one
(fastsum_distance_qmc), both through the C ABI: the same kernels in the same
order, so the designs must agree bit for bit.  Two calls in a row, the second
on a smaller problem (the array keeps the first call's contents), and a
request beyond the array's capacity, which must be refused before any
launch."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _start(P, d, seed):
    x = np.random.default_rng(seed).standard_normal((P, d))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return x.astype(np.float32)


def _call(name, x0, iters, lr):
    import torch
    from paper_2410_01316_amd import _lib as L
    t = torch.from_numpy(np.ascontiguousarray(x0)).cuda()
    stream = torch.cuda.current_stream()
    fn = getattr(L.load(), name)
    st = fn(x0.shape[1], x0.shape[0], iters, lr, ctypes.c_void_p(t.data_ptr()),
            ctypes.c_void_p(stream.cuda_stream))
    L.check(st, name)
    stream.synchronize()          # the allocation-free call only enqueues
    return t.cpu().numpy()


def test_noalloc_matches_allocating_entry_point():
    cases = [(1500, 50, 30), (200, 7, 40)]          # second call smaller in P and d
    for P, d, iters in cases:
        x0 = _start(P, d, P + d)
        lr = 0.05 * P ** (-1.0 / (d - 1))
        print(f"noalloc P={P} d={d} iters={iters}", flush=True)
        a = _call("fastsum_distance_qmc_noalloc", x0, iters, lr)
        b = _call("fastsum_distance_qmc", x0, iters, lr)
        assert np.array_equal(a, b), np.abs(a - b).max()
        assert np.abs(np.linalg.norm(a, axis=1) - 1.0).max() < 1e-5
        assert not np.array_equal(a, x0)


def test_noalloc_refuses_requests_beyond_its_array():
    import torch
    from paper_2410_01316_amd import _lib as L
    lib = L.load()
    t = torch.zeros((4096, 64), dtype=torch.float32, device="cuda")
    st = lib.fastsum_distance_qmc_noalloc(64, 4096, 5, 0.01, ctypes.c_void_p(t.data_ptr()),
                                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == L.EINVAL
    torch.cuda.synchronize()
    assert not t.any()                  # nothing was launched
