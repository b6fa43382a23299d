"""Targets given as the first M rows of the sources (y and x the same
device pointer, M < N): the exec projects those rows once, in both roles.
Sums and all three adjoints must equal, bit for bit, those of the same
targets passed as a separate copy (the same arithmetic on the same values),
on every path; the sorted path keeps the targets in rows of their own.
Against the Fourier oracle O3 the prefix sums meet the parity bar (checked
once, on the fused path)."""
import numpy as np
import pytest

import oracle as O
from helpers import to_dev, err_scale, DEFAULT_T
from workloads.directions import directions

pytestmark = pytest.mark.gpu

PATHS = {
    # name: (kernel, d, plan keywords)
    "fused": ("gauss", 5, {}),
    "stored": ("gauss", 5, dict(materialize=True)),
    "tile_gemm": ("energy", 100, {}),
    "sorted": ("energy", 5, dict(sorting=True)),
}


@pytest.mark.parametrize("path", list(PATHS))
def test_prefix_targets_equal_copied_targets(path):
    import paper_2410_01316_amd as F
    import torch
    kernel, d, kw = PATHS[path]
    N, M, P = 1000, 300, 40
    rng = np.random.default_rng(len(path) + d)
    x = rng.standard_normal((N, d))
    w = rng.standard_normal(N)
    v = rng.standard_normal(M)
    R = 2.05 * float(np.linalg.norm(x, axis=1).max())
    xi = directions("orth" if d > 50 else "distance", d, P, 3)
    plan = F.Plan(xi, kernel=kernel, n_ft=128 if kernel == "gauss" else 1024, scale=1.0, R=R,
                  T=DEFAULT_T[kernel], grad=True, n_max=N, m_max=N, **kw)
    print(path, plan.info()["fused"], flush=True)
    xd, wd, vd = to_dev(x, w, v)
    s1 = plan(xd, wd, xd[:M]).clone()
    g1 = plan.grad(vd, want_x=True)
    plan.check()
    s2 = plan(xd, wd, xd[:M].clone()).clone()
    g2 = plan.grad(vd, want_x=True)
    plan.check()
    torch.cuda.synchronize()
    assert torch.equal(s1, s2)
    for a, b in zip(g1, g2):
        assert torch.equal(a, b)
    if path == "fused":
        f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
        tau = O.rescale_tau(kernel, R, 1.0, DEFAULT_T[kernel])
        ref = O.kernel_sum_fourier(kernel, f32(x), f32(x[:M]), f32(w), f32(xi), 1.0, 128, tau)
        s_abs = O.kernel_sum_direct(kernel, f32(x), f32(x[:M]), np.abs(f32(w)), 1.0)
        e = err_scale(s1.cpu().numpy(), ref, s_abs)     # signed weights: relative to sum |w| K
        print("prefix fused vs O3: err_scale %.2e" % e)
        assert e < 1e-4
    plan.close()


def test_prefix_targets_longer_than_sources_rejected():
    """y == x with M > N is an argument error, found before any GPU work."""
    import ctypes
    import paper_2410_01316_amd as F
    from paper_2410_01316_amd import _lib as L
    d, N = 3, 100
    xi = directions("distance", d, 8, 1)
    plan = F.Plan(xi, kernel="gauss", n_ft=128, scale=1.0, R=10.0, n_max=2 * N, m_max=2 * N)
    x, w = to_dev(np.zeros((2 * N, d)), np.ones(2 * N))
    out = to_dev(np.zeros(2 * N))[0]
    st = L.load().fastsum_exec(plan._h, ctypes.c_void_p(x.data_ptr()), N,
                               ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(x.data_ptr()), N + 1,
                               ctypes.c_void_p(out.data_ptr()), None)
    assert st == L.EINVAL
    plan.close()
