"""MMD gradient flow with momentum (App. MMD flows) on the GPU against the
same flow run with the FP64 oracle's sliced Fourier gradient."""
import numpy as np
import pytest

import oracle as O
from workloads import directions
from helpers import rel_l2, to_dev

pytestmark = pytest.mark.gpu


def _oracle_gradient(kernel, x, y, xi, scale, n_ft, T, R):
    N, M = x.shape[0], y.shape[0]
    z = np.vstack([x, y])
    w = np.concatenate([np.full(N, 1.0 / N**2), np.full(M, -1.0 / (M * N))])
    tau = O.rescale_tau(kernel, R, scale, T)
    return O.grad_y_fourier(kernel, z, x, w, xi, scale, n_ft, tau)


@pytest.mark.parametrize("kernel,scale", [("energy", 1.0), ("gauss", 2.0)])
def test_flow_matches_oracle_flow(kernel, scale):
    import torch
    import paper_2410_01316_amd as F
    rng = np.random.default_rng(21)
    N, M, d, P, n_ft = 300, 250, 5, 64, 256
    T = {"energy": 0.45, "gauss": 0.3}[kernel]
    y = rng.standard_normal((M, d)) * 0.5 + 2.0
    x0 = rng.standard_normal((N, d))
    xi = directions("distance", d, P, 5)
    step, steps = float(N), 6          # the gradient is O(1/N): move O(1) per step
    flow = F.MMDFlow(to_dev(y)[0], xi, N, kernel=kernel, n_ft=n_ft, scale=scale, T=T,
                     step=step, momentum=0.9)
    Rs = []
    xg = flow.run(to_dev(x0)[0], steps, callback=lambda k, x, R: Rs.append(R))
    xg = xg.cpu().numpy().astype(np.float64)
    # the same flow in FP64 with the oracle gradient at the R each step used
    x, v = x0.astype(np.float32).astype(np.float64), np.zeros_like(x0)
    yy = y.astype(np.float32).astype(np.float64)
    xio = xi.astype(np.float32).astype(np.float64)
    for R in Rs:
        v = _oracle_gradient(kernel, x, yy, xio, scale, n_ft, T, R) + 0.9 * v
        x = x - step * v
    e = rel_l2(xg - x0, x - x0)
    print(kernel, "displacement rel-L2 %.2e, plan rebuilds %d" % (e, flow.rebuilds))
    assert e < 1e-4
    flow.close()


def test_flow_decreases_mmd():
    """The energy MMD (direct FP64 sums) falls along the flow."""
    import paper_2410_01316_amd as F
    rng = np.random.default_rng(5)
    N, M, d = 400, 400, 3
    y = rng.standard_normal((M, d)) * 0.5 + 1.5
    x0 = rng.standard_normal((N, d))

    def mmd(x):
        def k(a, b):
            return -np.linalg.norm(a[:, None, :] - b[None, :, :], axis=2)
        return k(x, x).mean() / 2 - k(x, y).mean() + k(y, y).mean() / 2

    flow = F.MMDFlow(to_dev(y)[0], directions("distance", d, 128, 6), N, kernel="energy",
                     n_ft=512, step=float(N), momentum=0.9)
    xg = flow.run(to_dev(x0)[0], 30).cpu().numpy().astype(np.float64)
    print("MMD %.4e -> %.4e" % (mmd(x0), mmd(xg)))
    assert mmd(xg) < 0.5 * mmd(x0)
    flow.close()


def test_sorted_flow_matches_oracle_flow():
    """The flow with exact sorted 1-D sums and derivatives (the paper's
    method for the negative distance kernel) against the same flow run with
    the oracle's exact sliced gradient; every particle is a source and a
    target of the sum, so each step meets coincident projections, which both
    sides take with sign(0) = 0."""
    import paper_2410_01316_amd as F
    rng = np.random.default_rng(23)
    N, M, d, P = 300, 250, 5, 64
    y = rng.standard_normal((M, d)) * 0.5 + 2.0
    x0 = rng.standard_normal((N, d))
    xi = directions("distance", d, P, 5)
    step, steps = float(N), 6
    flow = F.MMDFlow(to_dev(y)[0], xi, N, kernel="energy", sorting=True, step=step,
                     momentum=0.9)
    xg = flow.run(to_dev(x0)[0], steps).cpu().numpy().astype(np.float64)
    x, v = x0.astype(np.float32).astype(np.float64), np.zeros_like(x0)
    yy = y.astype(np.float32).astype(np.float64)
    xio = xi.astype(np.float32).astype(np.float64)
    w = np.concatenate([np.full(N, 1.0 / N**2), np.full(M, -1.0 / (M * N))])
    for _ in range(steps):
        _, g, _ = O.grad_sliced_energy(np.vstack([x, yy]), x, w, np.ones(N), xio)
        v = g + 0.9 * v
        x = x - step * v
    e = rel_l2(xg - x0, x - x0)
    print("sorted flow displacement rel-L2 %.2e" % e)
    assert e < 1e-4
    flow.close()


@pytest.mark.parametrize("d,zmode", [(64, "rows"), (37, "rows"), (64, "none"), (37, "same")])
def test_flow_update_entry(d, zmode):
    """fastsum_flow_update against the momentum step written out in FP64
    (App. MMD flows): v' = g + m v, x' = x - tau v', z rows = x', and the
    largest ||x'||^2.  d = 64 takes the 16-byte path, d = 37 the scalar
    one; z separate, absent, or the particles themselves.  FP32 with one
    rounding per fused multiply-add: 1e-6 of the values' scale."""
    import ctypes
    import torch
    from paper_2410_01316_amd import _lib as L
    rng = np.random.default_rng(40 + d)
    N, m, tau = 1003, 0.9, 0.37
    g, v, x = (rng.standard_normal((N, d)).astype(np.float32) for _ in range(3))
    gd, vd, xd = (torch.from_numpy(a.copy()).cuda() for a in (g, v, x))
    zd = torch.full((N + 5, d), 7.0, device="cuda")
    n2 = torch.full((1,), -1.0, device="cuda")
    zp = {"rows": zd.data_ptr(), "none": None, "same": xd.data_ptr()}[zmode]
    st = L.load().fastsum_flow_update(N, d, m, tau, ctypes.c_void_p(gd.data_ptr()),
                                      ctypes.c_void_p(vd.data_ptr()),
                                      ctypes.c_void_p(xd.data_ptr()), ctypes.c_void_p(zp),
                                      ctypes.c_void_p(n2.data_ptr()),
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    L.check(st, "fastsum_flow_update")
    torch.cuda.synchronize()
    v1 = g.astype(np.float64) + m * v.astype(np.float64)
    x1 = x.astype(np.float64) - tau * v1
    assert np.abs(vd.cpu().numpy() - v1).max() < 1e-6 * np.abs(v1).max()
    assert np.abs(xd.cpu().numpy() - x1).max() < 1e-6 * np.abs(x1).max()
    zc = zd.cpu().numpy()
    if zmode == "rows":
        assert np.array_equal(zc[:N], xd.cpu().numpy())
    assert np.all(zc[N:] == 7.0) and (zmode == "rows" or np.all(zc == 7.0))
    ref = (x1 ** 2).sum(1).max()
    assert abs(float(n2.item()) - ref) < 1e-5 * ref
