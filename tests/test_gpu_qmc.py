"""Distance QMC directions built on the GPU (App. H) against the oracle's
FP64 projected Adam iteration from the same start."""
import ctypes

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


def _run(x0, iters, lr):
    import torch
    import paper_2410_01316_amd as F
    from paper_2410_01316_amd import _lib as L
    t = torch.from_numpy(np.ascontiguousarray(x0, dtype=np.float32)).cuda()
    st = L.load().fastsum_distance_qmc(x0.shape[1], x0.shape[0], iters, lr,
                                        ctypes.c_void_p(t.data_ptr()),
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    L.check(st, "fastsum_distance_qmc")
    return t.cpu().numpy().astype(np.float64)


def _start(P, d, seed):
    x = np.random.default_rng(seed).standard_normal((P, d))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return x.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("P,d", [(100, 3), (300, 20), (257, 50), (1, 4)])
def test_one_and_fifty_steps(P, d):
    """One step agrees to FP32 rounding; after 50 steps the FP32 iteration
    stays within 1e-3 of the FP64 one and reaches the same energy to 1e-6."""
    x0 = _start(P, d, P + d)
    lr = 0.05 * P ** (-1.0 / max(d - 1, 1))
    g1 = _run(x0, 1, lr)
    o1 = O.projected_adam(x0, 1, lr)
    assert np.abs(g1 - o1).max() < 2e-6
    g50 = _run(x0, 50, lr)
    o50 = O.projected_adam(x0, 50, lr)
    err = np.abs(g50 - o50).max()
    de = abs(O.distance_energy(g50) - O.distance_energy(o50)) / O.distance_energy(o50)
    print("P=%d d=%d: 1 step %.1e, 50 steps %.1e, energy %.1e" %
          (P, d, np.abs(g1 - o1).max(), err, de))
    assert err < 1e-3 and de < 1e-6
    assert np.allclose(np.linalg.norm(g50, axis=1), 1.0, atol=1e-6)


def test_orthonormal_minimiser():
    """P <= d ends at an orthonormal system (App. H)."""
    g = _run(_start(8, 8, 3), 2000, 0.05)
    assert np.abs(g @ g.T - np.eye(8)).max() < 1e-3


def test_api_and_errors():
    import paper_2410_01316_amd as F
    xi = F.distance_qmc(10, 64, iters=50, seed=4)
    assert xi.shape == (10, 64) and xi.dtype == np.float32
    assert np.allclose(np.linalg.norm(xi, axis=0), 1.0, atol=1e-6)
    with pytest.raises(F.FastSumError):
        F.distance_qmc(65, 10, iters=1)


def test_reproducible():
    x0 = _start(700, 20, 5)
    assert np.array_equal(_run(x0, 30, 0.02), _run(x0, 30, 0.02))


def test_register_widths():
    """d at the edges of the register-row widths (16, 32, 48, 64): the energy
    after 20 steps matches the FP64 iteration (Adam's normalised first steps
    turn FP32-level differences in a near-zero gradient component into a
    full step of either sign, so single coordinates are not compared), and
    for P = d the iteration ends orthonormal."""
    for d in (16, 17, 32, 33, 48, 49, 64):
        x0 = _start(130, d, d)
        lr = 0.05 * 130 ** (-1.0 / (d - 1))
        e_gpu = O.distance_energy(_run(x0, 20, lr))
        e_ref = O.distance_energy(O.projected_adam(x0, 20, lr))
        assert abs(e_gpu - e_ref) < 1e-6 * e_ref, d
        g = _run(_start(d, d, d + 1), 1500, 0.05)
        assert np.abs(g @ g.T - np.eye(d)).max() < 2e-3, d


@pytest.mark.parametrize("d", [33, 48])
def test_one_step_elementwise_48_wide_rows(d):
    """One step at d = 33 and 48 (the 48-wide register rows), element by
    element.  The first Adam step moves every coordinate by +-lr (m/sqrt(v)
    is the sign of the gradient), so a coordinate whose tangent gradient is
    at FP32 noise level may flip; the rows compared are those whose every
    coordinate's gradient is clear of that level, and they must agree to
    FP32 rounding."""
    P = 130
    x0 = _start(P, d, 1000 + d)
    lr = 0.05 * P ** (-1.0 / (d - 1))
    g = O.distance_energy_grad(x0)
    g -= (g * x0).sum(1, keepdims=True) * x0
    stable = np.abs(g).min(axis=1) > 1e-3 * np.abs(g).max()
    assert stable.sum() >= P // 2
    g1 = _run(x0, 1, lr)
    o1 = O.projected_adam(x0, 1, lr)
    err = np.abs(g1 - o1)[stable].max()
    print("d=%d: one step on %d of %d rows, max |gpu - oracle| %.1e" % (d, stable.sum(), P, err))
    assert err < 2e-6


def _haar(d, rng):
    q, r = np.linalg.qr(rng.standard_normal((d, d)))
    return q * np.sign(np.diag(r))


@pytest.mark.parametrize("P,d", [(1, 1), (257, 3), (100, 17), (3500, 50), (513, 64)])
def test_rotate_directions_matches_oracle(P, d):
    """fastsum_rotate_directions (App. E) against the oracle's FP64 rotation
    with the same FP32 matrix, element by element.  Rows and q rows are unit,
    so every output is a dot product with sum |q_ij x_j| <= 1: FP32 sums of
    d <= 64 terms stay within 64 * 2^-24 < 4e-6."""
    import torch
    from paper_2410_01316_amd import _lib as L
    rng = np.random.default_rng(900 + d)
    x0 = _start(P, d, 17 * d + P)
    q = _haar(d, rng).astype(np.float32)
    t = torch.from_numpy(x0.astype(np.float32)).cuda()
    qd = torch.from_numpy(q).cuda()
    st = L.load().fastsum_rotate_directions(d, P, ctypes.c_void_p(qd.data_ptr()),
                                             ctypes.c_void_p(t.data_ptr()),
                                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    L.check(st, "fastsum_rotate_directions")
    ref = O.rotate_directions(q.astype(np.float64), x0)
    assert np.abs(t.cpu().numpy().astype(np.float64) - ref).max() < 4e-6


def test_distance_qmc_rotation_is_the_library_rotation():
    """distance_qmc(rotate=True) is the unrotated design rotated by the Haar
    draw that follows the start in the seeded stream (App. E)."""
    import paper_2410_01316_amd as F
    d, P, seed = 12, 200, 5
    plain = F.distance_qmc(d, P, iters=20, seed=seed, rotate=False)
    rot = F.distance_qmc(d, P, iters=20, seed=seed, rotate=True)
    rng = np.random.default_rng(seed)
    rng.standard_normal((P, d))
    q = _haar(d, rng).astype(np.float32).astype(np.float64)
    ref = O.rotate_directions(q, plain.T.astype(np.float64)).T
    assert np.abs(rot - ref).max() < 4e-6
    assert np.allclose(np.linalg.norm(rot, axis=0), 1.0, atol=1e-6)
