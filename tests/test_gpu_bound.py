"""The bound of App. J, eq. radius_xy, on the GPU: R >= max ||x|| + max ||y||.

Every point inside R on its own is not enough: with max ||x|| = max ||y|| =
0.8 R the projected differences reach 1.6 T, past the half period where the
periodic rescaled kernel equals the true one (for the energy kernel the
triangle wave wraps).  Each path (fused split, stored FP32 GEMM, tile GEMM
in FP32 and BF16, sorted sums, both batched forms) must report such an exec
through the range flag, and report nothing for a following exec inside the
bound (the slots are cleared by the check)."""
import numpy as np
import pytest

from helpers import to_dev

pytestmark = pytest.mark.gpu


def _sphere(n, d, radius, rng):
    """n points with norm exactly `radius` (up to float32 rounding)."""
    a = rng.standard_normal((n, d))
    return a / np.linalg.norm(a, axis=1, keepdims=True) * radius


def test_bound_matches_host_norms():
    import paper_2410_01316_amd as F
    rng = np.random.default_rng(0)
    for d, N, M in [(1, 5, 3), (3, 1000, 777), (50, 4097, 65), (784, 300, 2000), (3072, 70, 9)]:
        x = rng.standard_normal((N, d)) * 3.0
        y = rng.standard_normal((M, d)) + 1.0
        xd, yd = to_dev(x, y)
        x32 = x.astype(np.float32).astype(np.float64)
        y32 = y.astype(np.float32).astype(np.float64)
        ref = np.linalg.norm(x32, axis=1).max() + np.linalg.norm(y32, axis=1).max()
        assert F.bound(xd, yd) == pytest.approx(ref, rel=1e-6), d
        assert F.bound(xd) == pytest.approx(2 * np.linalg.norm(x32, axis=1).max(), rel=1e-6)


def test_bound_rejects_non_finite():
    import paper_2410_01316_amd as F
    from paper_2410_01316_amd import _lib as L
    x = to_dev(np.ones((10, 4)))[0]
    x[7, 2] = float("nan")
    with pytest.raises(F.FastSumError) as e:
        F.bound(x)
    assert e.value.status == L.ERANGE


PATHS = {
    # name: (kernel, d, plan keywords, expected fused flag)
    "fused": ("gauss", 3, {}, 1),
    "stored_fp32": ("gauss", 3, dict(materialize=True), 0),
    "tile_gemm_fp32": ("gauss", 100, {}, 0),
    "tile_gemm_bf16": ("energy", 100, dict(proj="bf16"), 0),
    "sorted": ("energy", 5, dict(sorting=True), 0),
}


@pytest.mark.parametrize("path", list(PATHS))
def test_sum_bound_violation_is_flagged(path):
    import paper_2410_01316_amd as F
    from paper_2410_01316_amd import _lib as L
    from workloads import directions
    kernel, d, kw, fused = PATHS[path]
    rng = np.random.default_rng(len(path))
    R, N, M, P = 2.0, 900, 700, 24
    xi = directions("orth" if d > 50 else "distance", d, P, 5)
    plan = F.Plan(xi, kernel=kernel, n_ft=128 if kernel == "gauss" else 1024, scale=1.0, R=R,
                  n_max=N, m_max=M, **kw)
    assert plan.info()["fused"] == fused
    w = to_dev(rng.standard_normal(N))[0]
    print(path, flush=True)
    # each point inside R, their norms adding to 1.6 R
    x, y = to_dev(_sphere(N, d, 0.8 * R, rng), _sphere(M, d, 0.8 * R, rng))
    plan(x, w, y)
    with pytest.raises(F.FastSumError) as e:
        plan.check()
    assert e.value.status == L.ERANGE
    # inside the bound: 0.8 R + 0.15 R
    y_in = to_dev(_sphere(M, d, 0.15 * R, rng))[0]
    plan(x, w, y_in)
    plan.check()
    # targets = sources: 2 * 0.6 R > R, then 2 * 0.45 R <= R
    xs = to_dev(_sphere(M, d, 0.6 * R, rng))[0]
    plan(xs, w[:M].contiguous(), xs)
    with pytest.raises(F.FastSumError):
        plan.check()
    xs = to_dev(_sphere(M, d, 0.45 * R, rng))[0]
    plan(xs, w[:M].contiguous(), xs)
    plan.check()
    plan.close()


@pytest.mark.parametrize("materialize", [False, True], ids=["fused", "stored"])
def test_batch_sum_bound_violation_is_flagged(materialize):
    import paper_2410_01316_amd as F
    from paper_2410_01316_amd import _lib as L
    from workloads import directions
    rng = np.random.default_rng(3)
    P, R = 32, 3.0
    sizes = [(3, 1500, 900), (10, 800, 1200), (50, 600, 400)]
    descs = [dict(xi=directions("distance", d, P, 11 + d), n_ft=128, scale=1.5, R=R, n_max=N,
                  m_max=M) for d, N, M in sizes]
    b = F.Batch(descs, kernel="gauss", materialize=materialize)
    ws = [to_dev(rng.standard_normal(N))[0] for _, N, _ in sizes]
    inside = [to_dev(_sphere(N, d, 0.5 * R, rng), _sphere(M, d, 0.45 * R, rng))
              for d, N, M in sizes]
    xs = [p[0] for p in inside]
    ys = [p[1] for p in inside]
    b(xs, ws, ys)
    b.check()
    # problem 1 alone breaks the sum bound (each point inside R)
    ys_bad = list(ys)
    ys_bad[1] = to_dev(_sphere(sizes[1][2], sizes[1][0], 0.8 * R, rng))[0]
    xs_bad = list(xs)
    xs_bad[1] = to_dev(_sphere(sizes[1][1], sizes[1][0], 0.8 * R, rng))[0]
    b(xs_bad, ws, ys_bad)
    with pytest.raises(F.FastSumError) as e:
        b.check()
    assert e.value.status == L.ERANGE
    # replaying the first inputs again is clean (slots cleared by the check)
    b(xs, ws, ys)
    b(xs, ws, ys)
    b.check()
    b.close()


@pytest.mark.parametrize("path", list(PATHS))
def test_prefix_targets_bound(path):
    """Targets passed as the first M rows of the sources (y == x, M < N): the
    bound takes the targets' own largest norm, not the sources' twice."""
    import paper_2410_01316_amd as F
    from paper_2410_01316_amd import _lib as L
    from workloads import directions
    kernel, d, kw, fused = PATHS[path]
    rng = np.random.default_rng(7 + len(path))
    R, N, M, P = 2.0, 900, 300, 24
    xi = directions("orth" if d > 50 else "distance", d, P, 5)
    plan = F.Plan(xi, kernel=kernel, n_ft=128 if kernel == "gauss" else 1024, scale=1.0, R=R,
                  n_max=N, m_max=N, **kw)
    w = to_dev(rng.standard_normal(N))[0]
    print(path, flush=True)
    # targets at 0.3 R, the other sources at 0.6 R: 0.9 R <= R
    x = to_dev(np.concatenate([_sphere(M, d, 0.3 * R, rng), _sphere(N - M, d, 0.6 * R, rng)]))[0]
    plan(x, w, x[:M])
    plan.check()
    # targets at 0.45 R: 1.05 R > R
    x = to_dev(np.concatenate([_sphere(M, d, 0.45 * R, rng), _sphere(N - M, d, 0.6 * R, rng)]))[0]
    plan(x, w, x[:M])
    with pytest.raises(F.FastSumError) as e:
        plan.check()
    assert e.value.status == L.ERANGE
    plan.close()
