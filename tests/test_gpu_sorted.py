"""Exact sliced sums of the energy kernel by sorting (plans with sorting=True)
against the oracle's exact sliced sum (eq. (3) with f(t) = -c_d |t|, FP64).

With no Fourier series left, the only difference from the oracle is the
FP32 projection: each key carries an error of about 1e-7 tau |x|, so a term
c_d |x~ - y~| / tau is off by at most ~2e-7 c_d R, against terms of size
~|x - y| ~ R / 2 on average (c_d E|<xi, z>| = |z|).  Summed with aligned
signs that is ~4e-7 c_d relative to the unsigned sum s_abs (1.2e-6 at
d = 5, 1.4e-5 at d = 784); the bars below sit at those worst cases."""
import numpy as np
import pytest

import oracle as O
from workloads.configs import make_config
from workloads.directions import directions
from helpers import rel_l2, max_rel, err_scale, to_dev, oracle_inputs, DEFAULT_T

pytestmark = pytest.mark.gpu


def _bar(d):
    return 4e-7 * O.energy_cd(d) + 1e-6


def _plan(cfg, n_max=None, m_max=None, proj="fp32", xi=None, R=None):
    import paper_2410_01316_amd as F
    xi = cfg["xi"] if xi is None else xi
    return F.Plan(xi, kernel="energy", n_ft=cfg.get("n_ft") or 1024, R=R or cfg["R"],
                  T=DEFAULT_T["energy"], proj=proj, sorting=True,
                  n_max=n_max or cfg["x"].shape[0], m_max=m_max or cfg["y"].shape[0])


def _gpu(plan, cfg, same=False):
    x, y, w = to_dev(cfg["x"], cfg["y"], cfg["w"])
    if same:
        y = x
    s = plan(x, w, y).cpu().numpy().astype(np.float64)
    plan.check()
    return s


def _oracle(cfg, idx=None):
    x, y, w, xi = oracle_inputs(cfg)
    if idx is not None:
        y = y[idx]
    s2 = O.kernel_sum_sliced("energy", x, y, w, xi, 1.0)
    s_abs = O.kernel_sum_direct("energy", x, y, np.abs(w), 1.0)
    return s2, s_abs


def _points(N, M, d, seed, ties=0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((N, d))
    y = rng.standard_normal((M, d)) * 0.7 + 0.2
    if ties:
        # repeated sources, and targets that sit exactly on sources
        x[1:ties + 1] = x[0]
        y[:ties] = x[N - ties:N]
    w = rng.standard_normal(N)
    R = float(np.linalg.norm(x, axis=1).max() + np.linalg.norm(y, axis=1).max())
    return dict(x=x, y=y, w=w, R=R, kernel="energy", scale=1.0, n_ft=1024)


@pytest.mark.parametrize("N,M,d,P", [(1500, 1300, 5, 32), (9001, 3, 3, 17), (1, 1, 2, 1),
                                     (5, 700, 64, 40), (900, 1100, 65, 24)])
def test_sorted_matches_exact_sliced(N, M, d, P):
    """Ragged sizes (one point, one direction, a row past one 8192-entry
    chunk of the prefix-sum pass), d at both sides of the fused / stored
    projection boundary."""
    cfg = _points(N, M, d, seed=N + 7 * M + d)
    cfg["xi"] = directions("distance" if d > 1 else "orth", d, P, 5)
    plan = _plan(cfg)
    assert plan.info()["fused"] == 0
    s = _gpu(plan, cfg)
    plan.close()
    s2, s_abs = _oracle(cfg)
    e = err_scale(s, s2, s_abs)
    print("sorted N=%d M=%d d=%d P=%d: err_scale %.2e" % (N, M, d, P, e))
    assert e < _bar(d)


def test_sorted_ties_and_smaller_calls():
    """Equal keys (repeated sources, targets on sources) and a plan reused
    at smaller N and M, so stale keys from the first call sit in the padding
    of the second."""
    big = _points(3000, 2500, 4, seed=3, ties=40)
    big["xi"] = directions("distance", 4, 48, 6)
    small = _points(1100, 700, 4, seed=4, ties=25)
    small["xi"] = big["xi"]
    # one plan bound R >= max|x| + max|y| for both point sets
    big["R"] = small["R"] = max(big["R"], small["R"])
    plan = _plan(big)
    s_big = _gpu(plan, big)
    s_small = _gpu(plan, small)
    plan.close()
    for s, cfg in ((s_big, big), (s_small, small)):
        s2, s_abs = _oracle(cfg)
        e = err_scale(s, s2, s_abs)
        print("ties N=%d M=%d: err_scale %.2e" % (cfg["x"].shape[0], cfg["y"].shape[0], e))
        assert e < _bar(4)


def test_sorted_sources_equal_targets_d784():
    """The precision workload's shape (x = y, weights +-1/n, d = 784, tile
    GEMM projections), where s cancels: compared relative to s_abs."""
    cfg = make_config("precision", frac=0.005, P=64)
    plan = _plan(cfg)
    s = _gpu(plan, cfg, same=True)
    plan.close()
    s2, s_abs = _oracle(cfg)
    e = err_scale(s, s2, s_abs)
    print("sorted d784 x=y: err_scale %.2e" % e)
    assert e < _bar(784)


def test_sorted_agrees_with_fourier_and_projections():
    """Same plan data through the Fourier path: the difference is the
    Fourier error alone (App. J, a few 1e-5 of s_abs at N_ft = 1024); the
    stored projections read back equal those of a materialised plan."""
    import paper_2410_01316_amd as F
    cfg = make_config("mmd", kernel="energy", frac=0.005, P=64)
    plan = _plan(cfg)
    s = _gpu(plan, cfg)
    pf = F.Plan(cfg["xi"], kernel="energy", n_ft=1024, R=cfg["R"], T=DEFAULT_T["energy"],
                materialize=True, n_max=cfg["N"], m_max=cfg["M"])
    sf = _gpu(pf, cfg)
    for which in (0, 1):
        assert np.array_equal(plan.debug_read(which), pf.debug_read(which))
    with pytest.raises(F.FastSumError):
        plan.debug_read(2)
    plan.close()
    pf.close()
    s2, s_abs = _oracle(cfg)
    e_sort = err_scale(s, s2, s_abs)
    e_four = err_scale(sf, s2, s_abs)
    print("mmd energy: sorted %.2e, Fourier %.2e (err_scale vs exact sliced)" % (e_sort, e_four))
    assert e_sort < _bar(20) and e_four < 1e-4 and e_sort < e_four


def test_sorted_plan_errors():
    import paper_2410_01316_amd as F
    xi = directions("distance", 3, 8, 1)
    with pytest.raises(F.FastSumError):
        F.Plan(xi, kernel="gauss", n_ft=128, scale=1.0, R=4.0, sorting=True, n_max=10, m_max=10)
    with pytest.raises(F.FastSumError):
        F.Plan(xi, kernel="laplace", n_ft=1024, scale=1.0, R=4.0, sorting=True, grad=True,
               n_max=10, m_max=10)
    with pytest.raises(F.FastSumError):       # bucket counters beyond the LDS budget
        F.Plan(xi, kernel="energy", n_ft=1024, R=4.0, sorting=True, n_max=(1 << 24) + 1,
               m_max=10)
    plan = F.Plan(xi, kernel="energy", n_ft=1024, R=4.0, sorting=True, n_max=10, m_max=10)
    import torch
    x = torch.zeros((10, 3), device="cuda")
    x[0, 0] = 10.0          # outside the bound R
    w = torch.ones(10, device="cuda")
    plan(x, w, x)
    with pytest.raises(F.FastSumError):
        plan.check()
    with pytest.raises(F.FastSumError):
        plan(torch.zeros((11, 3), device="cuda"), torch.ones(11, device="cuda"), x)
    plan.close()


def test_sorted_precision_full_size():
    """d = 784, x = y = 2e5 image-like points, weights +-1/n: 64 of the 2000
    directions against the oracle on 24 sampled targets (the estimator is a
    mean over directions, so a subset is the same computation at full N),
    and all 2000 directions against the Fourier path on the same targets."""
    import paper_2410_01316_amd as F
    cfg = make_config("precision")
    rng = np.random.default_rng(12)
    idx = np.sort(rng.choice(cfg["M"], 24, replace=False))
    sub = dict(cfg, xi=cfg["xi"][:, :64])
    plan = _plan(sub)
    s64 = _gpu(plan, sub, same=True)
    plan.close()
    s2, s_abs = _oracle(sub, idx)
    e = err_scale(s64[idx], s2, s_abs)
    plan = _plan(cfg)
    s = _gpu(plan, cfg, same=True)
    plan.close()
    pf = F.Plan(cfg["xi"], kernel="energy", n_ft=1024, R=cfg["R"], T=DEFAULT_T["energy"],
                n_max=cfg["N"], m_max=cfg["M"])
    sf = _gpu(pf, cfg, same=True)
    pf.close()
    ef = err_scale(s[idx], sf[idx], s_abs)
    print("precision full size sorted: 64 dirs vs oracle %.2e; 2000 dirs vs Fourier %.2e"
          % (e, ef))
    assert e < _bar(784) and ef < 1e-4


def test_sorted_bf16_projection():
    """BF16 projections (inputs and directions rounded to 8 mantissa bits)
    with exact 1-D sums: the error is the projection's, as in the Fourier
    path's BF16 form (bar 2e-3 of s_abs)."""
    cfg = make_config("precision", frac=0.004, P=96)
    plan = _plan(cfg, proj="bf16")
    s = _gpu(plan, cfg, same=True)
    plan.close()
    s2, s_abs = _oracle(cfg)
    e = err_scale(s, s2, s_abs)
    print("sorted bf16 d784: err_scale %.2e" % e)
    assert e < 2e-3


def _grid_points(N, M, d, seed):
    """Points on a 1/8 grid in [-2, 2]^d: along the coordinate axes every
    projection is exact in FP32 and many of them coincide (ties)."""
    rng = np.random.default_rng(seed)
    x = rng.integers(-16, 17, size=(N, d)) / 8.0
    y = rng.integers(-16, 17, size=(M, d)) / 8.0
    y[: M // 4] = x[: M // 4]                    # targets on sources
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    return x, y, f32(rng.standard_normal(N)), f32(rng.standard_normal(M))


def _sorted_grads(x, y, w, v, xi, same=False):
    import paper_2410_01316_amd as F
    import torch
    R = float(np.linalg.norm(x, axis=1).max() + np.linalg.norm(y, axis=1).max()) + 0.5
    plan = F.Plan(xi, kernel="energy", n_ft=1024, R=R, T=DEFAULT_T["energy"], sorting=True,
                  grad=True, n_max=x.shape[0], m_max=y.shape[0])
    xd, yd, wd, vd = to_dev(x, y, w, v)
    if same:
        yd = xd
    s = plan(xd, wd, yd)
    gx, gy, gw = plan.grad(vd, want_x=True)
    torch.cuda.synchronize()
    plan.check()
    plan.close()
    f = lambda t: t.cpu().numpy().astype(np.float64)
    return f(s), f(gx), f(gy), f(gw)


@pytest.mark.parametrize("same", [False, True])
def test_sorted_gradients_exact_ties(same):
    """Axis directions and grid points: exact keys with many ties, so the
    adjoint must take sign(0) = 0 for every coincident pair (the symmetric
    difference quotient the oracle pins).  Bar 1e-5 rel-L2: the per-direction
    one-sided sums are combined in FP32."""
    N, M, d = 700, 500, 3
    x, y, w, v = _grid_points(N, M, d, seed=31)
    if same:
        y = x
        v = np.random.default_rng(32).standard_normal(N).astype(np.float32).astype(np.float64)
    xi = np.concatenate([np.eye(d), -np.eye(d)], axis=1)
    s, gx, gy, gw = _sorted_grads(x, y, w, v, xi, same)
    ox, oy, ow = O.grad_sliced_energy(x, y, w, v, xi)
    s2 = O.kernel_sum_sliced("energy", x, y, w, xi, 1.0)
    e = [rel_l2(s, s2), rel_l2(gx, ox), rel_l2(gy, oy), rel_l2(gw, ow)]
    print("sorted grads, ties (same=%s): s %.1e gx %.1e gy %.1e gw %.1e" % (same, *e))
    assert max(e) < 1e-5


@pytest.mark.parametrize("levels,d,same", [(2, 2, False), (2, 2, True), (17, 3, False)])
def test_sorted_gradients_runs_across_chunks(levels, d, same):
    """Equal keys in runs longer than the adjoint's 4096-entry chunks: with
    coordinates in {0, 1} each axis direction has two keys, so a run covers
    whole chunks and its values are written when it ends (entries of
    earlier chunks read back); with 17 levels in [-1, 1] runs of ~900
    entries straddle chunk boundaries.  same: one sorted copy of the points,
    each entry source and target."""
    N, M = 9000, 6000
    rng = np.random.default_rng(81 + levels + 2 * d + same)
    grid = np.linspace(0.0, 1.0, 2) if levels == 2 else np.linspace(-1.0, 1.0, levels)
    x = grid[rng.integers(0, levels, size=(N, d))]
    y = x.copy() if same else grid[rng.integers(0, levels, size=(M, d))]
    M = y.shape[0]
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    w = f32(rng.standard_normal(N))
    v = f32(rng.standard_normal(M))
    xi = np.concatenate([np.eye(d), -np.eye(d)], axis=1)
    s, gx, gy, gw = _sorted_grads(x, y, w, v, xi, same)
    ox, oy, ow = O.grad_sliced_energy(x, y, w, v, xi)
    e = [rel_l2(gx, ox), rel_l2(gy, oy), rel_l2(gw, ow)]
    print("sorted grads, long runs (levels %d, same=%s): gx %.1e gy %.1e gw %.1e"
          % (levels, same, *e))
    assert max(e) < 1e-5
    assert max_rel(gx, ox) < 1e-4 and max_rel(gy, oy) < 1e-4


def test_sorted_gradients_qmc_directions():
    """Distance-QMC directions at d = 5: the FP32 projections can order a
    source and a target differently from the FP64 oracle when they lie
    within ~1e-7 of each other (a few of 6e7 pairs), each flipping one sign
    in one direction's derivative, so the derivative bar is 2e-3 rel-L2;
    the transposed sum (grad_w) has no such jump and meets 1e-5."""
    N, M, d, P = 1500, 1300, 5, 32
    cfg = _points(N, M, d, seed=41)
    x, y, w = cfg["x"], cfg["y"], cfg["w"]
    v = np.random.default_rng(42).standard_normal(M).astype(np.float32).astype(np.float64)
    xi = directions("distance", d, P, 7)
    s, gx, gy, gw = _sorted_grads(x, y, w, v, xi)
    xo, yo, wo, xio = oracle_inputs(dict(x=x, y=y, w=w, xi=xi))
    ox, oy, ow = O.grad_sliced_energy(xo, yo, wo, v, xio)
    e = [rel_l2(gx, ox), rel_l2(gy, oy), rel_l2(gw, ow)]
    print("sorted grads, QMC: gx %.1e gy %.1e gw %.1e" % tuple(e))
    assert e[0] < 2e-3 and e[1] < 2e-3 and e[2] < 1e-5


@pytest.mark.parametrize("d,P", [(100, 40), (102, 72)])
def test_sorted_gradients_tile_gemm_backprojection(d, P):
    """Above the fused range the derivative matrices are back-projected on
    the split-f16 tile GEMM (rows scaled by a power of two, FP32-level
    products): d = 100 takes the 16-byte stores, d = 102 the element stores
    of the ragged row end; P is not a whole number of 32-column k-blocks.
    Bars as for the QMC case (FP32 key order at near-ties)."""
    N, M = 1500, 1300
    cfg = _points(N, M, d, seed=43 + d)
    x, y, w = cfg["x"], cfg["y"], cfg["w"]
    v = np.random.default_rng(44).standard_normal(M).astype(np.float32).astype(np.float64)
    xi = directions("orth", d, P, 9)
    s, gx, gy, gw = _sorted_grads(x, y, w, v, xi)
    xo, yo, wo, xio = oracle_inputs(dict(x=x, y=y, w=w, xi=xi))
    ox, oy, ow = O.grad_sliced_energy(xo, yo, wo, v, xio)
    e = [rel_l2(gx, ox), rel_l2(gy, oy), rel_l2(gw, ow)]
    print("sorted grads, d=%d P=%d: gx %.1e gy %.1e gw %.1e" % (d, P, *e))
    assert e[0] < 2e-3 and e[1] < 2e-3 and e[2] < 1e-5


def test_sorted_autograd_matches_plan_grad():
    import paper_2410_01316_amd as F
    import torch
    x, y, w, v = _grid_points(300, 200, 3, seed=51)
    xi = directions("distance", 3, 16, 8)
    R = float(np.linalg.norm(x, axis=1).max() + np.linalg.norm(y, axis=1).max()) + 0.5
    plan = F.Plan(xi, kernel="energy", n_ft=1024, R=R, sorting=True, grad=True,
                  n_max=300, m_max=200)
    xd, yd, wd, vd = to_dev(x, y, w, v)
    xa, ya, wa = (t.clone().requires_grad_(True) for t in (xd, yd, wd))
    s = F.FastSum.apply(plan, xa, ya, wa)
    (s * vd).sum().backward()
    plan(xd, wd, yd)
    gx, gy, gw = plan.grad(vd, want_x=True)
    for a, b in ((xa.grad, gx), (ya.grad, gy), (wa.grad, gw)):
        assert torch.equal(a, b)
    plan.close()


def test_sorted_gradient_subsets():
    """Requesting one adjoint alone computes only its pieces and gives the
    same values as requesting all three."""
    import paper_2410_01316_amd as F
    x, y, w, v = _grid_points(400, 300, 3, seed=61)
    xi = directions("distance", 3, 24, 9)
    R = float(np.linalg.norm(x, axis=1).max() + np.linalg.norm(y, axis=1).max()) + 0.5
    plan = F.Plan(xi, kernel="energy", n_ft=1024, R=R, sorting=True, grad=True,
                  n_max=400, m_max=300)
    xd, yd, wd, vd = to_dev(x, y, w, v)
    plan(xd, wd, yd)
    gx, gy, gw = (t.cpu().numpy() for t in plan.grad(vd, want_x=True))
    gy1, _ = plan.grad(vd, want_y=True, want_w=False)
    _, gw1 = plan.grad(vd, want_y=False, want_w=True)
    gx1, _, _ = plan.grad(vd, want_x=True, want_y=False, want_w=False)
    plan.close()
    assert np.array_equal(gy1.cpu().numpy(), gy)
    assert np.array_equal(gw1.cpu().numpy(), gw)
    assert np.array_equal(gx1.cpu().numpy(), gx)


def test_sorted_bitwise_reproducible():
    """The stable sorts and the fixed-order scans make repeated calls
    bitwise identical, gradients included."""
    import paper_2410_01316_amd as F
    x, y, w, v = _grid_points(2000, 1500, 3, seed=71)
    x = x + np.random.default_rng(72).standard_normal(x.shape) * 0.01
    xi = directions("distance", 3, 40, 10)
    R = float(np.linalg.norm(x, axis=1).max() + np.linalg.norm(y, axis=1).max()) + 0.5
    plan = F.Plan(xi, kernel="energy", n_ft=1024, R=R, sorting=True, grad=True,
                  n_max=2000, m_max=1500)
    xd, yd, wd, vd = to_dev(x, y, w, v)
    runs = []
    for _ in range(2):
        s = plan(xd, wd, yd).cpu().numpy()
        g = [t.cpu().numpy() for t in plan.grad(vd, want_x=True)]
        runs.append([s] + g)
    plan.close()
    for a, b in zip(*runs):
        assert np.array_equal(a, b)


def test_sorted_padding_keys_finite_in_reused_memory():
    """The padding between a row's sources and targets (N not a multiple of
    64) is sorted along with zero weight; a plan made in device memory that
    last held NaN must still give finite sums that match the oracle."""
    import paper_2410_01316_amd as F
    import torch
    N, M, d, P = 1001, 777, 4, 24
    junk = torch.full((64 << 20,), float("nan"), device="cuda")
    torch.cuda.synchronize()
    del junk
    torch.cuda.empty_cache()
    cfg = _points(N, M, d, seed=91)
    cfg["xi"] = directions("distance", d, P, 3)
    plan = _plan(cfg)
    s = _gpu(plan, cfg)
    plan.close()
    s2, s_abs = _oracle(cfg)
    assert np.all(np.isfinite(s))
    assert err_scale(s, s2, s_abs) < _bar(d)


@pytest.mark.parametrize("N,M", [(1, 1), (1, 4097), (4097, 1), (4096, 4096)])
def test_sorted_gradients_degenerate_sizes(N, M):
    """One source or one target, one bucket exactly full (4096 targets) and
    one entry past it: the adjoint's staging and placement at their edges,
    against the oracle's exact sliced gradients."""
    rng = np.random.default_rng(N + 3 * M)
    d, P = 3, 8
    x = rng.standard_normal((N, d))
    y = rng.standard_normal((M, d))
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    x, y = f32(x), f32(y)
    w = f32(rng.standard_normal(N))
    v = f32(rng.standard_normal(M))
    xi = directions("distance", d, P, 6)
    s, gx, gy, gw = _sorted_grads(x, y, w, v, xi)
    xio = xi.astype(np.float32).astype(np.float64)
    ox, oy, ow = O.grad_sliced_energy(x, y, w, v, xio)
    e = [rel_l2(gx, ox), rel_l2(gy, oy), rel_l2(gw, ow)]
    print("sorted grads N=%d M=%d: gx %.1e gy %.1e gw %.1e" % (N, M, *e))
    assert e[0] < 2e-3 and e[1] < 2e-3 and e[2] < 1e-5
