"""GPU parity of the fused path (projections computed inside the spreading
and gathering kernels, d <= 64) against the path that stores projections,
and against the FP64 oracle, over the launch shapes and edge sizes.

The two paths differ only in FP32 rounding order: the fused spread sums the
coordinates of each projection in another order (16-byte operand groups),
keeps per-slice cell sums in FP32 instead of FP64, and sums four directions
in FP32 before the FP64 sum over directions.  Measured relative to
s_abs = sum_n |w_n| |F(||x_n - y_m||)| (err_scale) that is ~1e-7: bar 1e-6.

Against the oracle O3 the weights are signed, so s cancels (in d = 50 all
pair distances are close to the median and s is a small difference of
nearly equal sums): the window error is measured relative to
s_abs = sum_n |w_n| F(||x_n - y_m||) (err_scale), W = 4 bar 2e-5."""
import numpy as np
import pytest

import oracle as O
from workloads import make_config, directions
from workloads.points import median_rule_sigma
from helpers import rel_l2, err_scale, gpu_plan, to_dev, oracle_inputs, DEFAULT_T

pytestmark = pytest.mark.gpu


def _o3(cfg):
    x, y, w, xi = oracle_inputs(cfg)
    tau = O.rescale_tau(cfg["kernel"], cfg["R"], cfg["scale"], DEFAULT_T[cfg["kernel"]])
    return O.kernel_sum_fourier(cfg["kernel"], x, y, w, xi, cfg["scale"], cfg["n_ft"], tau)


def _err3(cfg, s):
    x, y, w, xi = oracle_inputs(cfg)
    return err_scale(s, _o3(cfg), _sabs(cfg))


def _sabs(cfg):
    x, y, w, xi = oracle_inputs(cfg)
    return np.abs(O.kernel_sum_direct(cfg["kernel"], x, y, np.abs(w), cfg["scale"]))


def _both(cfg, **kw):
    x, y, w = to_dev(cfg["x"], cfg["y"], cfg["w"])
    out = []
    for mat in (False, True):
        plan = gpu_plan(cfg, materialize=mat, **kw)
        assert plan.info()["fused"] == (0 if mat else 1)
        out.append(plan(x, w, y).cpu().numpy())
        plan.check()
    return out


def _ragged(d, N, M, P, seed, n_ft=128, kernel="gauss", scale=None):
    # scale None: the median rule (Sec. 4.1), which keeps the sliced spectrum
    # well inside the N_ft band in any dimension
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((N, d))
    y = rng.standard_normal((M, d)) * 0.8
    w = rng.standard_normal(N)
    R = float(np.linalg.norm(x, axis=1).max() + np.linalg.norm(y, axis=1).max())
    if scale is None:
        scale = 1.3 if d < 10 else median_rule_sigma(x, y, np.random.default_rng(0))
    return dict(x=x, y=y, w=w, xi=directions("distance", d, P, seed), kernel=kernel,
                scale=scale, n_ft=n_ft, R=R)


@pytest.mark.parametrize("d,N,M,P", [(1, 5000, 3001, 16), (3, 4097, 515, 17), (7, 777, 1333, 37),
                                     (50, 9000, 1025, 70), (64, 8191, 600, 33)])
def test_fused_equals_stored_projections(d, N, M, P):
    cfg = _ragged(d, N, M, P, seed=d)
    s_f, s_m = _both(cfg)
    e3 = _err3(cfg, s_f)
    em = err_scale(s_f, s_m, _sabs(cfg))
    print("d=%d fused-stored %.2e fused-O3 %.2e (err_scale)" % (d, em, e3))
    assert em < 1e-6
    assert e3 < 2e-5


def test_fused_scale_workload_sample():
    # d = 50 mixture with signed weights, full grid (n_ft = 1024)
    cfg = make_config("scale", frac=0.05, P=48)
    s_f, s_m = _both(cfg)
    assert err_scale(s_f, s_m, _sabs(cfg)) < 1e-6
    assert rel_l2(s_f, _o3(cfg)) < 1e-4         # mixture data: little cancellation


@pytest.mark.parametrize("chunk_len,dir_range", [(4096, 16), (8192, 32), (4096 * 3, 48), (0, 0),
                                               (3008, 16), (5008, 32)])
def test_fused_launch_shapes(chunk_len, dir_range):
    """Chunk lengths that are not whole fixed-point slices (3008, 5008 = 16 k)
    put slice boundaries inside chunks: each piece is scaled by its own
    slice's exponent."""
    cfg = _ragged(20, 20000, 3000, 100, seed=9, n_ft=256)
    x, y, w = to_dev(cfg["x"], cfg["y"], cfg["w"])
    plan = gpu_plan(cfg)
    ref = plan(x, w, y).cpu().numpy()
    plan.set_launch(chunk_len, dir_range)
    s = plan(x, w, y).cpu().numpy()
    info = plan.info()
    if chunk_len:
        assert info["last_spread_chunks"] == -(-20000 // chunk_len)
    if dir_range:
        assert info["last_gather_groups"] == -(-100 // dir_range)
    assert err_scale(s, ref, _sabs(cfg)) < 1e-6
    assert _err3(cfg, s) < 2e-5


def test_fused_plan_stores_no_projections():
    import paper_2410_01316_amd as F
    cfg = make_config("tiny", frac=0.1)
    plan = gpu_plan(cfg)
    x, y, w = to_dev(cfg["x"], cfg["y"], cfg["w"])
    plan(x, w, y)
    with pytest.raises(F.FastSumError) as e:
        plan.debug_read(0)
    assert e.value.status == 6            # ESTATE
    assert plan.debug_read(2).shape[0] == cfg["xi"].shape[1]


def test_fused_energy_and_laplace():
    for kernel, n_ft in [("energy", 256), ("laplace", 512)]:
        cfg = _ragged(10, 6000, 2000, 40, seed=11, n_ft=n_ft, kernel=kernel)
        s_f, s_m = _both(cfg)
        assert err_scale(s_f, s_m, _sabs(cfg)) < 1e-6
        assert _err3(cfg, s_f) < 2e-5


@pytest.mark.parametrize("d,N,M,P,W,same", [(3, 5001, 2077, 37, 4, False),
                                            (20, 3000, 1300, 64, 6, False),
                                            (64, 1500, 1500, 21, 8, True)])
def test_fused_wide_grids_equal_stored(d, N, M, P, W, same):
    """Energy kernel at N_ft = 1024, T = 0.45: grids of ~1856 cells, past the
    narrow fused kernels (16 nr > 16384 cells): the wide spread (64 cell
    accumulators per thread) and the one-buffer gathers (fewer target
    batches; W = 8 the fewest) against the stored plan on the same inputs,
    the sum and all three adjoints, element by element (ragged tiles and
    direction groups, sources equal to targets); and the fused sum against
    O3 on sampled targets."""
    rng = np.random.default_rng(d * 11 + P)
    x = rng.standard_normal((N, d)) * 0.7
    y = x if same else rng.standard_normal((M, d)) * 0.7
    M = y.shape[0]
    w = rng.standard_normal(N)
    from workloads.configs import bound_R
    cfg = dict(x=x, y=y, w=w, xi=directions("distance", d, P, d), kernel="energy", scale=1.0,
               n_ft=1024, R=bound_R(x, y))
    v = rng.standard_normal(M)
    res = {}
    for mat in (False, True):
        plan = gpu_plan(cfg, grad=True, materialize=mat, window_w=W)
        info = plan.info()
        assert info["fused"] == (0 if mat else 1)
        assert 16 * info["grid_nr"] > 16384
        xd, wd = to_dev(x, w)
        yd = xd if same else to_dev(y)[0]
        s = plan(xd, wd, yd)
        gx, gy, gw = plan.grad(to_dev(v)[0], want_x=True)
        plan.check()
        res[mat] = [g.cpu().numpy().astype(np.float64) for g in (s, gy, gw, gx)]
    es = err_scale(res[False][0], res[True][0], _sabs(cfg))
    ey, ew, ex = [rel_l2(a, b) for a, b in zip(res[False][1:], res[True][1:])]
    print(f"wide d={d} W={W} nr={info['grid_nr']}: s {es:.2e} grad_y {ey:.2e} grad_w {ew:.2e} "
          f"grad_x {ex:.2e}")
    assert es < 1e-6 and ey < 5e-5 and ew < 5e-5 and ex < 5e-5
    idx = np.sort(np.random.default_rng(5).choice(M, 48, replace=False))
    sub = dict(cfg, y=y[idx])
    e3 = err_scale(res[False][0][idx], _o3(sub), _sabs(sub))
    print(f"wide d={d} W={W}: fused vs O3 on 48 targets {e3:.2e}")
    assert e3 < 2e-5


@pytest.mark.parametrize("d,N,M,P,same", [(3, 3001, 2077, 37, False), (20, 2500, 1300, 64, False),
                                          (50, 1800, 1800, 45, True), (64, 1000, 517, 16, False)])
def test_fused_adjoint_equals_stored(d, N, M, P, same):
    """grad_y (derivative gather back-projected on the matrix cores) and
    grad_w (the transposed fused sum) of a fused GRAD plan against the stored
    plan's on the same inputs, element by element; ragged target tiles,
    ragged direction groups, sources equal to targets."""
    import torch
    rng = np.random.default_rng(d * 7 + P)
    x = rng.standard_normal((N, d)) * 0.7
    y = x if same else rng.standard_normal((M, d)) * 0.7
    M = y.shape[0]
    w = rng.standard_normal(N)
    xi = rng.standard_normal((d, P))
    xi /= np.linalg.norm(xi, axis=0)
    from workloads.configs import bound_R
    cfg = dict(x=x, y=y, w=w, xi=xi, kernel="gauss", scale=1.5 * np.sqrt(d), n_ft=256,
               R=bound_R(x, y))
    v = rng.standard_normal(M)
    res = {}
    for mat in (False, True):
        plan = gpu_plan(cfg, grad=True, materialize=mat)
        assert plan.info()["fused"] == (0 if mat else 1)
        xd, wd = to_dev(x, w)
        yd = xd if same else to_dev(y)[0]
        plan(xd, wd, yd)
        gx, gy, gw = plan.grad(to_dev(v)[0], want_x=True)
        plan.check()
        res[mat] = [g.cpu().numpy().astype(np.float64) for g in (gy, gw, gx)]
    ey, ew, ex = [rel_l2(a, b) for a, b in zip(res[False], res[True])]
    print(f"d={d} N={N} M={M} P={P} same={same} grad_y {ey:.2e} grad_w {ew:.2e} grad_x {ex:.2e}")
    assert ey < 2e-5 and ew < 2e-5 and ex < 2e-5


@pytest.mark.parametrize("chunk_len", [0, 3008])
def test_weights_spanning_decades_within_slices(chunk_len):
    """Spreading rounds each term to 2^-19 of its slice's largest |w|: weights
    log-uniform over six decades, in random order inside every 4096-source
    slice (signed), against the exact Fourier sum (err_scale) and the stored
    path; with chunk boundaries inside slices too."""
    rng = np.random.default_rng(23)
    cfg = _ragged(10, 12000, 2500, 48, seed=23, n_ft=256)
    w = np.exp(rng.uniform(np.log(1e-4), np.log(1e2), 12000)) * rng.choice([-1.0, 1.0], 12000)
    cfg["w"] = w
    x, y, wd = to_dev(cfg["x"], cfg["y"], w)
    fused = gpu_plan(cfg)
    fused.set_launch(chunk_len, 0)
    s_f = fused(x, wd, y).cpu().numpy()
    stored = gpu_plan(cfg, materialize=True)
    s_m = stored(x, wd, y).cpu().numpy()
    em = err_scale(s_f, s_m, _sabs(cfg))
    e3 = _err3(cfg, s_f)
    print("decades: fused-stored %.2e fused-O3 %.2e (err_scale)" % (em, e3))
    assert em < 1e-6 and e3 < 2e-5
