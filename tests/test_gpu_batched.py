"""Batched form on the GPU: many uneven problems in one launch per phase,
replayed from a HIP graph, each checked against the FP64 oracle.  Batches of
d <= 64 run the fused kernels (projections inside spread and gather); with
materialize=True, or a problem of d > 64, the stored-projection kernels."""
import numpy as np
import pytest

import oracle as O
from workloads.configs import make_batched
from helpers import rel_l2, to_dev, oracle_inputs, DEFAULT_T

pytestmark = pytest.mark.gpu


def _problems(n=10, P=24, frac=0.03, seed=50):
    import paper_2410_01316_amd as F
    probs = make_batched(n_problems=n, P=P, frac=frac, seed=seed)
    for pr in probs:
        pr["n_ft"] = F.choose_nft("gauss", pr["d"], pr["R"], scale=pr["scale"], T=0.3,
                                  candidates=(256, 512, 1024))
    return probs


def _batch(probs, materialize=False, **tuning):
    import paper_2410_01316_amd as F
    return F.Batch([dict(xi=p["xi"], n_ft=p["n_ft"], scale=p["scale"], R=p["R"], n_max=p["N"],
                         m_max=p["M"]) for p in probs], kernel="gauss", T=0.3, tuning=tuning,
                   materialize=materialize)


def _plan(p, materialize=False):
    import paper_2410_01316_amd as F
    return F.Plan(p["xi"], kernel="gauss", n_ft=p["n_ft"], scale=p["scale"], R=p["R"], T=0.3,
                  n_max=p["N"], m_max=p["M"], materialize=materialize)


def _inputs(probs):
    xs, ys, ws = [], [], []
    for p in probs:
        x, y, w = to_dev(p["x"], p["y"], p["w"])
        xs.append(x); ys.append(y); ws.append(w)
    return xs, ws, ys


def _o3(p):
    x, y, w, xi = oracle_inputs(p)
    tau = O.rescale_tau("gauss", p["R"], p["scale"], 0.3)
    return O.kernel_sum_fourier("gauss", x, y, w, xi, p["scale"], p["n_ft"], tau)


def test_batched_matches_oracle_per_problem():
    probs = _problems()
    b = _batch(probs)
    xs, ws, ys = _inputs(probs)
    outs = b(xs, ws, ys)
    b.check()
    for p, s in zip(probs, outs):
        e = rel_l2(s.cpu().numpy(), _o3(p))
        print(p["name"], p["d"], p["N"], p["M"], p["n_ft"], "%.2e" % e)
        assert e < 1e-4


def test_batched_equals_single_plans_and_replays():
    import paper_2410_01316_amd as F
    probs = _problems(n=6, seed=70)
    b = _batch(probs)
    xs, ws, ys = _inputs(probs)
    first = [s.cpu().numpy().copy() for s in b(xs, ws, ys)]
    outs = [s.clone() for s in b(xs, ws, ys)]     # graph replay
    for a, s in zip(first, outs):
        assert np.array_equal(a, s.cpu().numpy())
    for p, a, x, w, y in zip(probs, first, xs, ws, ys):
        # the fused batch runs the single plan's fused kernel bodies (split-f16
        # projections): same results up to chunking and accumulation order
        e1 = rel_l2(a, _plan(p)(x, w, y).cpu().numpy())
        # stored FP32-MFMA projections round differently (FP32 level)
        e2 = rel_l2(a, _plan(p, materialize=True)(x, w, y).cpu().numpy())
        print(p["name"], p["d"], p["N"], p["M"], "%.1e %.1e" % (e1, e2))
        assert e1 < 1e-6 and e2 < 1e-5


def test_materialized_batch_equals_stored_plans():
    probs = _problems(n=6, seed=75)
    b = _batch(probs, materialize=True)
    xs, ws, ys = _inputs(probs)
    outs = b(xs, ws, ys)
    b.check()
    for p, s, x, w, y in zip(probs, outs, xs, ws, ys):
        a = s.cpu().numpy()
        assert rel_l2(a, _plan(p, materialize=True)(x, w, y).cpu().numpy()) < 1e-6
        assert rel_l2(a, _o3(p)) < 1e-4


def test_batch_with_a_large_d_problem_and_tiny_problems():
    """A problem of d = 70 sends the whole batch to the stored-projection
    kernels; problems of one source or one target and same-x-y problems
    run in both forms."""
    from workloads.configs import _finish, bound_R
    from workloads.points import gaussian_mixture, median_rule_sigma
    from workloads.directions import directions
    rng = np.random.default_rng(333)
    base = _problems(n=3, seed=140)
    extra = []
    for d, n, m in [(70, 900, 700), (10, 1, 300), (3, 500, 1)]:
        x, means = gaussian_mixture(n, d, rng)
        y, _ = gaussian_mixture(m, d, rng, means=means)
        sigma = median_rule_sigma(np.vstack([x, y]), np.vstack([y, x]), rng)
        xi = directions("orth", d, 24, seed=9)
        cfg = _finish(dict(x=x, y=y, w=rng.standard_normal(n), xi=xi, kernel="gauss",
                           scale=sigma, n_ft=256, name=f"extra d={d}"))
        extra.append(cfg)
    same = dict(base[0], y=base[0]["x"], M=base[0]["N"], name="same x y")
    same["R"] = bound_R(same["x"], same["y"])
    small = base + extra[1:] + [same]
    for probs, label in [(small, "fused"), (small + extra[:1], "stored")]:
        b = _batch(probs)
        xs, ws, ys = _inputs(probs)
        k = len(small) - 1
        xs[k] = ys[k]                         # same tensor: sources are the targets
        outs = b(xs, ws, ys)
        b.check()
        for p, s in zip(probs, outs):
            e = rel_l2(s.cpu().numpy(), _o3(p))
            print(label, p["name"], p["d"], p["N"], p["M"], "%.2e" % e)
            assert e < 1e-4


def test_batched_size_change_recaptures_and_direct_mode():
    probs = _problems(n=5, seed=90)
    b = _batch(probs)
    xs, ws, ys = _inputs(probs)
    b(xs, ws, ys)
    # smaller inputs: new task lists and a new graph
    xs2 = [x[: max(1, x.shape[0] // 2)].contiguous() for x in xs]
    ws2 = [w[: max(1, w.shape[0] // 2)].contiguous() for w in ws]
    ys2 = [y[: max(1, y.shape[0] // 3)].contiguous() for y in ys]
    outs = b(xs2, ws2, ys2)
    for p, s, x, w, y in zip(probs, outs, xs2, ws2, ys2):
        sub = dict(p, x=p["x"][: x.shape[0]], w=p["w"][: w.shape[0]], y=p["y"][: y.shape[0]])
        assert rel_l2(s.cpu().numpy(), _o3(sub)) < 1e-4
    b.set_tuning(use_graph=-1, blocks_per_cu=2, gather_group=16, spread_chunk=4096)
    outs_direct = b(xs2, ws2, ys2)
    for s, t in zip(outs, outs_direct):
        assert rel_l2(t.cpu().numpy(), s.cpu().numpy()) < 1e-6


def test_autotuner_picks_a_valid_tuning(tmp_path):
    from paper_2410_01316_amd.autotune import autotune
    probs = _problems(n=4, seed=120)
    b = _batch(probs)
    xs, ws, ys = _inputs(probs)
    cache = str(tmp_path / "tune.json")
    best, t = autotune(b, xs, ws, ys, reps=2, cache_path=cache,
                       candidates={"blocks_per_cu": [2, 4], "gather_group": [0, 16]})
    assert t > 0 and set(best) == {"blocks_per_cu", "gather_group"}
    best2, _ = autotune(b, xs, ws, ys, reps=2, cache_path=cache)
    assert best2 == best                          # served from the cache
    outs = b(xs, ws, ys)
    for p, s in zip(probs, outs):
        assert rel_l2(s.cpu().numpy(), _o3(p)) < 1e-4
