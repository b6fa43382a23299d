"""Batched form on the GPU: many uneven problems in one persistent launch per
phase, replayed from a HIP graph, each checked against the FP64 oracle."""
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


def _batch(probs, **tuning):
    import paper_2410_01316_amd as F
    return F.Batch([dict(xi=p["xi"], n_ft=p["n_ft"], scale=p["scale"], R=p["R"], n_max=p["N"],
                         m_max=p["M"]) for p in probs], kernel="gauss", T=0.3, tuning=tuning)


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
        # the batched kernels share the stored-projection path's arithmetic
        # (FP32 MFMA projections): same results up to accumulation order
        plan = F.Plan(p["xi"], kernel="gauss", n_ft=p["n_ft"], scale=p["scale"], R=p["R"],
                      T=0.3, n_max=p["N"], m_max=p["M"], materialize=True)
        assert rel_l2(a, plan(x, w, y).cpu().numpy()) < 1e-6
        # the default single plan projects with split-f16 MFMAs (FP32-level,
        # different rounding)
        fused = F.Plan(p["xi"], kernel="gauss", n_ft=p["n_ft"], scale=p["scale"], R=p["R"],
                       T=0.3, n_max=p["N"], m_max=p["M"])
        assert rel_l2(a, fused(x, w, y).cpu().numpy()) < 1e-5


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
