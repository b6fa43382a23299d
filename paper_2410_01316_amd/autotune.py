"""Launch-shape autotuner for the batched form.

Times a small grid of persistent-launch shapes (workgroups per compute unit,
spread chunk size, gather direction-group size) on the actual batch and
inputs, keeps the fastest, and caches the choice in a JSON file keyed by the
device and a signature of the workload.
"""
import hashlib
import itertools
import json
import os
import time

import torch

DEFAULT_CANDIDATES = {
    "blocks_per_cu": [2, 4, 8],
    "spread_chunk": [0, 16384, 65536],
    "gather_group": [0, 32, 128],
}


def workload_signature(batch, xs, ys):
    dev = torch.cuda.get_device_properties(batch.device)
    key = dict(device=dev.name, cus=dev.multi_processor_count, P=batch.P, n=batch.n,
               d=sorted(set(batch.d)),
               sizes=[(int(x.shape[0]), int(y.shape[0])) for x, y in zip(xs, ys)])
    return hashlib.sha256(json.dumps(key, sort_keys=True).encode()).hexdigest()[:24]


def _time(batch, xs, ws, ys, outs, reps):
    batch(xs, ws, ys, outs)                # first call records the graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        batch(xs, ws, ys, outs)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def autotune(batch, xs, ws, ys, outs=None, candidates=None, reps=5, cache_path=None,
             log=None):
    """Pick the fastest tuning for this batch and inputs; returns
    (tuning dict, seconds per call).  The batch is left set to that tuning."""
    cands = candidates or DEFAULT_CANDIDATES
    if outs is None:
        outs = [torch.empty(y.shape[0], dtype=torch.float32, device=batch.device) for y in ys]
    sig = workload_signature(batch, xs, ys)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if sig in cache:
        best = cache[sig]["tuning"]
        batch.set_tuning(**best)
        return best, cache[sig]["seconds"]
    keys = list(cands)
    best, best_t = None, float("inf")
    for vals in itertools.product(*[cands[k] for k in keys]):
        tun = dict(zip(keys, vals))
        batch.set_tuning(**tun)
        t = _time(batch, xs, ws, ys, outs, reps)
        if log:
            log(f"autotune {tun}: {t * 1e3:.3f} ms")
        if t < best_t:
            best, best_t = tun, t
    batch.set_tuning(**best)
    if cache_path:
        cache[sig] = {"tuning": best, "seconds": best_t}
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return best, best_t
