"""The five benchmark workloads as seeded synthetic inputs.

Each entry mirrors one workload of the project's benchmark definition:
  tiny      Gauss, d=3, N=M=1000, uniform ball, P=64 distance-QMC, N_ft=128
  scale     d=50, N=M=60000, 10-component Gaussian mixture, w~N(0,1),
            Gauss or Laplace, P=1000, N_ft=1024
  precision energy kernel, d=784, image-like vectors, sources = targets =
            [X;Y] (2e5 points), weights (1/N, -1/M), P=2000, N_ft=1024
  batched   256 independent Gauss problems, N,M log-uniform in [1e3,1e5],
            d in {3,10,50}, P=256 (see make_batched)
  mmd       one MMD gradient-flow step, d=20, N=M=2e5, Gauss or energy,
            P=512, N_ft=1024
``frac`` scales N and M down (for tests) while keeping every other recipe
parameter.  Arrays are float64; callers cast to float32 for the GPU.
"""
import functools
import numpy as np

from .points import (unit_ball, gaussian_mixture, image_like, mmd_particles,
                     median_rule_sigma)
from .directions import directions

# Paper defaults for the rescaling threshold T and the number of Fourier
# modes N_ft (App. I, Steps 1-2); the energy kernel takes T=0.45 with its
# periodic extension (App. J).
DEFAULT_T = {"gauss": 0.3, "laplace": 0.1, "energy": 0.45,
             "matern32": 0.2, "matern52": 0.2, "matern72": 0.2}
DEFAULT_NFT = {"gauss": 128, "laplace": 1024, "energy": 1024,
               "matern32": 512, "matern52": 512, "matern72": 512}

CONFIGS = ("tiny", "scale", "precision", "batched", "mmd")


@functools.lru_cache(maxsize=32)
def _cached_dirs(kind, d, P, seed):
    return directions(kind, d, P, seed)


def bound_R(x, y):
    """max ||x_n|| + max ||y_m|| about the origin (App. I, Step 1)."""
    return float(np.linalg.norm(x, axis=1).max() + np.linalg.norm(y, axis=1).max())


def _finish(cfg):
    cfg["R"] = bound_R(cfg["x"], cfg["y"])
    cfg["T"] = DEFAULT_T[cfg["kernel"]]
    cfg["N"] = cfg["x"].shape[0]
    cfg["M"] = cfg["y"].shape[0]
    cfg["d"] = cfg["x"].shape[1]
    cfg["P"] = cfg["xi"].shape[1]
    return cfg


def make_config(name, kernel=None, frac=1.0, dirs=None, P=None, seed=None):
    """Build one workload.  Returns a dict with x (N,d), y (M,d), w (N,),
    xi (d,P), kernel, scale (sigma = 1/alpha), n_ft, T, R and sizes."""
    if name == "tiny":
        rng = np.random.default_rng(0 if seed is None else seed)
        n = max(int(round(1000 * frac)), 1)
        x = unit_ball(n, 3, rng)
        y = unit_ball(n, 3, rng)
        w = rng.random(n)
        sigma = median_rule_sigma(x, y, rng, n_pairs=10**6)
        P = P or 64
        xi = _cached_dirs(dirs or "distance", 3, P, 100)
        cfg = dict(x=x, y=y, w=w, xi=xi, kernel=kernel or "gauss",
                   scale=sigma, n_ft=128)
    elif name == "scale":
        rng = np.random.default_rng(1 if seed is None else seed)
        n = max(int(round(60000 * frac)), 1)
        x, means = gaussian_mixture(n, 50, rng)
        y, _ = gaussian_mixture(n, 50, rng, means=means)
        w = rng.standard_normal(n)
        sigma = median_rule_sigma(x, y, rng)
        P = P or 1000
        xi = _cached_dirs(dirs or "distance", 50, P, 101)
        cfg = dict(x=x, y=y, w=w, xi=xi, kernel=kernel or "gauss",
                   scale=sigma, n_ft=1024)
    elif name == "precision":
        rng = np.random.default_rng(2 if seed is None else seed)
        n = max(int(round(100000 * frac)), 1)
        a = image_like(n, 784, rng)
        b = image_like(n, 784, rng)
        z = np.concatenate([a, b], axis=0)
        w = np.concatenate([np.full(n, 1.0 / n), np.full(n, -1.0 / n)])
        P = P or 2000
        xi = _cached_dirs(dirs or "orth", 784, P, 102)
        cfg = dict(x=z, y=z, w=w, xi=xi, kernel=kernel or "energy",
                   scale=1.0, n_ft=1024, same_xy=True)
    elif name == "mmd":
        rng = np.random.default_rng(4 if seed is None else seed)
        n = max(int(round(200000 * frac)), 1)
        part, targ = mmd_particles(n, n, 20, rng)
        src = np.concatenate([part, targ], axis=0)
        w = np.concatenate([np.full(n, 1.0 / n**2), np.full(n, -1.0 / (n * n))])
        kern = kernel or "gauss"
        sigma = median_rule_sigma(part, targ, rng) if kern != "energy" else 1.0
        P = P or 512
        xi = _cached_dirs(dirs or "distance", 20, P, 104)
        # the targets (particles) are the first n sources
        cfg = dict(x=src, y=part, w=w, xi=xi, kernel=kern, scale=sigma,
                   n_ft=1024, targets_prefix=True)
    else:
        raise ValueError(f"unknown workload {name!r}")
    cfg["name"] = name
    return _finish(cfg)


def make_batched(n_problems=256, P=256, frac=1.0, seed=3):
    """Independent Gauss problems with N_i, M_i = round(10^U[3,5]) (times
    frac), d_i uniform in {3,10,50}, mixture points with per-problem means,
    per-problem sigma by the median rule, and a distance-QMC set per d with
    a per-problem random rotation."""
    from .directions import random_rotation
    probs = []
    for i in range(n_problems):
        rng = np.random.default_rng(seed + i)
        d = int(rng.choice([3, 10, 50]))
        n = max(int(round(10 ** rng.uniform(3, 5) * frac)), 1)
        m = max(int(round(10 ** rng.uniform(3, 5) * frac)), 1)
        x, means = gaussian_mixture(n, d, rng)
        y, _ = gaussian_mixture(m, d, rng, means=means)
        w = rng.standard_normal(n)
        sigma = median_rule_sigma(x, y, rng)
        xi = random_rotation(d, rng) @ _cached_dirs("distance", d, P, 103)
        cfg = dict(x=x, y=y, w=w, xi=xi, kernel="gauss", scale=sigma,
                   n_ft=None, name=f"batched[{i}]")
        probs.append(_finish(cfg))
    return probs
