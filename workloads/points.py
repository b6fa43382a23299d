"""Seeded point clouds and weights shaped like the paper's workloads.

The paper measures on Letters, MNIST, FashionMNIST and CIFAR10 (Sec. 4.3,
App. K); none of these datasets is used here.  The generators below draw
synthetic stand-ins with the same sizes and dimensions.
"""
import numpy as np


def unit_ball(n, d, rng):
    """n points i.i.d. uniform in the unit ball of R^d (Gaussian direction
    times a U^(1/d) radius)."""
    g = rng.standard_normal((n, d))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    r = rng.random(n) ** (1.0 / d)
    return g * r[:, None]


def gaussian_mixture(n, d, rng, n_comp=10, mean_var=4.0, means=None):
    """n points from an equal-weight Gaussian mixture with unit covariance and
    component means drawn from N(0, mean_var I).  Returns (points, means)."""
    if means is None:
        means = rng.standard_normal((n_comp, d)) * np.sqrt(mean_var)
    comp = rng.integers(0, means.shape[0], size=n)
    return means[comp] + rng.standard_normal((n, d)), means


def image_like(n, d, rng, p_zero=0.8):
    """n points in [0,1]^d where each entry is exactly zero with probability
    p_zero and uniform on [0,1) otherwise (sparse, image-like vectors)."""
    z = rng.random((n, d))
    keep = rng.random((n, d)) >= p_zero
    return np.where(keep, z, 0.0)


def mmd_particles(n_particles, n_targets, d, rng, shift=3.0, var=0.5):
    """Target points y ~ N(0, I) and particles x ~ N(shift*1, var*I) for one
    MMD gradient-flow step (App. K.3 setting, synthetic)."""
    y = rng.standard_normal((n_targets, d))
    x = shift + np.sqrt(var) * rng.standard_normal((n_particles, d))
    return x, y


def median_rule_sigma(x, y, rng, n_pairs=1000, gamma=1.0):
    """Kernel width by the median rule (Sec. 4.1): gamma times the median of
    ||x_i - y_j|| over n_pairs seeded random pairs (all pairs when
    len(x)*len(y) <= n_pairs)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if x.shape[0] * y.shape[0] <= n_pairs:
        dist = np.linalg.norm(x[:, None, :] - y[None, :, :], axis=-1).ravel()
    else:
        i = rng.integers(0, x.shape[0], size=n_pairs)
        j = rng.integers(0, y.shape[0], size=n_pairs)
        dist = np.linalg.norm(x[i] - y[j], axis=1)
    return gamma * float(np.median(dist))
