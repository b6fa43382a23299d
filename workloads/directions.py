"""Seeded direction sets xi_1..xi_P on the sphere S^{d-1} (Sec. 4.1, App. E, H).

Every function returns a (d, P) float64 array whose columns are unit vectors.
These are inputs of the summation method (the paper excludes their
construction from its timings); they are produced here, once, on the host.
"""
import numpy as np
from scipy.stats import qmc
from scipy.special import ndtri


def _unit_columns(a):
    return a / np.linalg.norm(a, axis=0, keepdims=True)


def iid_directions(d, P, rng):
    """P i.i.d. uniform directions (normalised Gaussian vectors)."""
    return _unit_columns(rng.standard_normal((d, P)))


def random_rotation(d, rng):
    """A Haar-distributed orthogonal d x d matrix (Q factor of a Gaussian
    matrix with the signs of R's diagonal folded in)."""
    q, r = np.linalg.qr(rng.standard_normal((d, d)))
    return q * np.sign(np.diag(r))[None, :]


def sobol_directions(d, P, rng):
    """Scrambled Sobol points in [0,1]^d mapped through the normal inverse CDF
    and projected to the sphere (Sec. 4.1, 'Sobol Sequence')."""
    u = qmc.Sobol(d, scramble=True, seed=rng).random(P)
    u = np.clip(u, 1e-12, 1 - 1e-12)
    return _unit_columns(ndtri(u).T)


def orthogonal_directions(d, P, rng):
    """ceil(P/d) independent Haar orthogonal matrices; the first P of their
    columns (Sec. 4.1, 'Orthogonal')."""
    blocks = [random_rotation(d, rng) for _ in range(-(-P // d))]
    return np.concatenate(blocks, axis=1)[:, :P]


def _distance_qmc_torch(xi0, iters, lr, device):
    """The same projected-Adam iteration as below, in float64 torch on
    `device` (used for large P, where the O(P^2 d) energy gradient dominates)."""
    import torch
    xi = torch.tensor(xi0, dtype=torch.float64, device=device)
    m = torch.zeros_like(xi)
    v = torch.zeros_like(xi)
    b1, b2, eps = 0.9, 0.999, 1e-12
    eye = torch.eye(xi.shape[0], dtype=torch.bool, device=device)
    for it in range(1, iters + 1):
        g = (xi @ xi.T).clamp_(-1.0, 1.0)
        ia = 1.0 / torch.sqrt(torch.clamp(2.0 - 2.0 * g, min=1e-24))
        ia.masked_fill_(eye, 0.0)
        ib = 1.0 / torch.sqrt(torch.clamp(2.0 + 2.0 * g, min=1e-24))
        grad = xi * (ia.sum(1) + ib.sum(1))[:, None] + (ib - ia) @ xi
        grad -= (grad * xi).sum(1, keepdim=True) * xi
        m = b1 * m + (1 - b1) * grad
        v = b2 * v + (1 - b2) * grad * grad
        step = lr * (1.0 - 0.9 * it / iters)
        xi = xi + step * (m / (1 - b1 ** it)) / (torch.sqrt(v / (1 - b2 ** it)) + eps)
        xi = xi / torch.linalg.norm(xi, dim=1, keepdim=True)
    return xi.cpu().numpy()


def distance_qmc_directions(d, P, rng, iters=400, lr=None, device=None):
    """Distance QMC design: P unit vectors that (locally) minimise the
    symmetrised distance energy E_sym(xi) = -2 sum_{p,q} (|xi_p - xi_q| +
    |xi_p + xi_q|)  (eq. distance-sym, App. H), by projected Adam steps
    started from i.i.d. directions.  For P <= d an orthonormal system is
    returned, which is a minimiser (App. H)."""
    if P <= d:
        return random_rotation(d, rng)[:, :P]
    xi = iid_directions(d, P, rng).T.copy()          # (P, d) rows
    if lr is None:                       # a fraction of the typical spacing
        lr = 0.05 * P ** (-1.0 / max(d - 1, 1))
    if device is not None:
        return _distance_qmc_torch(xi, iters, lr, device).T.copy()
    m = np.zeros_like(xi)
    v = np.zeros_like(xi)
    b1, b2, eps = 0.9, 0.999, 1e-12
    for it in range(1, iters + 1):
        g = np.clip(xi @ xi.T, -1.0, 1.0)
        a = np.sqrt(np.maximum(2.0 - 2.0 * g, 1e-24))
        b = np.sqrt(np.maximum(2.0 + 2.0 * g, 1e-24))
        ia = 1.0 / a
        np.fill_diagonal(ia, 0.0)
        ib = 1.0 / b
        # ascent direction of sum(|xi_p - xi_q| + |xi_p + xi_q|)
        grad = xi * (ia.sum(1) + ib.sum(1))[:, None] + (ib - ia) @ xi
        grad -= (grad * xi).sum(1, keepdims=True) * xi      # tangent part
        m = b1 * m + (1 - b1) * grad
        v = b2 * v + (1 - b2) * grad * grad
        step = lr * (1.0 - 0.9 * it / iters)
        xi = xi + step * (m / (1 - b1 ** it)) / (np.sqrt(v / (1 - b2 ** it)) + eps)
        xi /= np.linalg.norm(xi, axis=1, keepdims=True)
    return xi.T.copy()


def directions(kind, d, P, seed, rotate=True, device=None, iters=400):
    """Direction set by name ('iid', 'sobol', 'orth', 'distance'); QMC sets
    get a seeded Haar rotation so the estimator is unbiased (App. E).
    device: optional torch device for the distance-QMC construction;
    iters: its number of projected-Adam steps."""
    rng = np.random.default_rng(seed)
    if kind == "iid":
        return iid_directions(d, P, rng)
    if kind == "sobol":
        xi = sobol_directions(d, P, rng)
    elif kind == "orth":
        xi = orthogonal_directions(d, P, rng)
    elif kind == "distance":
        xi = distance_qmc_directions(d, P, rng, iters=iters, device=device)
    else:
        raise ValueError(f"unknown direction set {kind!r}")
    if rotate:
        xi = random_rotation(d, rng) @ xi
    return _unit_columns(xi)
