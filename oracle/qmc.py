"""Distance QMC designs (App. H): P unit vectors that locally maximise the
sum of pairwise distances sum_{p,q} (|xi_p - xi_q| + |xi_p + xi_q|), i.e.
minimise the symmetrised distance energy of eq. distance-sym, built by
projected Adam steps (oracle; test infrastructure only, FP64)."""
import numpy as np


def distance_energy(xi):
    """sum_{p,q} (|xi_p - xi_q| + |xi_p + xi_q|) for the rows xi_p of xi (P, d)."""
    xi = np.asarray(xi, dtype=np.float64)
    dm = np.linalg.norm(xi[:, None, :] - xi[None, :, :], axis=2)
    dp = np.linalg.norm(xi[:, None, :] + xi[None, :, :], axis=2)
    return float(dm.sum() + dp.sum())


def distance_energy_grad(xi):
    """Gradient of distance_energy / 2 with respect to row p (each pair is
    counted twice in the double sum):
    sum_{q != p} (xi_p - xi_q)/|xi_p - xi_q| + sum_q (xi_p + xi_q)/|xi_p + xi_q|."""
    xi = np.asarray(xi, dtype=np.float64)
    diff = xi[:, None, :] - xi[None, :, :]
    summ = xi[:, None, :] + xi[None, :, :]
    nd = np.linalg.norm(diff, axis=2)
    ns = np.linalg.norm(summ, axis=2)
    with np.errstate(divide="ignore", invalid="ignore"):
        a = np.where(nd > 0, 1.0 / nd, 0.0)
        b = np.where(ns > 0, 1.0 / ns, 0.0)
    return np.einsum("pq,pqd->pd", a, diff) + np.einsum("pq,pqd->pd", b, summ)


def projected_adam(xi0, iters, lr, b1=0.9, b2=0.999, eps=1e-12):
    """Ascent on distance_energy by Adam on the tangent component of the
    gradient, each step followed by renormalising the rows; the step size
    decays linearly from lr to lr/10 over the iterations."""
    xi = np.array(xi0, dtype=np.float64)
    xi /= np.linalg.norm(xi, axis=1, keepdims=True)
    m = np.zeros_like(xi)
    v = np.zeros_like(xi)
    for it in range(1, iters + 1):
        g = distance_energy_grad(xi)
        g -= (g * xi).sum(1, keepdims=True) * xi
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        step = lr * (1.0 - 0.9 * it / iters)
        xi = xi + step * (m / (1 - b1 ** it)) / (np.sqrt(v / (1 - b2 ** it)) + eps)
        xi /= np.linalg.norm(xi, axis=1, keepdims=True)
    return xi


def rotate_directions(q, xi):
    """The randomised design of App. E for a given orthogonal matrix q: every
    direction (row of xi, shape (P, d)) mapped to q xi_p, then rescaled to
    unit length (which only removes rounding when q is orthogonal)."""
    q = np.asarray(q, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)
    out = xi @ q.T                         # row p: sum_j q[i, j] xi[p, j]
    return out / np.linalg.norm(out, axis=1, keepdims=True)
