"""O1: the exact kernel sum s_m = sum_n w_n F(||x_n - y_m||), eq. (kernel_sum),
and its gradient in y_m, in float64 with explicit differences (oracle; test
infrastructure only)."""
import numpy as np

from .kernels import basis_F, basis_dF


def _chunk(n_src, d, budget=2.0e7):
    return max(1, int(budget // max(n_src * d, 1)))


def kernel_sum_direct(kernel, x, y, w, scale):
    """s (M,) = sum_n w_n F(||x_n - y_m||) for every target y_m."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    s = np.empty(y.shape[0])
    step = _chunk(x.shape[0], x.shape[1])
    for a in range(0, y.shape[0], step):
        diff = y[a:a + step, None, :] - x[None, :, :]
        r = np.sqrt(np.einsum("mnd,mnd->mn", diff, diff))
        s[a:a + step] = basis_F(kernel, r, scale) @ w
    return s


def grad_y_direct(kernel, x, y, w, scale):
    """ds_m/dy_m (M, d) = sum_n w_n F'(r) (y_m - x_n)/r,  r = ||y_m - x_n||;
    a coincident pair (r = 0) contributes 0 (F'(0) (y-x)/r has no limit for
    the energy kernel and is 0 for Gauss)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    g = np.empty_like(y)
    step = _chunk(x.shape[0], x.shape[1])
    for a in range(0, y.shape[0], step):
        diff = y[a:a + step, None, :] - x[None, :, :]
        r = np.sqrt(np.einsum("mnd,mnd->mn", diff, diff))
        with np.errstate(divide="ignore", invalid="ignore"):
            coef = np.where(r > 0, basis_dF(kernel, r, scale) / r, 0.0) * w[None, :]
        g[a:a + step] = np.einsum("mn,mnd->md", coef, diff)
    return g


def kernel_sum_direct_gram(kernel, x, y, w, scale, budget=2.0e7):
    """s (M,) = sum_n w_n F(||x_n - y_m||) as kernel_sum_direct, with the
    squared distances from the identity ||x - y||^2 = ||x||^2 + ||y||^2 -
    2 <x, y> (clamped at 0), so the O(NMd) work is one matrix product per
    block of targets instead of an (M, N, d) array of differences; for large
    d.  Rounding: about 1e-16 (||x||^2 + ||y||^2) in the squared distance,
    i.e. ~1e-8 ||x|| in r where points coincide (0 exactly in
    kernel_sum_direct)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    xx = np.einsum("nd,nd->n", x, x)
    yy = np.einsum("md,md->m", y, y)
    s = np.empty(y.shape[0])
    step = max(1, int(budget // max(x.shape[0], 1)))
    for a in range(0, y.shape[0], step):
        r2 = yy[a:a + step, None] + xx[None, :] - 2.0 * (y[a:a + step] @ x.T)
        r = np.sqrt(np.maximum(r2, 0.0))
        s[a:a + step] = basis_F(kernel, r, scale) @ w
    return s
