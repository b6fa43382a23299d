"""O3: Fourier slicing as an exact non-uniform DFT (oracle; test
infrastructure only).

Rescale (App. I, Step 1):  x~_{n,p} = tau <xi_p, x_n>,  y~_{m,p} = tau <xi_p, y_m>.
Per direction (App. I, Step 3, eq. 1d_sum_fourier):
    w^_{k,p} = sum_n w_n exp(-2 pi i k x~_{n,p})
    t_{m,p}  = sum_{k=-K}^{K} c'_k w^_{k,p} exp(2 pi i k y~_{m,p})
Average (eq. kernel_sum_sliced / Fourier-slicing):  s_m = (1/P) sum_p Re t_{m,p}.
c'_k are the coefficients of the rescaled kernel with half weight at +-K.
Cost O(P (2K+1) (N+M)), no FFT: every exponential is evaluated.
"""
import numpy as np

from .kernels import fourier_coefficients, truncated_coefficients


def project(x, xi, tau):
    """Rescaled projections tau <xi_p, x_n>, shape (N, P)."""
    return tau * (np.asarray(x, dtype=np.float64) @ np.asarray(xi, dtype=np.float64))


def _modes(kernel, d, scale, tau, n_ft):
    c = fourier_coefficients(kernel, d, scale, tau, n_ft)
    return truncated_coefficients(c)


def _adjoint_ndft(pts, weights, ks, budget=2.0e7):
    """w^_k = sum_n weights_n exp(-2 pi i k pts_n) for one direction."""
    out = np.zeros(len(ks), dtype=np.complex128)
    step = max(1, int(budget // len(ks)))
    for a in range(0, len(pts), step):
        e = np.exp(-2j * np.pi * np.outer(ks, pts[a:a + step]))
        out += e @ weights[a:a + step]
    return out


def _ndft(pts, coeffs, ks, budget=2.0e7):
    """sum_k coeffs_k exp(2 pi i k pts_m) for one direction."""
    out = np.empty(len(pts), dtype=np.complex128)
    step = max(1, int(budget // len(ks)))
    for a in range(0, len(pts), step):
        e = np.exp(2j * np.pi * np.outer(pts[a:a + step], ks))
        out[a:a + step] = e @ coeffs
    return out


def kernel_sum_fourier(kernel, x, y, w, xi, scale, n_ft, tau):
    """s (M,) by Fourier slicing with exact non-uniform DFTs."""
    xi = np.asarray(xi, dtype=np.float64)
    d, P = xi.shape
    ks, cp = _modes(kernel, d, scale, tau, n_ft)
    xt = project(x, xi, tau)
    yt = project(y, xi, tau)
    w = np.asarray(w, dtype=np.float64)
    s = np.zeros(yt.shape[0])
    for p in range(P):
        what = _adjoint_ndft(xt[:, p], w, ks)
        s += _ndft(yt[:, p], cp * what, ks).real
    return s / P


def grad_y_fourier(kernel, x, y, w, xi, scale, n_ft, tau):
    """ds_m/dy_m (M, d) = (tau/P) sum_p xi_p Re sum_k (2 pi i k) c'_k
    w^_{k,p} exp(2 pi i k y~_{m,p})  (chain rule through y~ = tau <xi, y>)."""
    xi = np.asarray(xi, dtype=np.float64)
    d, P = xi.shape
    ks, cp = _modes(kernel, d, scale, tau, n_ft)
    xt = project(x, xi, tau)
    yt = project(y, xi, tau)
    w = np.asarray(w, dtype=np.float64)
    g = np.zeros((yt.shape[0], d))
    for p in range(P):
        what = _adjoint_ndft(xt[:, p], w, ks)
        tprime = _ndft(yt[:, p], 2j * np.pi * ks * cp * what, ks).real
        g += np.outer(tprime, xi[:, p])
    return g * (tau / P)


def grad_w_fourier(kernel, x, y, v, xi, scale, n_ft, tau):
    """Vector-Jacobian product with respect to the weights:
    (K^T v)_n = sum_m v_m ds_m/dw_n
              = (1/P) sum_p Re sum_k c'_k exp(-2 pi i k x~_{n,p}) sum_m v_m exp(2 pi i k y~_{m,p})."""
    xi = np.asarray(xi, dtype=np.float64)
    d, P = xi.shape
    ks, cp = _modes(kernel, d, scale, tau, n_ft)
    xt = project(x, xi, tau)
    yt = project(y, xi, tau)
    v = np.asarray(v, dtype=np.float64)
    g = np.zeros(xt.shape[0])
    for p in range(P):
        vhat = np.conj(_adjoint_ndft(yt[:, p], v, ks))      # sum_m v_m e^{+2 pi i k y~}
        g += _ndft(xt[:, p], np.conj(cp * vhat), ks).conj().real
    return g / P


def grad_x_fourier(kernel, x, y, w, v, xi, scale, n_ft, tau):
    """Vector-Jacobian product with respect to the sources:
    sum_m v_m ds_m/dx_n = w_n (tau/P) sum_p xi_p Re sum_k (-2 pi i k) c'_k
        exp(-2 pi i k x~_{n,p}) sum_m v_m exp(2 pi i k y~_{m,p})
    (chain rule through x~ = tau <xi, x> in the source factor of eq.
    Fourier-slicing)."""
    xi = np.asarray(xi, dtype=np.float64)
    d, P = xi.shape
    ks, cp = _modes(kernel, d, scale, tau, n_ft)
    xt = project(x, xi, tau)
    yt = project(y, xi, tau)
    v = np.asarray(v, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    g = np.zeros((xt.shape[0], d))
    for p in range(P):
        vhat = np.conj(_adjoint_ndft(yt[:, p], v, ks))      # sum_m v_m e^{+2 pi i k y~}
        # sum_k (-2 pi i k) c'_k vhat_k e^{-2 pi i k x~}
        dx = _ndft(xt[:, p], np.conj(-2j * np.pi * ks * cp * vhat), ks).conj().real
        g += np.outer(dx, xi[:, p])
    return g * (tau / P) * w[:, None]
