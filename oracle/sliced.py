"""O2: the sliced kernel sum with the exact 1-D basis function,
s_m ~ (1/P) sum_p sum_n w_n f(|<xi_p, x_n - y_m>|), eq. (kernel_sum_sliced),
in float64 (oracle; test infrastructure only).  Cost O(P N M): small inputs."""
import numpy as np

from .kernels import SlicedBasis


def kernel_sum_sliced(kernel, x, y, w, xi, scale, basis=None):
    """xi is (d, P) with unit columns."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)
    d, P = xi.shape
    px = x @ xi                                  # <xi_p, x_n>   (N, P)
    py = y @ xi                                  # <xi_p, y_m>   (M, P)
    if basis is None:
        t_max = (np.abs(px).max(initial=0.0) + np.abs(py).max(initial=0.0)) * 1.0001 + 1e-300
        basis = SlicedBasis(kernel, d, scale, t_max)
    s = np.empty(y.shape[0])
    for m in range(y.shape[0]):
        fv = basis(np.abs(px - py[m][None, :]))  # f(|<xi_p, x_n - y_m>|)  (N, P)
        s[m] = (w @ fv).sum() / P
    return s
