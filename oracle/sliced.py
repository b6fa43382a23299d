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


def grad_sliced_energy(x, y, w, v, xi):
    """Vector-Jacobian products of the exact sliced energy sum
    s_m = (1/P) sum_p sum_n w_n (-c_d) |<xi_p, x_n - y_m>| (eq.
    kernel_sum_sliced with f(t) = -c_d |t|, Table 'tab:kernels' Riesz row,
    r = 1) for the cotangent v:
      grad_y[m] = v_m ds_m/dy_m = (c_d/P) v_m sum_p sum_n w_n sign(t) xi_p,
      grad_x[n] = sum_m v_m ds_m/dx_n = -(c_d/P) w_n sum_p sum_m v_m sign(t) xi_p,
      grad_w[n] = sum_m v_m ds_m/dw_n = (1/P) sum_p sum_m v_m (-c_d) |t|,
    t = <xi_p, x_n - y_m>, with sign(0) = 0 at coincident projections (the
    symmetric difference quotient of |t| there)."""
    from .kernels import energy_cd
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)
    d, P = xi.shape
    cd = energy_cd(d)
    px = x @ xi                                  # (N, P)
    py = y @ xi                                  # (M, P)
    gy = np.zeros_like(y)
    gx = np.zeros_like(x)
    gw = np.zeros(x.shape[0])
    for p in range(P):
        t = px[:, p][:, None] - py[:, p][None, :]          # (N, M)
        sg = np.sign(t)
        gy += np.outer(v * (w @ sg), xi[:, p])
        gx += np.outer(w * (sg @ v), xi[:, p])
        gw += np.abs(t) @ v
    return -cd / P * gx, cd / P * gy, -cd / P * gw
