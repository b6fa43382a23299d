"""Basis-function pairs (F, f), the sliced Fourier transform and the Fourier
coefficients of the rescaled 1-D kernel, in float64 (oracle; test
infrastructure only).

Kernels (Table 'tab:kernels', App. A):
  gauss    F(r) = exp(-r^2 / (2 sigma^2))
  laplace  F(r) = exp(-alpha r),  alpha = 1/scale  (Euclidean norm)
  energy   F(r) = -r  (Riesz kernel with r = 1, 'negative distance')
  matern32, matern52, matern72
           Matern with nu = 3/2, 5/2, 7/2 and width beta = scale (Sec. 4.1
           uses nu = p + 1/2, p in {1, 3}):
           F(r) = 2^{1-nu}/Gamma(nu) z^nu K_nu(z),  z = sqrt(2 nu) r / beta,
           which for half-integer nu is exp(-z) times a polynomial in z
"""
import functools
from math import lgamma, log, pi, sqrt

import mpmath as mp
import numpy as np

KERNELS = ("gauss", "laplace", "energy", "matern32", "matern52", "matern72")
MATERN_NU = {"matern32": 1.5, "matern52": 2.5, "matern72": 3.5}


def _matern_poly(nu):
    """Coefficients a_j (ascending powers of z) with F = exp(-z) sum_j a_j z^j
    for nu = p + 1/2:  F = exp(-z) p!/(2p)! sum_{i=0}^{p} (p+i)!/(i!(p-i)!)
    (2z)^{p-i}  (the half-integer closed form of z^nu K_nu(z))."""
    from math import factorial
    p = int(round(nu - 0.5))
    a = np.zeros(p + 1)
    for i in range(p + 1):
        a[p - i] += (factorial(p) / factorial(2 * p) * factorial(p + i)
                     / (factorial(i) * factorial(p - i)) * 2.0 ** (p - i))
    return a


def basis_F(kernel, r, scale):
    """F(r) of Table 'tab:kernels', column 2."""
    r = np.asarray(r, dtype=np.float64)
    if kernel == "gauss":
        return np.exp(-r * r / (2.0 * scale * scale))
    if kernel == "laplace":
        return np.exp(-r / scale)
    if kernel == "energy":
        return -r
    if kernel in MATERN_NU:
        nu = MATERN_NU[kernel]
        z = sqrt(2.0 * nu) * r / scale
        return np.exp(-z) * np.polynomial.polynomial.polyval(z, _matern_poly(nu))
    raise ValueError(kernel)


def basis_dF(kernel, r, scale):
    """dF/dr, used by the gradient of the direct sum."""
    r = np.asarray(r, dtype=np.float64)
    if kernel == "gauss":
        return -r / (scale * scale) * basis_F(kernel, r, scale)
    if kernel == "laplace":
        return -basis_F(kernel, r, scale) / scale
    if kernel == "energy":
        return -np.ones_like(r)
    if kernel in MATERN_NU:
        # d/dz [exp(-z) q(z)] = exp(-z) (q'(z) - q(z)),  dz/dr = sqrt(2 nu)/beta
        nu = MATERN_NU[kernel]
        a = _matern_poly(nu)
        z = sqrt(2.0 * nu) * r / scale
        P = np.polynomial.polynomial
        return (sqrt(2.0 * nu) / scale) * np.exp(-z) * (P.polyval(z, P.polyder(a)) - P.polyval(z, a))
    raise ValueError(kernel)


def energy_cd(d):
    """Constant of the sliced negative-distance kernel, f(t) = -c_d |t|
    (Table 'tab:kernels', Riesz row with r = 1):
    c_d = sqrt(pi) Gamma((d+1)/2) / Gamma(d/2)."""
    return float(np.exp(0.5 * log(pi) + lgamma((d + 1) / 2.0) - lgamma(d / 2.0)))


def _log_ft_d(kernel, omega, d, scale):
    """log of the d-dimensional Fourier transform of F(||.||) at radius omega
    (Table 'tab:kernels', column 3; convention of eq. (Fourier))."""
    omega = np.abs(np.asarray(omega, dtype=np.float64))
    if kernel == "gauss":
        s2 = scale * scale
        return 0.5 * d * np.log(2.0 * pi * s2) - 2.0 * pi * pi * s2 * omega ** 2
    if kernel == "laplace":
        alpha = 1.0 / scale
        return (lgamma((d + 1) / 2.0) + d * log(2.0) + 0.5 * (d - 1) * log(pi)
                - d * log(alpha)
                - 0.5 * (d + 1) * np.log1p(4.0 * pi * pi * omega ** 2 / alpha ** 2))
    if kernel in MATERN_NU:
        return log_ft_matern(omega, d, scale, MATERN_NU[kernel])
    raise ValueError(f"no classical Fourier transform for {kernel!r}")


def log_ft_matern(omega, d, beta, nu):
    """log F_d[F(||.||)](omega) of the Matern kernel of order nu, any nu > 0
    (Table 'tab:kernels', column 3):
    Gamma(nu + d/2) 2^{d/2} pi^{d/2} beta^d / (Gamma(nu) nu^{d/2})
    * (1 + 2 pi^2 beta^2 omega^2 / nu)^{-(nu + d/2)}."""
    omega = np.abs(np.asarray(omega, dtype=np.float64))
    return (lgamma(nu + 0.5 * d) + 0.5 * d * log(2.0) + 0.5 * d * log(pi) + d * log(beta)
            - lgamma(nu) - 0.5 * d * log(nu)
            - (nu + 0.5 * d) * np.log1p(2.0 * pi * pi * beta * beta * omega ** 2 / nu))


def sliced_ft(kernel, omega, d, scale):
    """One-dimensional Fourier transform of t -> f(|t|), obtained from the
    d-dimensional one by  F_1[f(|.|)](w) = pi^{d/2}/Gamma(d/2) |w|^{d-1}
    F_d[F(||.||)](|w|)  (the relation the paper takes from RQS2024,
    Prop. 3.1, App. A).  Evaluated in log space so that large d does not
    overflow.  Table column 5 is not used: its Gauss and Laplace prefactors
    are misprinted (they fail the d = 1 reduction to the textbook 1-D
    transforms)."""
    omega = np.abs(np.asarray(omega, dtype=np.float64))
    logft = _log_ft_d(kernel, omega, d, scale)
    if d == 1:
        return np.exp(logft)
    with np.errstate(divide="ignore"):
        lw = np.log(omega)
    out = np.exp(0.5 * d * log(pi) - lgamma(d / 2.0) + (d - 1) * lw + logft)
    return np.where(omega == 0.0, 0.0, out)


# ---------------------------------------------------------------------------
# The 1-D basis function f (Table 'tab:kernels', column 4)
# ---------------------------------------------------------------------------

def _f_gauss_mp(t, d, sigma):
    """f(t) = 1F1(d/2; 1/2; -t^2/(2 sigma^2))."""
    return mp.hyp1f1(mp.mpf(d) / 2, mp.mpf(1) / 2, -(mp.mpf(t) ** 2) / (2 * mp.mpf(sigma) ** 2))


def _f_laplace_mp(t, d, alpha):
    """f(t) = sum_n (-1)^n alpha^n sqrt(pi) Gamma((n+d)/2) /
    (n! Gamma(d/2) Gamma((n+1)/2)) t^n, the series of Table 'tab:kernels',
    summed in extended precision (the series alternates and cancels)."""
    u = mp.mpf(alpha) * mp.mpf(t)
    # G_n = Gamma((n+d)/2) / Gamma((n+1)/2),  G_{n+2} = G_n (n+d)/(n+1)
    g = [mp.gamma(mp.mpf(d) / 2) / mp.gamma(mp.mpf(1) / 2),
         mp.gamma(mp.mpf(d + 1) / 2) / mp.gamma(mp.mpf(1))]
    pref = mp.sqrt(mp.pi) / mp.gamma(mp.mpf(d) / 2)
    total = mp.mpf(0)
    powfac = mp.mpf(1)          # (-u)^n / n!
    n = 0
    biggest = mp.mpf(0)
    while True:
        term = powfac * g[n % 2] * pref
        total += term
        biggest = max(biggest, abs(term))
        if n > 2 * (u + d) + 20 and abs(term) < mp.mpf(10) ** (-mp.mp.dps + 5) * max(biggest, 1):
            break
        g[n % 2] = g[n % 2] * (n + d) / (n + 1)
        n += 1
        powfac = powfac * (-u) / n
    return total


class SlicedBasis:
    """The 1-D basis function f of the slicing relation (eq.
    sliced_basis_function), F(||x||) = E_xi f(|<xi, x>|), for one kernel,
    dimension and width, on [0, t_max].

    d = 1: f = F.  Energy kernel: f(t) = -c_d t exactly.  Gauss and Laplace,
    d >= 2: the column-4 expressions of Table 'tab:kernels' evaluated with
    mpmath at high precision on Chebyshev nodes, then interpolated (the
    interpolation error is checked against direct evaluation in the tests).
    Matern: d = 1 and d = 3 only, where f is exact (f = F, and f = (tF)'
    from eq. integral_transform at d = 3); the table gives the Matern f only
    by reference and the parity path needs only its transform.
    """

    def __init__(self, kernel, d, scale, t_max, nodes=400):
        self.kernel, self.d, self.scale = kernel, d, float(scale)
        self.t_max = float(t_max)
        self.exact = d == 1 or kernel == "energy" or kernel in MATERN_NU
        if kernel in MATERN_NU and d not in (1, 3):
            raise NotImplementedError("Matern f is provided for d = 1 and d = 3")
        if not self.exact:
            self._coef = _cheb_table(kernel, d, self.scale, self.t_max, nodes)

    def mp_value(self, t):
        """Direct extended-precision evaluation (slow)."""
        if self.kernel in MATERN_NU:
            return float(self(t))
        dps = 40 + int(2 * float(t) / self.scale) + self.d
        with mp.workdps(dps):
            if self.kernel == "gauss":
                return float(_f_gauss_mp(t, self.d, self.scale))
            return float(_f_laplace_mp(t, self.d, 1.0 / self.scale))

    def __call__(self, t):
        t = np.abs(np.asarray(t, dtype=np.float64))
        if self.kernel == "energy":
            return -energy_cd(self.d) * t
        if self.kernel in MATERN_NU and self.d == 3:
            return basis_F(self.kernel, t, self.scale) + t * basis_dF(self.kernel, t, self.scale)
        if self.d == 1:
            return basis_F(self.kernel, t, self.scale)
        if np.any(t > self.t_max * (1 + 1e-12)):
            raise ValueError("argument beyond the tabulated range")
        z = 2.0 * t / self.t_max - 1.0
        return np.polynomial.chebyshev.chebval(z, self._coef)


@functools.lru_cache(maxsize=64)
def _cheb_table(kernel, d, scale, t_max, nodes):
    j = np.arange(nodes)
    z = np.cos(pi * (j + 0.5) / nodes)              # Chebyshev points, 1st kind
    t = 0.5 * (z + 1.0) * t_max
    vals = np.empty(nodes)
    with mp.workdps(40 + int(2 * t_max / scale) + d):
        for i, ti in enumerate(t):
            if kernel == "gauss":
                vals[i] = float(_f_gauss_mp(ti, d, scale))
            else:
                vals[i] = float(_f_laplace_mp(ti, d, 1.0 / scale))
    # coefficients of the interpolant through the Chebyshev points
    k = np.arange(nodes)
    coef = (2.0 / nodes) * (np.cos(pi * np.outer(k, j + 0.5) / nodes) @ vals)
    coef[0] *= 0.5
    return coef


# ---------------------------------------------------------------------------
# Rescaling and Fourier coefficients (App. I Steps 1-2, App. J)
# ---------------------------------------------------------------------------

def rescale_tau(kernel, R, scale, T, gmax_factor=5.0):
    """tau = min{T/c, 1/(2 g_max)} with c (here the caller's bound R) =
    max ||x_n|| + max ||y_m|| and g_max = gmax_factor * scale (App. I,
    Step 1; Matern as Gauss and Laplace).  The energy kernel does not decay,
    so only T/R applies; its periodic extension (App. J) is built in
    fourier_coefficients."""
    if kernel == "energy":
        return T / R
    return min(T / R, 1.0 / (2.0 * gmax_factor * scale))


def fourier_coefficients(kernel, d, scale, tau, n_ft):
    """c_k, k = 0..K (K = n_ft/2), of the 1-periodic rescaled kernel
    g~(x) = f(|x|/tau) (c_{-k} = c_k since g~ is even and real).

    Gauss, Laplace, Matern: by Poisson summation c_k ~ F_1[g~](k) =
    tau F_1[f(|.|)](tau k) (App. I, Step 2).
    Energy: g~ is taken as the 1-periodic triangle wave equal to
    -(c_d/tau)|x| on [-1/2, 1/2) (a periodic extension in the sense of
    App. J), whose coefficients are c_0 = -c_d/(4 tau),
    c_k = c_d/(tau pi^2 k^2) for odd k and 0 for even k != 0."""
    if n_ft % 2:
        raise ValueError("n_ft must be even")
    K = n_ft // 2
    k = np.arange(K + 1, dtype=np.float64)
    if kernel == "energy":
        cd = energy_cd(d)
        c = np.zeros(K + 1)
        c[0] = -cd / (4.0 * tau)
        odd = (np.arange(K + 1) % 2) == 1
        c[odd] = cd / (tau * pi * pi * k[odd] ** 2)
        return c
    return tau * sliced_ft(kernel, tau * k, d, scale)


def truncated_coefficients(c):
    """c'_k for k = -K..K: c_k with half weight at k = +-K, i.e. the real part
    of the sum over k = -N_ft/2 .. N_ft/2 - 1 written in App. I, Step 3 and
    eq. (Fourier-slicing), made symmetric.  Returns (k, c')."""
    K = len(c) - 1
    ks = np.arange(-K, K + 1)
    cp = c[np.abs(ks)].astype(np.float64).copy()
    cp[0] *= 0.5
    cp[-1] *= 0.5
    return ks, cp
