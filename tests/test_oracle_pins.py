"""Pins of the FP64 oracle against facts fixed by the paper and by
mathematics, not by the oracle itself: closed forms, textbook special cases,
exact identities, statistical properties and values printed in the paper."""
import os
from math import gamma, lgamma, pi, sqrt, erf, exp

import numpy as np
import pytest
from scipy.special import roots_jacobi, roots_legendre

import oracle as O
from workloads import directions, random_rotation

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


# ---------------------------------------------------------------------------
# the 1-D basis function f
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kernel", ["gauss", "laplace"])
def test_f_d3_equals_derivative_of_tF(kernel):
    # At d = 3 eq. (integral_transform) reads F(t) = (1/t) int_0^t f, so
    # f = (t F)'.  Gauss: (1 - t^2/s^2) e^{-t^2/2s^2}; Laplace: (1 - a t) e^{-a t}.
    s = 0.7
    t = np.linspace(0.0, 6.0, 61)
    b = O.SlicedBasis(kernel, 3, s, 6.0)
    if kernel == "gauss":
        ref = (1 - t**2 / s**2) * np.exp(-t**2 / (2 * s**2))
    else:
        ref = (1 - t / s) * np.exp(-t / s)
    assert np.abs(b(t) - ref).max() < 1e-12


def test_energy_constant_d3_and_limits():
    # d = 3: f = (t F)' = (-t^2)' = -2t, so c_3 = 2; d = 1: f = F, c_1 = 1.
    assert abs(O.energy_cd(3) - 2.0) < 1e-14
    assert abs(O.energy_cd(1) - 1.0) < 1e-14
    # c_d ~ sqrt(pi d / 2) for large d (Gamma ratio asymptotics, DLMF 5.11.12)
    assert abs(O.energy_cd(784) / sqrt(pi * 784 / 2) - 1) < 1e-3


@pytest.mark.parametrize("kernel", ["gauss", "laplace", "energy"])
@pytest.mark.parametrize("d", [3, 10, 50])
def test_riemann_liouville_transform_recovers_F(kernel, d):
    # eq. (integral_transform): F(t) = 2 G(d/2)/(sqrt(pi) G((d-1)/2))
    #                                  int_0^1 f(ts) (1-s^2)^{(d-3)/2} ds
    scale = 1.0
    t_max = 4.0
    b = O.SlicedBasis(kernel, d, scale, t_max)
    a = (d - 3) / 2.0
    u, wq = roots_jacobi(80, a, 0.0)            # weight (1-u)^a on [-1, 1]
    sq = (1 + u) / 2                             # s in [0, 1]
    const = 2 * exp(lgamma(d / 2) - lgamma((d - 1) / 2)) / sqrt(pi)
    for t in [0.1, 0.5, 1.3, 2.7, 4.0]:
        integrand = b(t * sq) * (1 + sq) ** a / 2 ** a * 0.5
        F = const * np.dot(wq, integrand)
        ref = O.basis_F(kernel, t, scale)
        assert abs(F - ref) < 1e-9 * max(1.0, abs(ref)), (t, F, ref)


def test_chebyshev_table_matches_direct_evaluation():
    for kernel, d in [("gauss", 50), ("laplace", 50), ("laplace", 10)]:
        b = O.SlicedBasis(kernel, d, 1.0, 3.0)
        for t in [0.0, 0.37, 1.41, 2.99]:
            assert abs(b(t) - b.mp_value(t)) < 1e-10


def test_f_at_zero_is_F_at_zero():
    for kernel in ["gauss", "laplace"]:
        for d in [2, 3, 10, 50, 784]:
            b = O.SlicedBasis(kernel, d, 1.0, 1.0, nodes=40)
            assert abs(b(0.0) - 1.0) < 1e-11


# ---------------------------------------------------------------------------
# the sliced Fourier transform and the Fourier coefficients
# ---------------------------------------------------------------------------

def test_sliced_ft_d1_is_textbook_transform():
    w = np.linspace(0, 3, 31)
    s, al = 0.8, 1.7
    g = np.sqrt(2 * pi) * s * np.exp(-2 * pi**2 * s**2 * w**2)
    lap = 2 * al / (al**2 + 4 * pi**2 * w**2)
    assert np.abs(O.sliced_ft("gauss", w, 1, s) - g).max() < 1e-14
    assert np.abs(O.sliced_ft("laplace", w, 1, 1 / al) - lap).max() < 1e-14


def _numeric_ft(fun, omega, t_end, panels=400, order=20):
    x, wq = roots_legendre(order)
    edges = np.linspace(0.0, t_end, panels + 1)
    tot = np.zeros_like(omega)
    for a, b in zip(edges[:-1], edges[1:]):
        t = 0.5 * (b - a) * x + 0.5 * (a + b)
        tot += 0.5 * (b - a) * (np.cos(2 * pi * np.outer(omega, t)) @ (wq * fun(t)))
    return 2 * tot


@pytest.mark.parametrize("kernel,d", [("gauss", 3), ("gauss", 10), ("laplace", 3), ("laplace", 10)])
def test_sliced_ft_matches_numeric_transform_of_f(kernel, d):
    scale = 1.0
    t_end = 40.0 if kernel == "gauss" else 60.0
    if kernel == "gauss":
        b = O.SlicedBasis(kernel, d, scale, t_end, nodes=600)
        fun = b
    else:
        b = O.SlicedBasis(kernel, d, scale, 12.0, nodes=400)
        # beyond 12 scales f is below 1e-3 relative; tail handled by cutoff
        fun = lambda t: np.where(t <= 12.0, b(np.minimum(t, 12.0)), 0.0)
        t_end = 12.0
    omega = np.array([0.05, 0.1, 0.2, 0.35])
    num = _numeric_ft(fun, omega, t_end)
    ana = O.sliced_ft(kernel, omega, d, scale)
    tol = 1e-9 if kernel == "gauss" else 2e-3
    assert np.abs(num - ana).max() < tol * np.abs(ana).max(), (num, ana)


def test_gauss_d3_sliced_ft_closed_form():
    # f = (1 - t^2/s^2) e^{-t^2/2s^2} has transform sqrt(2 pi) s 4 pi^2 s^2 w^2 e^{-2 pi^2 s^2 w^2}
    s = 1.3
    w = np.linspace(0, 1.5, 16)
    ref = np.sqrt(2 * pi) * s * 4 * pi**2 * s**2 * w**2 * np.exp(-2 * pi**2 * s**2 * w**2)
    assert np.abs(O.sliced_ft("gauss", w, 3, s) - ref).max() < 1e-13


@pytest.mark.parametrize("kernel,d,n_ft", [("gauss", 3, 128), ("gauss", 50, 128),
                                           ("laplace", 3, 1024), ("laplace", 50, 1024)])
def test_fourier_series_reconstructs_periodised_kernel(kernel, d, n_ft):
    # Poisson summation (App. I, Step 2): the Fourier series with coefficients
    # F_1[g~](k), g~(x) = f(|x|/tau), is the 1-periodisation sum_l g~(x + l);
    # truncation to |k| <= K is the only other error.  Gauss: spectrally
    # small.  Laplace: f(|t|) has a kink at 0, its transform decays like
    # c_d alpha / (2 pi^2 w^2), so the discarded tail is at most
    # c_d alpha / (pi^2 tau K), attained at x = 0.
    scale, R, T = 1.0, 3.0, {"gauss": 0.3, "laplace": 0.1}[kernel]
    tau = O.rescale_tau(kernel, R, scale, T)
    K = n_ft // 2
    tol = 1e-12 if kernel == "gauss" else 1.05 * O.energy_cd(d) / scale / (pi**2 * tau * K)
    c = O.fourier_coefficients(kernel, d, scale, tau, n_ft)
    ks, cp = O.truncated_coefficients(c)
    x = np.linspace(-tau * R, tau * R, 41)
    series = (np.exp(2j * pi * np.outer(x, ks)) @ cp).real
    L = 3
    b = O.SlicedBasis(kernel, d, scale, (L + 0.5) / tau, nodes=1200)
    ref = sum(b(np.abs(x + l) / tau) for l in range(-L, L + 1))
    err = np.abs(series - ref)
    assert abs(cp.sum() - sum(b(np.array([l / tau]))[0] for l in range(-L, L + 1))) < tol
    assert err.max() < tol
    if kernel == "laplace":
        assert err.max() > 0.5 * tol                       # the bound is attained at 0
        assert err[np.abs(x) > 0.3 * tau * R].max() < 0.05 * tol
    # and g~ itself is reproduced up to the alias term, largest at |x| = T
    alias = max(abs(b(np.array([(1 - T) / tau]))[0]), 1e-15)
    assert np.abs(series - b(np.abs(x) / tau)).max() < tol + 2.5 * alias


def test_energy_coefficients_triangle_wave():
    # the periodic extension equals -(c_d/tau)|x| on [-1/2, 1/2); the truncated
    # series converges like 1/K away from the kinks at 0 and 1/2.
    d, tau, n_ft = 10, 0.2, 1024
    c = O.fourier_coefficients("energy", d, 1.0, tau, n_ft)
    ks, cp = O.truncated_coefficients(c)
    x = np.linspace(-0.45, 0.45, 37)
    series = (np.exp(2j * pi * np.outer(x, ks)) @ cp).real
    ref = -O.energy_cd(d) / tau * np.abs(x)
    K = n_ft // 2
    amp = O.energy_cd(d) / tau
    err = np.abs(series - ref)
    assert err.max() < 1.2 * amp / (pi**2 * K) * 2      # worst case at the kink x = 0
    assert err[np.abs(x) > 0.05].max() < 1e-5 * amp


# ---------------------------------------------------------------------------
# Matern kernels (Table 'tab:kernels', Matern row; App. I)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kernel,nu", [("matern32", 1.5), ("matern52", 2.5), ("matern72", 3.5)])
def test_matern_closed_form_is_the_bessel_form(kernel, nu):
    # column 2: 2^{1-nu}/Gamma(nu) z^nu K_nu(z), z = sqrt(2 nu) r / beta,
    # evaluated with the modified Bessel function itself
    from scipy.special import kv
    beta = 1.3
    r = np.array([1e-3, 0.05, 0.4, 1.0, 2.5, 6.0, 15.0])
    z = sqrt(2 * nu) * r / beta
    ref = 2 ** (1 - nu) / gamma(nu) * z ** nu * kv(nu, z)
    assert np.abs(O.basis_F(kernel, r, beta) - ref).max() < 1e-14
    assert O.basis_F(kernel, 0.0, beta) == 1.0


@pytest.mark.parametrize("d", [1, 3, 10, 50])
def test_matern_half_transform_is_laplace(d):
    # nu = 1/2 is the Laplace kernel with alpha = 1/beta (Sec. 3 remark); the
    # Matern column-3 transform must then equal the Laplace one
    from oracle.kernels import log_ft_matern, _log_ft_d
    w = np.array([0.0, 1e-3, 0.05, 0.3, 2.0, 9.0])
    assert np.abs(log_ft_matern(w, d, 1.7, 0.5) - _log_ft_d("laplace", w, d, 1.7)).max() < 1e-12


@pytest.mark.parametrize("kernel", ["matern32", "matern52", "matern72"])
def test_matern_d1_transform_is_numeric_transform_of_F(kernel):
    # d = 1: slicing is the identity, f = F, so the sliced transform must be
    # the plain 1-D Fourier transform of F(|x|)
    from scipy.integrate import quad
    beta = 1.3
    for w in [0.0, 0.02, 0.1, 0.25, 0.6]:
        g = lambda x: float(O.basis_F(kernel, x, beta))
        if w == 0.0:
            ref = 2 * quad(g, 0, np.inf, epsabs=1e-13)[0]
        else:
            ref = 2 * quad(g, 0, np.inf, weight="cos", wvar=2 * pi * w)[0]
        assert float(O.sliced_ft(kernel, w, 1, beta)) == pytest.approx(ref, rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("kernel", ["matern32", "matern52", "matern72"])
def test_matern_d3_transform_is_numeric_transform_of_tF_derivative(kernel):
    # d = 3: eq. integral_transform gives f = (tF)', whose 1-D transform is
    # the sliced transform the coefficients are built from
    from scipy.integrate import quad
    beta = 0.8
    g = lambda x: float(O.basis_F(kernel, x, beta) + x * O.basis_dF(kernel, x, beta))
    for w in [0.03, 0.15, 0.4, 1.0]:
        ref = 2 * quad(g, 0, np.inf, weight="cos", wvar=2 * pi * w)[0]
        assert float(O.sliced_ft(kernel, w, 3, beta)) == pytest.approx(ref, rel=1e-8, abs=1e-12)
    t = np.linspace(0.0, 5.0, 11)
    b = O.SlicedBasis(kernel, 3, beta, 5.0)
    assert np.abs(b(t) - np.array([g(v) for v in t])).max() < 1e-14


@pytest.mark.parametrize("kernel", ["matern32", "matern72"])
@pytest.mark.parametrize("d", [3, 50])
def test_matern_coefficients_sum_to_F0(kernel, d):
    # sum_k c'_k = g~(0) = f(0) = F(0) = 1 up to truncation and periodisation
    # at the paper's parameters (T = 0.2, g_max = 5 beta, N_ft = 512)
    scale, R = 1.0, 3.0
    tau = O.rescale_tau(kernel, R, scale, 0.2)
    _, cp = O.truncated_coefficients(O.fourier_coefficients(kernel, d, scale, tau, 512))
    assert cp.sum() == pytest.approx(1.0, abs=2e-3)


# ---------------------------------------------------------------------------
# O1: the direct sum
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kernel", ["gauss", "laplace", "energy", "matern32", "matern72"])
def test_direct_single_coincident_point(kernel):
    x = np.array([[0.3, -1.2, 2.0]])
    s = O.kernel_sum_direct(kernel, x, x, np.array([1.7]), 0.9)
    assert s[0] == pytest.approx(1.7 * O.basis_F(kernel, 0.0, 0.9), abs=1e-15)


def test_direct_gaussian_convolution_identity():
    # x_n ~ N(0, a^2 I), w = 1/N:  E s(y) = (s^2/(s^2+a^2))^{d/2} e^{-|y|^2/(2(s^2+a^2))}
    rng = np.random.default_rng(7)
    d, N, a, s = 5, 200000, 0.8, 1.1
    x = a * rng.standard_normal((N, d))
    y = rng.standard_normal((6, d)) * 0.7
    got = O.kernel_sum_direct("gauss", x, y, np.full(N, 1.0 / N), s)
    ref = (s**2 / (s**2 + a**2)) ** (d / 2) * np.exp(-(y**2).sum(1) / (2 * (s**2 + a**2)))
    sd = np.sqrt(ref * (1 - ref) / N) + 1e-12       # values lie in [0, 1]
    assert np.all(np.abs(got - ref) < 5 * sd + 1e-4)


def test_direct_energy_and_laplace_1d_integrals():
    # midpoint rule on [0,1]: (1/N) sum F(|x_n - y|) -> int_0^1 F(|x - y|) dx
    N = 20000
    x = ((np.arange(N) + 0.5) / N)[:, None]
    y = np.array([[0.0], [0.3], [0.77]])
    w = np.full(N, 1.0 / N)
    yy = y[:, 0]
    e = O.kernel_sum_direct("energy", x, y, w, 1.0)
    assert np.abs(e + (yy**2 + (1 - yy) ** 2) / 2).max() < 1e-8
    al = 2.5
    lap = O.kernel_sum_direct("laplace", x, y, w, 1 / al)
    ref = (2 - np.exp(-al * yy) - np.exp(-al * (1 - yy))) / al
    assert np.abs(lap - ref).max() < 1e-8


@pytest.mark.parametrize("kernel", ["gauss", "laplace", "energy", "matern52"])
@pytest.mark.parametrize("d", [1, 3, 50, 784])
def test_direct_gram_form_equals_explicit_differences(kernel, d):
    """The Gram-identity O1 against the explicit-difference O1 (itself pinned
    above), on image-like and Gaussian points; a target chunk smaller than M
    exercises the blocking; coincident points (sources = targets) leave
    r ~ 1e-8 |x| instead of 0, bounded against the terms' size."""
    rng = np.random.default_rng(d)
    x = np.where(rng.random((300, d)) < 0.8, 0.0, rng.random((300, d))) if d > 50 else \
        rng.standard_normal((300, d))
    y = rng.standard_normal((70, d)) * 0.5 + 0.2
    w = rng.standard_normal(300)
    sc = 0.7 * np.sqrt(d)
    ref = O.kernel_sum_direct(kernel, x, y, w, sc)
    got = O.kernel_sum_direct_gram(kernel, x, y, w, sc, budget=300 * 16)
    s_abs = O.kernel_sum_direct(kernel, x, y, np.abs(w), sc)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(s_abs).max()
    same = O.kernel_sum_direct_gram(kernel, x, x, w, sc)
    ref_same = O.kernel_sum_direct(kernel, x, x, w, sc)
    s_abs = O.kernel_sum_direct(kernel, x, x, np.abs(w), sc)
    assert np.abs(same - ref_same).max() < 1e-6 * np.abs(s_abs).max()


def test_energy_distance_of_identical_sets_is_zero():
    rng = np.random.default_rng(3)
    X = rng.random((40, 7))
    src = np.concatenate([X, X])
    w = np.concatenate([np.full(40, 1 / 40), np.full(40, -1 / 40)])
    Y = rng.random((25, 7))
    assert np.abs(O.kernel_sum_direct("energy", src, Y, w, 1.0)).max() < 1e-14
    xi = directions("distance", 7, 16, 5)
    tau = 0.45 / 3.0
    s3 = O.kernel_sum_fourier("energy", src, Y, w, xi, 1.0, 256, tau)
    assert np.abs(s3).max() < 1e-12


@pytest.mark.parametrize("kernel", ["gauss", "laplace", "energy"])
def test_symmetry_for_unit_weights(kernel):
    # for w = 1: 1^T s(X -> Y) = sum_{n,m} K(x_n, y_m) = 1^T s(Y -> X)
    rng = np.random.default_rng(11)
    X, Y = rng.standard_normal((30, 4)), rng.standard_normal((20, 4)) + 0.5
    a = O.kernel_sum_direct(kernel, X, Y, np.ones(30), 1.2).sum()
    b = O.kernel_sum_direct(kernel, Y, X, np.ones(20), 1.2).sum()
    assert a == pytest.approx(b, rel=1e-13)
    xi = directions("iid", 4, 9, 2)
    R = np.linalg.norm(X, axis=1).max() + np.linalg.norm(Y, axis=1).max()
    T = {"gauss": 0.3, "laplace": 0.1, "energy": 0.45}[kernel]
    tau = O.rescale_tau(kernel, R, 1.2, T)
    a3 = O.kernel_sum_fourier(kernel, X, Y, np.ones(30), xi, 1.2, 256, tau).sum()
    b3 = O.kernel_sum_fourier(kernel, Y, X, np.ones(20), xi, 1.2, 256, tau).sum()
    assert a3 == pytest.approx(b3, rel=1e-12, abs=1e-12)


# ---------------------------------------------------------------------------
# O2 / O3: special cases, convergence, unbiasedness, variance
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kernel", ["gauss", "laplace", "energy"])
def test_d1_slicing_is_exact(kernel):
    # d = 1: xi = +-1, f = F, so the sliced sum equals the direct sum, and
    # Fourier slicing is textbook 1-D fast Fourier summation.
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, (50, 1))
    y = rng.uniform(-1, 1, (40, 1))
    w = rng.standard_normal(50)
    xi = np.array([[1.0, -1.0]])
    s1 = O.kernel_sum_direct(kernel, x, y, w, 0.4)
    s2 = O.kernel_sum_sliced(kernel, x, y, w, xi, 0.4)
    assert rel(s2, s1) < 1e-13
    R = np.abs(x).max() + np.abs(y).max()
    T = {"gauss": 0.3, "laplace": 0.1, "energy": 0.45}[kernel]
    n_ft = {"gauss": 128, "laplace": 4096, "energy": 4096}[kernel]
    tol = {"gauss": 1e-12, "laplace": 1e-3, "energy": 1e-3}[kernel]
    tau = O.rescale_tau(kernel, R, 0.4, T)
    s3 = O.kernel_sum_fourier(kernel, x, y, w, xi, 0.4, n_ft, tau)
    assert rel(s3, s1) < tol


def test_fourier_slicing_converges_to_sliced_sum():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((40, 3))
    y = rng.standard_normal((30, 3))
    w = rng.standard_normal(40)
    xi = directions("distance", 3, 12, 3)
    R = np.linalg.norm(x, axis=1).max() + np.linalg.norm(y, axis=1).max()
    s2g = O.kernel_sum_sliced("gauss", x, y, w, xi, 1.0)
    tau = O.rescale_tau("gauss", R, 1.0, 0.3)
    assert rel(O.kernel_sum_fourier("gauss", x, y, w, xi, 1.0, 128, tau), s2g) < 1e-12
    s2l = O.kernel_sum_sliced("laplace", x, y, w, xi, 1.0)
    tau = O.rescale_tau("laplace", R, 1.0, 0.1)
    errs = [rel(O.kernel_sum_fourier("laplace", x, y, w, xi, 1.0, n, tau), s2l)
            for n in (128, 512, 2048)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 2e-3


@pytest.mark.parametrize("kernel,d", [("gauss", 3), ("laplace", 5), ("energy", 10)])
def test_randomly_rotated_qmc_estimator_is_unbiased(kernel, d):
    # App. E: for A ~ U(O(d)), E_A of the slicing estimate with directions A xi
    # equals the exact kernel sum.
    rng = np.random.default_rng(20 + d)
    x = rng.standard_normal((12, d))
    y = rng.standard_normal((5, d))
    w = rng.random(12)
    xi0 = directions("distance", d, 4, 9, rotate=False)
    exact = O.kernel_sum_direct(kernel, x, y, w, 1.5)
    R = np.linalg.norm(x, axis=1).max() + np.linalg.norm(y, axis=1).max()
    basis = O.SlicedBasis(kernel, d, 1.5, R)
    reps = np.array([O.kernel_sum_sliced(kernel, x, y, w, random_rotation(d, rng) @ xi0, 1.5, basis)
                     for _ in range(400)])
    mean, se = reps.mean(0), reps.std(0, ddof=1) / np.sqrt(len(reps))
    assert np.all(np.abs(mean - exact) < 4.5 * se + 1e-12), (mean, exact, se)


def _variance_by_quadrature(kernel, d, r, scale):
    # <xi, x> = r u with density G(d/2)/(sqrt(pi) G((d-1)/2)) (1-u^2)^{(d-3)/2}
    # on [-1, 1] (proof of Thm 1 ii); V = E f(r|u|)^2 - F(r)^2.
    b = O.SlicedBasis(kernel, d, scale, r * 1.0001)
    a = (d - 3) / 2.0
    u, wq = roots_jacobi(120, a, 0.0)          # on [0,1] via u = (1+v)/2, even integrand
    uu = (1 + u) / 2
    const = exp(lgamma(d / 2) - lgamma((d - 1) / 2)) / sqrt(pi)
    e2 = 2 * const * np.dot(wq, b(r * uu) ** 2 * (1 + uu) ** a / 2 ** a * 0.5)
    return e2 - O.basis_F(kernel, r, scale) ** 2


@pytest.mark.parametrize("d", [3, 10, 50, 784])
def test_riesz_variance_matches_theorem1(d):
    # Thm 1 ii) with r = 1: V = (sqrt(pi) G(3/2) G((d+1)/2)^2 / (G(1)^2 G(d/2) G(1+d/2)) - 1) F^2
    r = 1.7
    V = _variance_by_quadrature("energy", d, r, 1.0)
    ratio = exp(0.5 * np.log(pi) + lgamma(1.5) + 2 * lgamma((d + 1) / 2) - lgamma(d / 2) - lgamma(1 + d / 2)) - 1
    assert V == pytest.approx(ratio * r * r, rel=1e-9)


def test_laplace_variance_d3_matches_theorem1():
    # Thm 1 iv): V_3 = (1/(4 a|x|)) (1 - (2(a|x|)^2 + 2 a|x| + 1) F^2)
    for ax in [0.2, 1.0, 3.5]:
        V = _variance_by_quadrature("laplace", 3, ax, 1.0)
        F = exp(-ax)
        ref = (1 - (2 * ax**2 + 2 * ax + 1) * F**2) / (4 * ax)
        assert V == pytest.approx(ref, rel=1e-9)


def test_positive_definite_variance_bound():
    # Thm 1 i): V <= F(0)^2 - F(|x|)^2 for positive definite kernels
    for kernel in ["gauss", "laplace"]:
        for d in [3, 10]:
            for r in [0.3, 1.0, 2.5]:
                V = _variance_by_quadrature(kernel, d, r, 1.0)
                assert 0 <= V <= 1 - O.basis_F(kernel, r, 1.0) ** 2 + 1e-12


def test_iid_slicing_mse_is_variance_over_P():
    # Bienayme: E[(1/P sum f - F)^2] = V/P for i.i.d. directions
    rng = np.random.default_rng(5)
    d, P, reps, r = 10, 8, 4000, 1.3
    x = np.zeros(d); x[0] = r
    b = O.SlicedBasis("laplace", d, 1.0, r * 1.001)
    est = np.array([b(np.abs(x @ directions("iid", d, P, int(s)))).mean()
                    for s in rng.integers(0, 2**31, reps)])
    mse = np.mean((est - np.exp(-r)) ** 2)
    V = _variance_by_quadrature("laplace", d, r, 1.0)
    assert mse == pytest.approx(V / P, rel=0.1)


def test_moment_identity_for_iid_directions():
    # eq. (Exi^r): E|<xi,x>|^{2r} = |x|^{2r} G(r+1/2) G(d/2) / (sqrt(pi) G(r+d/2))
    d, r = 7, 1.5
    xi = directions("iid", d, 400000, 8)
    x = np.ones(d) / np.sqrt(d)
    mc = np.mean(np.abs(x @ xi) ** (2 * r))
    ref = gamma(r + 0.5) * gamma(d / 2) / (sqrt(pi) * gamma(r + d / 2))
    assert mc == pytest.approx(ref, rel=1e-2)


def test_orthonormal_directions_minimise_symmetric_energy():
    # App. H: for P <= d the pairwise term -(|a-b|+|a+b|)^2 = -4 - 2 sqrt(4 - 4<a,b>^2)
    # is minimal iff <a,b> = 0.
    xi = directions("distance", 12, 12, 1)
    g = xi.T @ xi
    assert np.abs(g - np.eye(12)).max() < 1e-12


# ---------------------------------------------------------------------------
# gradients
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kernel", ["gauss", "laplace", "energy", "matern32", "matern72"])
def test_direct_gradient_matches_finite_differences(kernel):
    rng = np.random.default_rng(4)
    x = rng.standard_normal((25, 3))
    y = rng.standard_normal((6, 3))
    w = rng.standard_normal(25)
    g = O.grad_y_direct(kernel, x, y, w, 1.1)
    h = 1e-6
    for m in range(6):
        for i in range(3):
            yp, ym = y.copy(), y.copy()
            yp[m, i] += h
            ym[m, i] -= h
            fd = (O.kernel_sum_direct(kernel, x, yp, w, 1.1)[m] - O.kernel_sum_direct(kernel, x, ym, w, 1.1)[m]) / (2 * h)
            assert fd == pytest.approx(g[m, i], rel=1e-6, abs=1e-8)


@pytest.mark.parametrize("kernel", ["gauss", "laplace", "energy", "matern52"])
def test_fourier_gradients_match_finite_differences(kernel):
    rng = np.random.default_rng(6)
    x = rng.standard_normal((20, 4))
    y = rng.standard_normal((5, 4))
    w = rng.standard_normal(20)
    xi = directions("iid", 4, 7, 3)
    R = 8.0
    T = {"gauss": 0.3, "laplace": 0.1, "energy": 0.45, "matern52": 0.2}[kernel]
    tau = O.rescale_tau(kernel, R, 1.0, T)
    n_ft = 256
    g = O.grad_y_fourier(kernel, x, y, w, xi, 1.0, n_ft, tau)
    h = 1e-6
    f = lambda yy: O.kernel_sum_fourier(kernel, x, yy, w, xi, 1.0, n_ft, tau)
    for m in range(5):
        for i in range(4):
            yp, ym = y.copy(), y.copy()
            yp[m, i] += h
            ym[m, i] -= h
            fd = (f(yp)[m] - f(ym)[m]) / (2 * h)
            assert fd == pytest.approx(g[m, i], rel=1e-6, abs=1e-7)
    # weights: the map is linear, so the VJP equals the explicit Jacobian
    v = rng.standard_normal(5)
    gw = O.grad_w_fourier(kernel, x, y, v, xi, 1.0, n_ft, tau)
    jac = np.stack([f.__call__(y) * 0 + O.kernel_sum_fourier(kernel, x, y, np.eye(20)[n], xi, 1.0, n_ft, tau)
                    for n in range(20)], axis=1)
    assert np.abs(gw - jac.T @ v).max() < 1e-10 * np.abs(jac).max() * np.abs(v).sum()


@pytest.mark.parametrize("kernel", ["gauss", "energy", "matern32"])
def test_source_gradient_matches_finite_differences_and_transposed_sum(kernel):
    # sum_m v_m s_m differentiated in x_n by central differences of the FP64
    # Fourier sum; and, the sliced Fourier sum being symmetric in sources and
    # targets, w_n times the target derivative of the transposed sum
    rng = np.random.default_rng(9)
    x = rng.standard_normal((12, 3))
    y = rng.standard_normal((7, 3))
    w = rng.standard_normal(12)
    v = rng.standard_normal(7)
    xi = directions("iid", 3, 5, 8)
    T = {"gauss": 0.3, "energy": 0.45, "matern32": 0.2}[kernel]
    tau = O.rescale_tau(kernel, 8.0, 1.0, T)
    n_ft = 256
    g = O.grad_x_fourier(kernel, x, y, w, v, xi, 1.0, n_ft, tau)
    f = lambda xx: v @ O.kernel_sum_fourier(kernel, xx, y, w, xi, 1.0, n_ft, tau)
    h = 1e-6
    for n in range(12):
        for i in range(3):
            xp, xm = x.copy(), x.copy()
            xp[n, i] += h
            xm[n, i] -= h
            assert (f(xp) - f(xm)) / (2 * h) == pytest.approx(g[n, i], rel=1e-6, abs=1e-8)
    gt = O.grad_y_fourier(kernel, y, x, v, xi, 1.0, n_ft, tau) * w[:, None]
    assert np.abs(g - gt).max() < 1e-12 * np.abs(g).max()


def test_golden_parameters_match_workload_defaults():
    from workloads.configs import DEFAULT_T, DEFAULT_NFT
    rows = [l.split() for l in open(os.path.join(GOLDEN, "app_i_parameters.txt")) if l.strip() and not l.startswith("#")]
    for kernel, T, gf, nft in rows:
        assert DEFAULT_T[kernel] == float(T)
        assert DEFAULT_NFT[kernel] == int(nft)


def test_sliced_energy_gradients_match_finite_differences():
    """The exact sliced energy sum is piecewise linear in x, y and w, so a
    central difference with a small step reproduces its derivative away from
    kinks, and at an exact tie (a target on a source, as in an MMD flow)
    gives the symmetric value sign(0) = 0 that the gradient takes there."""
    rng = np.random.default_rng(21)
    N, M, d, P = 14, 11, 4, 6
    x = rng.standard_normal((N, d))
    y = rng.standard_normal((M, d))
    y[3] = x[5]                                   # a coincident pair
    w = rng.standard_normal(N)
    v = rng.standard_normal(M)
    xi = rng.standard_normal((d, P))
    xi /= np.linalg.norm(xi, axis=0)
    gx, gy, gw = O.grad_sliced_energy(x, y, w, v, xi)

    def J(x_, y_, w_):
        return float(v @ O.kernel_sum_sliced("energy", x_, y_, w_, xi, 1.0))

    h = 1e-6
    for (m, i) in [(0, 0), (3, 1), (3, 3), (7, 2)]:
        e = np.zeros_like(y)
        e[m, i] = h
        fd = (J(x, y + e, w) - J(x, y - e, w)) / (2 * h)
        assert abs(fd - gy[m, i]) < 1e-6 * (1 + abs(gy[m, i])), (m, i, fd, gy[m, i])
    for (n, i) in [(0, 0), (5, 2), (9, 3)]:
        e = np.zeros_like(x)
        e[n, i] = h
        fd = (J(x + e, y, w) - J(x - e, y, w)) / (2 * h)
        assert abs(fd - gx[n, i]) < 1e-6 * (1 + abs(gx[n, i])), (n, i, fd, gx[n, i])
    for n in (0, 5, 13):
        e = np.zeros_like(w)
        e[n] = 1.0
        assert J(x, y, w + e) - J(x, y, w) == pytest.approx(gw[n], rel=1e-12, abs=1e-12)
    # the coincident pair contributes nothing to either gradient
    wz = w.copy()
    wz[5] = 0.0
    _, gy0, _ = O.grad_sliced_energy(x, y, wz, v, xi)
    _, gy1, _ = O.grad_sliced_energy(x, y, w, v, xi)
    tie_only = gy1[3] - gy0[3]
    t = (x[5] - y[3]) @ xi
    assert np.all(t == 0.0) and np.allclose(tie_only, 0.0, atol=1e-15)


def test_distance_energy_gradient_and_adam():
    """The distance-energy gradient against central differences; the
    projected Adam iteration keeps unit rows, raises the energy, and for
    P <= d ends at an orthonormal system, the minimiser of App. H."""
    rng = np.random.default_rng(33)
    xi = rng.standard_normal((7, 4))
    xi /= np.linalg.norm(xi, axis=1, keepdims=True)
    g = O.distance_energy_grad(xi)
    h = 1e-6
    for (p, i) in [(0, 0), (3, 2), (6, 3)]:
        e = np.zeros_like(xi)
        e[p, i] = h
        fd = (O.distance_energy(xi + e) - O.distance_energy(xi - e)) / (2 * h) / 2
        assert abs(fd - g[p, i]) < 1e-6 * (1 + abs(g[p, i]))
    out = O.projected_adam(xi, 300, 0.02)
    assert np.allclose(np.linalg.norm(out, axis=1), 1.0, atol=1e-12)
    assert O.distance_energy(out) > O.distance_energy(xi)
    x0 = rng.standard_normal((5, 5))
    orth = O.projected_adam(x0, 2000, 0.05)
    assert np.abs(orth @ orth.T - np.eye(5)).max() < 1e-3


def test_rotate_directions_orientation_and_invariants():
    """App. E rotation: a cyclic coordinate shift q (q[i, i+1] = 1) sends
    coordinate i+1 of each direction to coordinate i (a transposed q would
    shift the other way); an orthogonal q keeps every inner product and so
    the distance energy; a multiple of q gives the same unit rows."""
    rng = np.random.default_rng(71)
    d, P = 6, 9
    xi = rng.standard_normal((P, d))
    xi /= np.linalg.norm(xi, axis=1, keepdims=True)
    shift = np.zeros((d, d))
    for i in range(d):
        shift[i, (i + 1) % d] = 1.0
    out = O.rotate_directions(shift, xi)
    assert np.abs(out - np.roll(xi, -1, axis=1)).max() < 1e-15
    q, r = np.linalg.qr(rng.standard_normal((d, d)))
    q *= np.sign(np.diag(r))
    rot = O.rotate_directions(q, xi)
    assert np.abs(rot @ rot.T - xi @ xi.T).max() < 1e-13
    assert abs(O.distance_energy(rot) - O.distance_energy(xi)) < 1e-12 * O.distance_energy(xi)
    assert np.abs(O.rotate_directions(3.0 * q, xi) - rot).max() < 1e-15
    assert not np.allclose(rot, xi)
