"""CPU-side checks of the C ABI: the library loads, exports every declared
symbol, and its host-only FP64 precompute agrees with the oracle's
independent implementation.  No compute call touches a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_2410_01316_amd as F
from paper_2410_01316_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names += re.findall(r"FASTSUM_API\s+[\w\s\*]+?\b(fastsum_\w+)\s*\(", txt)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(F.LIB_PATH)
    names = _declared()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(L.SIGNATURES), "binding misses a declared entry point"


def test_status_strings():
    lib = L.load()
    assert lib.fastsum_status_string(0) == b"ok"
    assert lib.fastsum_status_string(4) == b"point outside the bound R"
    assert lib.fastsum_status_string(99) == b"unknown status"


@pytest.mark.parametrize("kernel,d,scale,R,n_ft", [
    ("gauss", 3, 1.03, 2.0, 128), ("gauss", 50, 20.4, 45.0, 1024),
    ("laplace", 50, 20.4, 45.0, 1024), ("laplace", 10, 0.7, 3.0, 256),
    ("energy", 784, 1.0, 30.0, 1024), ("energy", 20, 1.0, 10.0, 1024),
    ("matern32", 3, 0.9, 2.5, 512), ("matern32", 50, 20.4, 45.0, 512),
    ("matern52", 10, 1.3, 4.0, 512), ("matern72", 50, 20.4, 45.0, 512)])
def test_host_tables_match_oracle(kernel, d, scale, R, n_ft):
    T = {"gauss": 0.3, "laplace": 0.1, "energy": 0.45,
         "matern32": 0.2, "matern52": 0.2, "matern72": 0.2}[kernel]
    tau, ck, ph = F.host_tables(kernel, d, n_ft, R=R, scale=scale, T=T)
    assert tau == pytest.approx(O.rescale_tau(kernel, R, scale, T), rel=1e-15)
    ref = O.fourier_coefficients(kernel, d, scale, tau, n_ft)
    assert np.abs(ck - ref).max() <= 1e-11 * np.abs(ref).max()
    # the window transform is positive on the kept modes (deconvolution is safe)
    assert np.all(ph[: n_ft // 2 + 1] > 0)


def test_window_transform_close_to_exponential_of_semicircle():
    # the piecewise polynomial interpolates exp(beta(sqrt(1-z^2)-1)); its
    # transform must match the window's own (numerical quadrature) closely
    from scipy.special import roots_legendre
    n_ft, W = 128, 4
    n = 2 * n_ft
    beta = 2.6 * W
    _, _, ph = F.host_tables("gauss", 3, n_ft, R=2.0, scale=1.0, window_w=W)
    z, wq = roots_legendre(400)
    phi = np.exp(beta * (np.sqrt(1 - z**2) - 1))
    k = np.arange(n // 2 + 1)
    ref = (W / (2 * n)) * (np.cos(np.pi * np.outer(k, z) * W / n) @ (wq * phi))
    assert np.abs(ph - ref).max() < 2e-3 * ref[0]


@pytest.mark.parametrize("bad", [dict(n_ft=127), dict(n_ft=8), dict(R=0.0), dict(R=-1.0),
                                 dict(scale=0.0), dict(T=0.6), dict(window_w=5),
                                 dict(oversample=3), dict(n_ft=4096)])
def test_invalid_parameters_rejected(bad):
    kw = dict(kernel="gauss", d=3, n_ft=128, R=2.0, scale=1.0)
    kw.update(bad)
    with pytest.raises(F.FastSumError) as e:
        F.host_tables(**kw)
    assert e.value.status == L.EINVAL


def test_null_arguments_rejected_without_device():
    lib = L.load()
    prm = L.Params(3, 8, 128, 0, 0, 0, 0, 0, 1.0, 0.0, 0.0, 2.0)
    out = ctypes.c_void_p()
    assert lib.fastsum_plan_create(ctypes.byref(prm), None, 10, 10, None, ctypes.byref(out)) == L.EINVAL
    assert lib.fastsum_exec(None, None, 1, None, None, 1, None, None) == L.EINVAL
    assert lib.fastsum_grad(None, None, None, None, None) == L.EINVAL
    assert lib.fastsum_check(None) == L.EINVAL
    assert lib.fastsum_get_info(None, None) == L.EINVAL
    lib.fastsum_destroy(None)


def test_choose_nft_rule():
    # wide kernel relative to the data: the smallest candidate suffices;
    # Laplace keeps a k^-2 tail: the largest candidate is needed at tol 1e-4
    assert F.choose_nft("gauss", 3, 3.0, scale=1.0) == 256
    assert F.choose_nft("laplace", 10, 3.0, scale=1.0) == 1024
    # monotone in the tolerance
    v = [F.choose_nft("gauss", 10, 10.0, scale=0.3, tol=t) for t in (1e-2, 1e-6, 1e-12)]
    assert v == sorted(v)
    lib = L.load()
    bad = L.Params(3, 1, 128, 0, 0, 0, 0, 0, 1.0, 0.0, 0.0, -1.0)
    out = ctypes.c_int32()
    arr = (ctypes.c_int32 * 1)(256)
    assert lib.fastsum_choose_nft(ctypes.byref(bad), arr, 1, 1e-4, ctypes.byref(out)) == L.EINVAL


def test_batch_create_rejects_bad_arguments_without_device():
    lib = L.load()
    common = L.Params(0, 8, 0, 0, 0, 0, 1, 0, 1.0, 0.0, 0.0, 1.0)   # BF16: unsupported
    out = ctypes.c_void_p()
    desc = (L.ProblemDesc * 1)()
    assert lib.fastsum_batch_create(ctypes.byref(common), desc, 1, None, None,
                                    ctypes.byref(out)) == L.EUNSUPPORTED
    common.proj = 0
    assert lib.fastsum_batch_create(ctypes.byref(common), None, 1, None, None,
                                    ctypes.byref(out)) == L.EINVAL
    assert lib.fastsum_batch_exec(None, None, 0, None) == L.EINVAL
    assert lib.fastsum_batch_check(None) == L.EINVAL
    lib.fastsum_batch_destroy(None)


def test_sorted_flag_validation_without_device():
    """The sorted 1-D sums exist for the energy kernel only (with or without
    the adjoint); unknown flag bits are rejected; the QMC construction
    checks its arguments before touching a device."""
    lib = L.load()
    tau = ctypes.c_double()
    ck = np.empty(65)
    ph = np.empty(129)

    def tables(kernel, flags):
        prm = L.Params(3, 8, 128, 0, 0, L.KERNELS[kernel], 0, flags, 1.0, 0.0, 0.0, 2.0)
        return lib.fastsum_host_tables(ctypes.byref(prm), ctypes.byref(tau),
                                       ck.ctypes.data_as(ctypes.c_void_p),
                                       ph.ctypes.data_as(ctypes.c_void_p))

    assert tables("energy", L.FLAG_SORTED) == L.OK
    assert tables("energy", L.FLAG_SORTED | L.FLAG_GRAD) == L.OK
    for kernel in ("gauss", "laplace", "matern32"):
        assert tables(kernel, L.FLAG_SORTED) == L.EINVAL
    assert tables("energy", 8) == L.EINVAL
    buf = ctypes.c_void_p(1)            # never dereferenced: the arguments fail first
    assert lib.fastsum_distance_qmc(65, 10, 1, 0.01, buf, None) == L.EINVAL
    assert lib.fastsum_distance_qmc(3, 0, 1, 0.01, buf, None) == L.EINVAL
    assert lib.fastsum_distance_qmc(3, 10, 1, 0.0, buf, None) == L.EINVAL
    assert lib.fastsum_distance_qmc(3, 10, 1, 0.01, None, None) == L.EINVAL
    assert lib.fastsum_rotate_directions(65, 10, buf, buf, None) == L.EINVAL
    assert lib.fastsum_rotate_directions(0, 10, buf, buf, None) == L.EINVAL
    assert lib.fastsum_rotate_directions(3, 0, buf, buf, None) == L.EINVAL
    assert lib.fastsum_rotate_directions(3, 10, None, buf, None) == L.EINVAL
    assert lib.fastsum_rotate_directions(3, 10, buf, None, None) == L.EINVAL
    assert lib.fastsum_flow_update(0, 3, 0.9, 1.0, buf, buf, buf, None, buf, None) == L.EINVAL
    assert lib.fastsum_flow_update(10, 0, 0.9, 1.0, buf, buf, buf, None, buf, None) == L.EINVAL
    assert lib.fastsum_flow_update(10, 3, float("nan"), 1.0, buf, buf, buf, None, buf,
                                   None) == L.EINVAL
    assert lib.fastsum_flow_update(10, 3, 0.9, 1.0, None, buf, buf, None, buf, None) == L.EINVAL
    assert lib.fastsum_flow_update(10, 3, 0.9, 1.0, buf, buf, buf, None, None, None) == L.EINVAL
