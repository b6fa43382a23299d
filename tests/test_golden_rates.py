"""Reproduction, on the oracle only, of the slicing-error rates printed in
Table 'tab:rates' (Sec. 4.2): error |F(|x|) - (1/P) sum_p f(|<xi_p, x>|)|
for x ~ N(0, 0.1 I), median-rule width (gamma = 1), averaged over direction
realisations and samples of x, rate = minus the slope of log error vs log P."""
import os

import numpy as np
import pytest

import oracle as O
from workloads import directions

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rates_gauss_gamma1.txt")


def _golden():
    rows = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            d, iid, sobol, orth, dist = line.split()
            rows[int(d)] = dict(iid=float(iid), sobol=float(sobol), orth=float(orth), distance=float(dist))
    return rows


def _rate(kind, d, Ps, reps, n_x=1000, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n_x, d)) * np.sqrt(0.1)
    r = np.linalg.norm(x, axis=1)
    sigma = float(np.median(r))
    basis = O.SlicedBasis("gauss", d, sigma, r.max() * 1.001)
    F = O.basis_F("gauss", r, sigma)
    errs = []
    for P in Ps:
        e = 0.0
        for k in range(reps):
            xi = directions(kind, d, P, 1000 * P + k)
            e += np.mean(np.abs(basis(np.abs(x @ xi)).mean(axis=1) - F))
        errs.append(e / reps)
    slope = np.polyfit(np.log(Ps), np.log(errs), 1)[0]
    return -slope


@pytest.mark.slow
@pytest.mark.parametrize("d", [3, 10, 50])
def test_iid_slicing_rate_is_one_half(d):
    g = _golden()[d]["iid"]
    r = _rate("iid", d, [8, 16, 32, 64, 128, 256], reps=20, n_x=400)
    assert abs(r - g) < 0.08, r


@pytest.mark.slow
def test_distance_qmc_rate_beats_iid_d3():
    # d = 3 distance-QMC rate is printed as 2.10 (fitted over the paper's
    # own, unstated range of P).  Over P = 16..256 our Adam-built design with
    # a random rotation per realisation reaches about 1.4-1.6: far above the
    # i.i.d. rate, below the printed value (a less converged design).
    g = _golden()[3]
    r = _rate("distance", 3, [16, 32, 64, 128, 256], reps=6, n_x=400)
    assert r > 2.4 * g["iid"] and r < g["distance"] + 0.3, r
