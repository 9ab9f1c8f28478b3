"""Pins of the oracle's random numbers and radiation functions.

Each check uses something other than the oracle itself: published known-answer
vectors, an independent library evaluation of the definition, textbook series
and Mellin-transform identities.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate, special, stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(oracle):
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert oracle.philox4x32_10(ctr, key) == out


def test_box_muller_normals_are_standard(oracle):
    # 6 x 20000 draws: moments and Kolmogorov-Smirnov against N(0, 1)
    n = np.stack([oracle.normals(7, 3, i) for i in range(20000)])
    for c in range(6):
        col = n[:, c]
        assert abs(col.mean()) < 4.0 / math.sqrt(len(col))
        assert abs(col.var() - 1.0) < 4.0 * math.sqrt(2.0 / len(col))
        assert stats.kstest(col, "norm").pvalue > 1e-4
    # pairs are uncorrelated
    c = np.corrcoef(n.T)
    assert np.max(np.abs(c - np.eye(6))) < 4.0 / math.sqrt(len(n))


def test_normals_depend_on_counter_and_key(oracle):
    a = oracle.normals(1, 0, 5)
    assert np.array_equal(a, oracle.normals(1, 0, 5))
    assert not np.allclose(a, oracle.normals(1, 0, 6))
    assert not np.allclose(a, oracle.normals(1, 1, 5))
    assert not np.allclose(a, oracle.normals(2, 0, 5))


# ---- radiation functions ------------------------------------------------------

def _definition_gh(chi):
    """g and h from the defining xi integrals with the nested Int K_1/3 term,
    using scipy's Bessel functions (no integration by parts, no y map)."""
    def intk13(y):
        return integrate.quad(lambda s: special.kv(1 / 3, s), y, np.inf, limit=200,
                              epsabs=0, epsrel=1e-13)[0]

    def bracket(xi):
        y = 2 * xi / (3 * chi * (1 - xi))
        return (1 - xi + 1 / (1 - xi)) * special.kv(2 / 3, y) - intk13(y)

    pts = [3 * chi / (2 + 3 * chi) * t for t in (0.1, 1.0, 3.0)]
    ig = integrate.quad(lambda x: x * bracket(x), 0, 1, points=pts, limit=400,
                        epsabs=0, epsrel=1e-11)[0]
    ih = integrate.quad(lambda x: x * x * bracket(x), 0, 1, points=pts, limit=400,
                        epsabs=0, epsrel=1e-11)[0]
    return (math.sqrt(3) / (2 * math.pi * chi ** 2) * ig,
            24 / (55 * math.pi * chi ** 3) * ih)


@pytest.mark.parametrize("chi", [0.003, 0.1, 1.0, 7.0])
def test_gh_match_definition(oracle, chi):
    g_ref, h_ref = _definition_gh(chi)
    g, h = oracle.gh_quadrature(chi)
    assert abs(g - g_ref) <= 1e-11 * g_ref
    assert abs(h - h_ref) <= 1e-11 * h_ref


def test_gh_classical_normalisation_mellin():
    # Mellin moments of K_nu fix the classical power (2/3 alpha c/lambdabar chi^2)
    # and the classical second moment (55/(24 sqrt3)): integrate the small-chi
    # limit of the bracket, 2 K_2/3(y) - Int_y K_1/3, against y and y^2.
    def mellin(m, nu):
        return 2 ** (m - 2) * special.gamma((m - nu) / 2) * special.gamma((m + nu) / 2)

    def mom(n):
        # Int y^n [2 K23 - IntK13] dy, with Int y^n IntK13 = Int y^(n+1)/(n+1) K13
        return 2 * mellin(n + 1, 2 / 3) - mellin(n + 2, 1 / 3) / (n + 1)

    # numerically, independent of the closed form
    def num(n):
        f = lambda y: y ** n * (2 * special.kv(2 / 3, y) - integrate.quad(
            lambda s: special.kv(1 / 3, s), y, np.inf, epsrel=1e-12)[0])
        return integrate.quad(f, 0, np.inf, limit=200, epsrel=1e-10)[0]

    assert abs(mom(1) - 8 * math.pi / (9 * math.sqrt(3))) < 1e-12
    assert abs(mom(2) - 55 * math.pi / 81) < 1e-12
    assert abs(num(1) - mom(1)) < 1e-8 * mom(1)
    # g(0) = sqrt3/(2 pi) (3/2)^2 mom(1) = 1 ;  h(0) = 24/(55 pi) (3/2)^3 mom(2) = 1
    assert abs(math.sqrt(3) / (2 * math.pi) * 2.25 * mom(1) - 1) < 1e-13
    assert abs(24 / (55 * math.pi) * 3.375 * mom(2) - 1) < 1e-13


def _series():
    vals = {}
    with open(os.path.join(GOLDEN, "radiation_small_chi.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            vals[k] = float(v)
    return vals


def test_gh_small_chi_series(oracle):
    s = _series()
    assert abs(s["g1"] + 55 * math.sqrt(3) / 16) < 1e-14
    for chi in (1e-5, 3e-5, 1e-4):
        g, h = oracle.gh_quadrature(chi)
        # next terms: about -5e2 chi^3 for g (an asymptotic series with growing
        # coefficients) and about 2e2 chi^2 for h
        assert abs(g - (1 + s["g1"] * chi + s["g2"] * chi ** 2)) < 800 * chi ** 3 + 1e-13
        assert abs(h - (1 + s["h1"] * chi)) < 400 * chi ** 2
    # second-order coefficient of g, read off the quadrature
    chi = 2e-4
    g, _ = oracle.gh_quadrature(chi)
    assert abs((g - 1 - s["g1"] * chi) / chi ** 2 - 48.0) < 0.5


def test_radiation_table_matches_quadrature_and_derivatives(oracle):
    rng = np.random.default_rng(11)
    chis = np.exp(rng.uniform(np.log(2e-6), np.log(500.0), 60))
    for chi in chis:
        g, G1, G2, h = oracle.radiation(chi)
        gq, hq = oracle.gh_quadrature(chi)
        assert abs(g - gq) <= 2e-11 * gq
        assert abs(h - hq) <= 3e-10 * hq
        # derivatives against a finite difference of the quadrature itself
        e = 1e-3
        gp, _ = oracle.gh_quadrature(chi * math.exp(e))
        gm, _ = oracle.gh_quadrature(chi * math.exp(-e))
        d1 = (gp - gm) / (2 * e)           # dg/du = chi g'
        d2 = (gp - 2 * gq + gm) / (e * e)  # d2g/du2 = chi g' + chi^2 g''
        assert abs(G1 - d1) <= 1e-6 * abs(gq) + 1e-9
        assert abs(G2 - (d2 - d1)) <= 1e-5 * abs(gq) + 1e-8
    # below the table: series
    g, G1, G2, h = oracle.radiation(1e-7)
    assert abs(g - (1 - 5.953924651018015e-7)) < 1e-12
    assert abs(G1 + 5.953924651018015e-7) < 1e-12


def test_radiation_physical_bounds(oracle):
    chis = np.exp(np.linspace(np.log(1e-4), np.log(100.0), 200))
    gs = np.array([oracle.radiation(c)[0] for c in chis])
    hs = np.array([oracle.radiation(c)[3] for c in chis])
    assert np.all(gs < 1) and np.all(gs > 0) and np.all(np.diff(gs) < 0)
    assert np.all(hs < 1) and np.all(hs > 0) and np.all(np.diff(hs) < 0)
    # large chi: quantum power grows as chi^(2/3), so g ~ chi^(-4/3); the
    # local slope approaches it with corrections falling like chi^(-2/3)
    dev = []
    for c in (100.0, 200.0, 400.0):
        g1, g2 = oracle.radiation(c)[0], oracle.radiation(2 * c)[0]
        dev.append(math.log(g2 / g1) / math.log(2.0) + 4 / 3)
    assert all(d > 0 for d in dev) and dev[-1] < 0.02
    assert abs(dev[1] / dev[0] - 2 ** (-2 / 3)) < 0.05
    assert abs(dev[2] / dev[1] - 2 ** (-2 / 3)) < 0.05
    assert oracle.radiation(2e3)[0] != oracle.radiation(2e3)[0]  # NaN above range
