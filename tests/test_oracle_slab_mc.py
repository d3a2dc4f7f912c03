"""Pins of the oracle's bubbly-slab Monte Carlo: without bubbles it must
reproduce the closed-form incoherent slab; index-matched bubbles must be
invisible; energy is conserved per photon; the bubble deviation law must
agree with explicit vector ray tracing through a sphere."""
import math

import numpy as np
import pytest


def test_no_bubbles_matches_analytic_slab(orc):
    """rho_b = 0: R and T within 4 sigma of the closed-form slab (binomial
    sigma for R; T's spread is bounded the same way)."""
    cases = [(1.0, 550.0, 3.0, 1.52, 1e-7, 0.0), (0.5, 450.0, 5.0, 1.55, 1e-5, 0.3),
             (0.2, 700.0, 2.0, 1.50, 3e-6, 0.1), (0.85, 400.0, 4.0, 1.58, 1e-6, 0.05)]
    N = 200000
    for c, lam, d, n, k, tint in cases:
        R, T, A, W = orc.slab_mc(c, lam, d, 0.0, n, k, tint, seed=11, n_photons=N)
        Rr, Tr = orc.slab(c, lam, d, n, k, tint)
        sR = math.sqrt(max(Rr * (1 - Rr), 1e-12) / N)
        sT = math.sqrt(max(Tr * (1 - Tr), 1e-12) / N)
        assert abs(R[0] - Rr) < 4 * sR + 1e-12, (c, R[0], Rr)
        assert abs(T[0] - Tr) < 4 * sT + 1e-12, (c, T[0], Tr)
        assert W[0] < 1e-6                     # straight through: no lobe
        assert R[0] + T[0] + A[0] == pytest.approx(1.0, abs=1e-9)   # summation rounding


def test_index_matched_bubbles_are_invisible(orc):
    """n = 1, k = 0: no interface reflects, a bubble does not bend the ray, so
    T = exp(-alpha_tint d / cos) for every photon and the lobe is empty."""
    for c in (1.0, 0.6):
        R, T, A, W = orc.slab_mc(c, 550.0, 3.0, 30.0, 1.0, 0.0, 0.2, n_photons=2000)
        assert R[0] == pytest.approx(0.0, abs=1e-15)
        assert T[0] == pytest.approx(math.exp(-0.2 * 3.0 / c), rel=1e-12)
        assert W[0] < 1e-6


def test_energy_conservation_with_bubbles(orc):
    rng = np.random.default_rng(3)
    m = 40
    c = rng.uniform(0.05, 1.0, m)
    lam = rng.uniform(380, 780, m)
    d = rng.uniform(2, 5, m)
    rho = rng.uniform(0, 34, m)
    n = rng.uniform(1.5, 1.58, m)
    k = 10 ** rng.uniform(-7, -5, m)
    tint = rng.uniform(0, 0.5, m)
    R, T, A, W = orc.slab_mc(c, lam, d, rho, n, k, tint, n_photons=256)
    assert np.allclose(R + T + A, 1.0, atol=1e-12)
    assert np.all((R >= 0) & (T >= 0) & (A >= 0))
    assert np.all(W[rho > 5] > 0.01)           # bubbles open a transmitted lobe


def test_bubbles_scatter_more_with_density(orc):
    rhos = np.array([0.0, 5.0, 20.0, 34.0])
    R, T, A, W = orc.slab_mc(1.0, 550.0, 4.0, rhos, 1.52, 1e-7, 0.0, n_photons=20000)
    assert np.all(np.diff(W) > 0)              # wider lobe with more bubbles
    assert np.all(np.diff(R) > -3e-3)          # back-scatter does not drop


def _refract(d, nrm, eta):
    """Snell in vector form: d unit, nrm unit facing against d, eta = n1/n2."""
    ci = -np.dot(d, nrm)
    s2 = eta * eta * (1 - ci * ci)
    return eta * d + (eta * ci - math.sqrt(1 - s2)) * nrm


def _trace_sphere(d, ep, sin_i, n, p):
    """Explicit vector trace through a unit air sphere in glass of index n:
    refract in, p internal reflections, refract out."""
    d = np.asarray(d, float)
    centre = np.zeros(3)
    o = centre - 3.0 * d + sin_i * ep
    b = np.dot(o - centre, d)
    cc = np.dot(o - centre, o - centre) - 1.0
    t = -b - math.sqrt(b * b - cc)
    x = o + t * d
    nrm = (x - centre)
    d = _refract(d, nrm, n / 1.0)
    for k in range(p + 1):
        b = np.dot(x - centre, d)
        cc = np.dot(x - centre, x - centre) - 1.0
        t = -b + math.sqrt(max(b * b - cc, 0.0))
        x = x + t * d
        nrm = x - centre                        # outward
        if k < p:
            d = d - 2 * np.dot(d, nrm) * nrm     # internal reflection
        else:
            d = _refract(d, -nrm, 1.0 / n)      # back into glass
    return d / np.linalg.norm(d)


@pytest.mark.parametrize("sin_i,p", [(0.3, 0), (0.6, 0), (0.64, 0), (0.2, 1), (0.5, 1), (0.4, 2), (0.1, 3)])
def test_bubble_deviation_matches_vector_trace(orc, sin_i, p):
    n = 1.55
    assert n * sin_i < 1
    rng = np.random.default_rng(int(sin_i * 100) + p)
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    ep = np.cross(d, rng.normal(size=3))
    ep /= np.linalg.norm(ep)
    got = orc.bubble_dir(d, ep, sin_i, n, p)
    ref = _trace_sphere(d, ep, sin_i, n, p)
    assert np.allclose(got, ref, atol=1e-12)


def test_bubble_external_reflection_and_normal_incidence(orc):
    d = np.array([0.0, 0.0, 1.0])
    ep = np.array([1.0, 0.0, 0.0])
    assert np.allclose(orc.bubble_dir(d, ep, 0.0, 1.5, 0), d)      # straight through
    assert np.allclose(orc.bubble_dir(d, ep, 0.0, 1.5, 1), -d)     # one internal bounce
    assert np.allclose(orc.bubble_dir(d, ep, 0.0, 1.5, -1), -d)    # outer reflection
    out = orc.bubble_dir(d, ep, 0.5, 1.5, -1)
    nh = -math.sqrt(0.75) * d + 0.5 * ep
    assert np.allclose(out, d - 2 * np.dot(d, nh) * nh)
    # normal-incidence reflectance of the air gap, both orders
    assert orc.fresnel_real(1.5, 1.0, 1.0, 0) == pytest.approx((0.5 / 2.5) ** 2)
    assert orc.fresnel_real(1.0, 1.5, 1.0, 1) == pytest.approx((0.5 / 2.5) ** 2)
    # total reflection beyond the critical angle from glass into air
    assert orc.fresnel_real(1.5, 1.0, math.cos(math.asin(1 / 1.5) + 0.01), 0) == 1.0
