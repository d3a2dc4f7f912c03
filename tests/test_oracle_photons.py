"""Pins of the oracle's caustic photon map (photon mapping, Sec. 3.2).

- Sunlight that a clear pane lets straight through is the shadow rays'
  (next-event) light: a horizontal pane over a floor under an overhead sun
  stores no photon, and a bubbly pane without bubbles neither.
- A pane at 45 degrees reflects the overhead sun horizontally onto a wall:
  every stored photon lies on the wall in the reflected beam's footprint
  (the pane's shadow along the beam), with the wall's normal toward the
  beam, and the stored power adds up to sum_j E_j R_j(45 deg) A_proj (the
  sun's power on the pane's projected area times the slab reflectance, the
  closed-form slab), within 4 binomial standard errors.
- A render with the photon map over a scene where no pane turns light equals
  the render without it, bit for bit.
"""
import math

import numpy as np
import pytest

from paper_1912_05494_amd import synth
from scenes_for_tests import assemble, bubbly, glass, lambert, settings

SQ2 = math.sqrt(2.0)


def mirror_scene(half=0.5):
    """Floor z = 0, a wall at x = 2 (y in [-2, 2], z in [0, 3]) and a clear
    pane centred at (0, 0, 1) whose normal is (1, 0, 1) / sqrt(2); sun
    overhead."""
    fl = np.array([[-2, -2, 0], [2, -2, 0], [2, 2, 0], [-2, 2, 0]], dtype=np.float32)
    wall = np.array([[2, -2, 0], [2, 2, 0], [2, 2, 3], [2, -2, 3]], dtype=np.float32)
    a = half / SQ2
    pane = np.array([[-a, -half, 1 + a], [a, -half, 1 - a], [a, half, 1 - a], [-a, half, 1 + a]], dtype=np.float32)
    t = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    g = glass(n=1.52, k=1e-7, tint=0.0, thick=3.0, dispersive=True)
    return assemble([(fl, t, 0), (wall, t, 0), (pane, t, 1)], [lambert(0.5), g], sun_dir=(0.0, 0.0, 1.0),
                    sun_E=1.0, sky_L=0.0)


def test_straight_transmission_stores_nothing(orc):
    fl = np.array([[-2, -2, 0], [2, -2, 0], [2, 2, 0], [-2, 2, 0]], dtype=np.float32)
    p = np.array([[-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float32)
    t = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    st = settings(synth.Camera(eye=(0, -3, 2), target=(0, 0, 0), W=8, H=8), spp=1, max_depth=4)
    for pane in (glass(n=1.5, k=1e-6, tint=0.3), bubbly(density=0.0)):
        sc = assemble([(fl, t, 0), (p, t, 1)], [lambert(0.5), pane], sun_dir=(0.0, 0.0, 1.0))
        ph = orc.photon_map(orc.OracleScene(sc), st, 20000, 0.1)
        assert ph.shape == (0, 8)


def test_mirror_pane_power_and_footprint(orc):
    half = 0.5
    sc = mirror_scene(half)
    st = settings(synth.Camera(eye=(0, -3, 2), target=(0, 0, 0), W=8, H=8), spp=1, max_depth=4)
    N = 400000
    ph = orc.photon_map(orc.OracleScene(sc), st, N, 0.1)
    assert len(ph) > 500
    x, n, P, j = ph[:, :3], ph[:, 3:6], ph[:, 6], ph[:, 7].astype(int)
    assert np.allclose(x[:, 0], 2.0, atol=1e-9)
    assert np.all(np.abs(x[:, 1]) <= half + 1e-9)
    assert np.all(np.abs(x[:, 2] - 1.0) <= half / SQ2 + 1e-9)
    assert np.allclose(n, [-1.0, 0.0, 0.0], atol=1e-12)
    lam = st.lambda_nm.astype(np.float64)
    g = sc.materials[1]
    R, T = orc.slab(math.cos(math.pi / 4), lam, 3.0, np.interp(lam, synth.LAMBDA_81, g.n),
                    np.interp(lam, synth.LAMBDA_81, g.k), np.interp(lam, synth.LAMBDA_81, g.alpha_tint))
    a_proj = (2 * half) ** 2 / SQ2
    want = float(np.sum(R * 1.0 * a_proj))
    got = float(P.sum())
    # binomial error of the count of photons reflected toward the wall
    se = want / math.sqrt(len(ph))
    assert abs(got - want) <= 4 * se, (got, want, se)
    # every wavelength is represented, each with power E R A_proj nl / (photons shot of it)
    assert set(j) == set(range(len(lam)))


def test_photon_map_off_where_nothing_turns(orc):
    fl = np.array([[-2, -2, 0], [2, -2, 0], [2, 2, 0], [-2, 2, 0]], dtype=np.float32)
    p = np.array([[-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float32)
    t = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    sc = assemble([(fl, t, 0), (p, t, 1)], [lambert(0.5), glass(n=1.5, k=1e-6, tint=0.3)],
                  sun_dir=(0.0, 0.0, 1.0), sun_E=2.0, sky_L=0.5)
    st = settings(synth.Camera(eye=(0.3, -3, 2), target=(0, 0, 0.3), W=12, H=12), spp=3, max_depth=4)
    osc = orc.OracleScene(sc)
    a, _ = orc.render(osc, st)
    b, _ = orc.render(osc, st, photons=5000, photon_radius=0.1)
    assert np.array_equal(a, b)


def test_photon_parameter_checks(orc):
    sc = mirror_scene()
    st = settings(synth.Camera(eye=(0, -3, 2), target=(0, 0, 0), W=4, H=4), spp=1, max_depth=2)
    osc = orc.OracleScene(sc)
    with pytest.raises(ValueError):
        orc.photon_map(osc, st, -1, 0.1)
    with pytest.raises(ValueError):
        orc.photon_map(osc, st, 100, 0.0)
