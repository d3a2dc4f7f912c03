"""Pins of the oracle's distribution maps (Sec. 6: optical constants and
thickness distributed over the geometry; looked up through a hit's texture
coordinates, Sec. 3.1).

- The texel lookup against hand-computed cases on a unit quad whose texture
  coordinates are its (x, y): the material of texel (floor(s W), floor(t H)),
  clamped; the bilinear thickness equals the texel values at texel centres,
  their mean halfway between neighbours, and the edge values beyond the
  outer centres.
- A white furnace (uniform sky 1, no sun, orthographic view at normal
  incidence, one pane alone): each pixel is exactly R + T of the slab of the
  glass of the texel under it, from the closed-form slab.
- A map whose every texel names one glass renders the same image, bit for
  bit, as the pane made of that glass.
"""
import numpy as np
import pytest

from paper_1912_05494_amd import synth
from scenes_for_tests import assemble, glass, ortho_down, settings


def unit_quad_scene(maps, mat_of_pane, extra, thick=3.0):
    """Pane: the square [0, 1]^2 at z = 0 with uv = (x, y); materials: the
    pane's (index 0) and then `extra`."""
    p = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]], dtype=np.float32)
    t = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    pane = glass(n=1.5, thick=thick)
    pane.dist_map = mat_of_pane
    sc = assemble([(p, t, 0)], [pane] + extra, sun_E=0.0, sky_L=1.0)
    sc.uv = p[:, :2].copy()
    sc.maps = maps
    return sc


def bary(tri, x, y):
    """Barycentric (u, v) of point (x, y) in triangle 0 (0,0)-(1,0)-(1,1) or
    triangle 1 (0,0)-(1,1)-(0,1)."""
    if tri == 0:
        return x - y, y          # p = p0 + u (p1 - p0) + v (p2 - p0)
    return x, y - x


def test_texel_material_and_bilinear_thickness(orc):
    m = np.array([[1, 2, 1], [2, 2, 1]], dtype=np.int32)      # H = 2 rows, W = 3 columns
    th = np.array([[2.0, 3.0, 4.0], [5.0, 6.0, 7.0]], dtype=np.float32)
    sc = unit_quad_scene([synth.DistMap(W=3, H=2, material=m, thick_mm=th)], 1, [glass(1.6), glass(1.7)])
    osc = orc.OracleScene(sc)
    for x, y, want in [(0.1, 0.1, 1), (0.4, 0.2, 2), (0.9, 0.3, 1), (0.2, 0.8, 2), (0.5, 0.6, 2),
                       (0.95, 0.99, 1)]:
        tri = 0 if x >= y else 1
        u, v = bary(tri, x, y)
        mat, _ = orc.pane_at(osc, tri, u, v)
        assert mat == want, (x, y)
    # texel centres ((x + 0.5) / 3, (y + 0.5) / 2): the texel's own value
    for iy in range(2):
        for ix in range(3):
            x, y = (ix + 0.5) / 3, (iy + 0.5) / 2
            tri = 0 if x >= y else 1
            _, d = orc.pane_at(osc, tri, *bary(tri, x, y))
            assert d == pytest.approx(float(th[iy, ix]), abs=1e-12)
    # halfway between horizontal neighbours of row 0, and vertical of column 2
    x, y = 1.0 / 3.0, 0.25
    _, d = orc.pane_at(osc, 0, *bary(0, x, y))
    assert d == pytest.approx(2.5, abs=1e-12)
    x, y = 5.0 / 6.0, 0.5
    _, d = orc.pane_at(osc, 0, *bary(0, x, y))
    assert d == pytest.approx(5.5, abs=1e-12)
    # beyond the outer centres: clamped to the edge texels
    _, d = orc.pane_at(osc, 0, *bary(0, 0.05, 0.01))
    assert d == pytest.approx(2.0, abs=1e-12)
    _, d = orc.pane_at(osc, 1, *bary(1, 0.97, 0.99))
    assert d == pytest.approx(7.0, abs=1e-12)
    # a material without a map keeps its own
    sc2 = unit_quad_scene([], 0, [])
    assert orc.pane_at(orc.OracleScene(sc2), 0, 0.3, 0.2) == (0, pytest.approx(3.0))


def test_map_furnace_closed_form(orc):
    """Orthographic view straight down at a pane in a uniform sky: each
    sample's weight is R + T of the slab under it and the path then escapes,
    so a pixel is exactly R + T of its texel's glass (closed-form slab)."""
    g1 = glass(n=1.5, k=1e-6, tint=0.4, thick=3.0)
    g2 = glass(n=1.65, k=3e-7, tint=1.5, thick=3.0, dispersive=True)
    m = np.array([[1, 2], [2, 1]], dtype=np.int32)
    p = np.array([[-1, -1, 0], [1, -1, 0], [1, 1, 0], [-1, 1, 0]], dtype=np.float32)
    t = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    pane = glass(n=1.5)
    pane.dist_map = 1
    sc = assemble([(p, t, 0)], [pane, g1, g2], sun_E=0.0, sky_L=1.0, vthick=2.5)
    sc.uv = (p[:, :2] + 1.0) / 2.0
    sc.maps = [synth.DistMap(W=2, H=2, material=m)]
    st = settings(ortho_down(1.0, 2.0, W=8, H=8), spp=3, max_depth=3)
    spec, _ = orc.render(orc.OracleScene(sc), st)
    lam = st.lambda_nm.astype(np.float64)
    for j in range(8):
        for i in range(8):
            o, d = orc.camera_ray(st, i, j, 0.5, 0.5)
            x = o + (-o[2] / d[2]) * d
            s_, t_ = (x[0] + 1) / 2, (x[1] + 1) / 2
            gm = [g1, g2][m[int(t_ * 2), int(s_ * 2)] - 1]
            n = np.interp(lam, synth.LAMBDA_81, gm.n)
            k = np.interp(lam, synth.LAMBDA_81, gm.k)
            tint = np.interp(lam, synth.LAMBDA_81, gm.alpha_tint)
            R, T = orc.slab(1.0, lam, 2.5, n, k, tint)
            assert np.allclose(spec[j, i], R + T, rtol=1e-12, atol=0), (i, j)


def test_uniform_map_equals_plain_pane(orc):
    g1 = glass(n=1.58, k=2e-6, tint=0.7, thick=4.0, dispersive=True)
    p = np.array([[-1, -1, 0.5], [1, -1, 0.5], [1, 1, 0.5], [-1, 1, 0.5]], dtype=np.float32)
    t = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    fl = np.array([[-3, -3, 0], [3, -3, 0], [3, 3, 0], [-3, 3, 0]], dtype=np.float32)
    from scenes_for_tests import lambert
    pane = glass(n=1.5)
    pane.dist_map = 1
    mapped = assemble([(fl, t, 2), (p, t, 0)], [pane, g1, lambert(0.5)], sun_dir=(0.3, 0.2, 1.0),
                      sun_E=2.0, sky_L=0.5)
    mapped.uv = np.concatenate([np.zeros((4, 2)), (p[:, :2] + 1) / 2]).astype(np.float32)
    mapped.maps = [synth.DistMap(W=3, H=5, material=np.full((5, 3), 1, np.int32),
                                 thick_mm=np.full((5, 3), 4.0, np.float32))]
    plain = assemble([(fl, t, 2), (p, t, 1)], [glass(n=1.5), g1, lambert(0.5)], sun_dir=(0.3, 0.2, 1.0),
                     sun_E=2.0, sky_L=0.5)
    cam = synth.Camera(eye=(0.4, -2.5, 2.0), target=(0.0, 0.0, 0.3), W=16, H=16, vfov_deg=50.0)
    st = settings(cam, spp=4, max_depth=4)
    a, _ = orc.render(orc.OracleScene(mapped), st)
    b, _ = orc.render(orc.OracleScene(plain), st)
    assert np.array_equal(a, b)
    assert a.max() > 0


def test_map_validation(orc):
    m = np.zeros((1, 1), dtype=np.int32)
    bad_ref = unit_quad_scene([synth.DistMap(W=1, H=1, material=m)], 1, [])   # texel names the mapped pane
    with pytest.raises(ValueError):
        orc.OracleScene(bad_ref)
    no_uv = unit_quad_scene([synth.DistMap(W=1, H=1, material=m + 1)], 1, [glass()])
    no_uv.uv = None
    with pytest.raises(ValueError):
        orc.OracleScene(no_uv)
    bad_thick = unit_quad_scene([synth.DistMap(W=1, H=1, material=m + 1, thick_mm=np.zeros((1, 1), np.float32))],
                                1, [glass()])
    with pytest.raises(ValueError):
        orc.OracleScene(bad_thick)
