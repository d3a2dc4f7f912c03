"""Pins of the oracle's event signatures (the debug aid that explains a
pixel's difference by a path that decided differently) and of its work-item
ranges (a render split into runs of items, as the checkpointed GPU render
is).  The event hash is the SplitMix64 output function, checked here against
that generator's published first outputs; the signatures of closed-form
scenes are then written out event by event."""
import numpy as np
import pytest

from paper_1912_05494_amd import synth
from paper_1912_05494_amd.synth import Camera
from scenes_for_tests import assemble, glass, lambert, ortho_down, quad, settings

M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def out(z):
    """SplitMix64 (Steele, Lea and Flood 2014): the output for state z + gamma."""
    z = (z + GAMMA) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def hit(vtx, smp, tri):
    return out(1 << 56 | vtx << 48 | smp << 32 | (tri + 1))


def shadow(vtx, panes=(), occluded=False):
    k = out(2 << 56 | vtx << 48 | (0xFFFF if occluded else len(panes)))
    if not occluded:
        for t in panes:
            k += out(3 << 56 | t)
    return k & M64


def test_hash_is_splitmix64():
    """The first three outputs of SplitMix64 seeded with 0."""
    assert out(0) == 0xE220A8397B1DCDAF
    assert out(GAMMA) == 0x6E789E6AA1B965F4
    assert out(2 * GAMMA & M64) == 0x06C45D188009454F


def test_empty_scene_signature(orc):
    """No geometry: each path's only event is a miss at vertex 0."""
    sc = assemble([], [lambert(0.5)])
    st = settings(ortho_down(1.0, 1.0, W=5, H=3), spp=3, max_depth=3)
    spec, _, ev = orc.render(orc.OracleScene(sc), st, events=True)
    want = sum(hit(0, s, -1) for s in range(3)) & M64
    assert np.all(ev == np.uint64(want))
    assert np.all(spec == 1.0)


def test_floor_signature(orc):
    """One Lambert triangle under an orthographic camera: every sample hits
    triangle 0 at vertex 0, its shadow ray is free (no pane), and the cosine
    bounce leaves the scene at vertex 1."""
    p = np.array([[-10, -10, 0], [10, -10, 0], [0, 10, 0]], dtype=np.float32)
    t = np.array([[0, 1, 2]], dtype=np.int32)
    sc = assemble([(p, t, 0)], [lambert(0.4)], sun_dir=(0.3, 0.2, 0.9), sun_E=1.0, sky_L=1.0)
    for depth in (1, 2):
        st = settings(ortho_down(1.0, 1.0, W=4, H=4), spp=2, max_depth=depth)
        _, _, ev = orc.render(orc.OracleScene(sc), st, events=True)
        per = [hit(0, s, 0) + shadow(0) + (hit(1, s, -1) if depth == 2 else 0) for s in range(2)]
        assert np.all(ev == np.uint64(sum(per) & M64)), depth


def test_pane_shadow_signature(orc):
    """A pane between the floor and the sun: a sample's shadow event names
    the pane triangle its shadow ray crosses, or no pane.  Every pixel's
    signature must be one of the sums these choices allow."""
    pf = np.array([[-10, -10, 0], [10, -10, 0], [0, 10, 0]], dtype=np.float32)
    tf = np.array([[0, 1, 2]], dtype=np.int32)
    pg, tg = quad(0.5, 0.2)
    sc = assemble([(pf, tf, 0), (pg, tg, 1)], [lambert(0.4), glass(k=1e-6)], sun_dir=(0.0, 0.0, 1.0),
                  sun_E=1.0, sky_L=0.0, vthick=3.0)
    spp = 2
    st = settings(ortho_down(0.3, 0.8, W=12, H=12), spp=spp, max_depth=1)
    _, _, ev = orc.render(orc.OracleScene(sc), st, events=True)
    choices = [shadow(0), shadow(0, [1]), shadow(0, [2])]
    allowed = set()
    for a in choices:
        for b in choices:
            allowed.add((hit(0, 0, 0) + hit(0, 1, 0) + a + b) & M64)
    vals = set(int(x) for x in ev.reshape(-1))
    assert vals <= allowed
    # both shadowed and free samples occur
    assert (hit(0, 0, 0) + hit(0, 1, 0) + 2 * choices[0]) & M64 in vals
    assert len(vals) >= 3


def test_signature_independent_of_decomposition(orc):
    sc = synth.tiny_scene()
    st = synth.tiny_settings(W=20, H=12, spp=2)
    osc = orc.OracleScene(sc)
    _, _, e0 = orc.render(osc, st, events=True)
    _, _, e1 = orc.render(osc, st, events=True, n_bands=4, tile=7)
    _, _, e2 = orc.render(osc, st, events=True, use_bvh=False)
    assert np.array_equal(e0, e1) and np.array_equal(e0, e2)
    px = np.array([0, 5, 119, 239], dtype=np.int32)
    _, ep = orc.render_pixels(osc, st, px, events=True)
    assert np.array_equal(ep, e0.reshape(-1, e0.shape[-1])[px])


def test_item_ranges_compose(orc):
    """Items run in plan order (tile rows, tiles, bands); rendering them in
    two runs fills the image exactly as one run does, and a run leaves the
    other items' entries untouched."""
    sc = synth.tiny_scene()
    st = synth.tiny_settings(W=24, H=20, spp=2)
    st.n_bands = 3
    osc = orc.OracleScene(sc)
    full, _ = orc.render(osc, st, tile=8)
    n_items = 3 * 3 * 3
    part, _ = orc.render(osc, st, tile=8, items=(0, 4))
    # items 0..3: tile (0, 0) bands 0, 1, 2 and tile (1, 0) band 0
    bands = [(0, 6), (6, 11), (11, 16)]
    mask = np.zeros(full.shape, dtype=bool)
    for tx, b in [(0, 0), (0, 1), (0, 2), (1, 0)]:
        mask[0:8, 8 * tx:8 * tx + 8, bands[b][0]:bands[b][1]] = True
    assert np.array_equal(part[mask], full[mask])
    assert np.all(part[~mask] == 0.0)
    rest, _ = orc.render(osc, st, tile=8, items=(4, 0), spec=part)
    assert np.array_equal(rest, full)
    # three runs, the last one past the end
    a, _ = orc.render(osc, st, tile=8, items=(0, 10))
    a, _ = orc.render(osc, st, tile=8, items=(10, 10), spec=a)
    a, _ = orc.render(osc, st, tile=8, items=(20, 100), spec=a)
    assert np.array_equal(a, full)
    assert n_items == 27


def _grazing_scene(vthick):
    floor = np.array([[-5, -5, 0], [5, -5, 0], [5, 5, 0], [-5, 5, 0]], dtype=np.float32)
    ft = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    pane = np.array([[-5, 0, 0.001], [5, 0, 0.001], [5, 0, 300], [-5, 0, 300]], dtype=np.float32)
    pt = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    sun = (0.0, 0.002, np.sqrt(1 - 0.002 ** 2))
    vt = np.concatenate([np.full(4, 3.0), vthick]).astype(np.float32)
    return assemble([(floor, ft, 0), (pane, pt, 1)], [lambert(0.5), glass(n=1.52, k=0.0, tint=0.3)],
                    sun_dir=sun, sun_E=1.0, sky_L=0.0, vthick=vt)


REL, CEPS, EPS = 4 * 2.0 ** -24, 5 * 2.0 ** -24, 2.0 ** -23


def test_precision_bound_cosine(orc):
    """A floor under a sun 0.1146 degrees from the vertical and a tall
    vertical pane of constant thickness in the plane y = 0: shadow rays from
    floor points with y < 0 cross the pane at a sun cosine c = 0.002.  The
    single-precision bound of such a pixel is its value times (3 factors of
    the light sum + 1 glass factor) x REL + CEPS / c + CEPS / cos_sun at the
    floor; pixels with y > 0 (no pane on the way) get 3 REL + CEPS /
    cos_sun.  The camera looks straight down and sees the pane edge-on."""
    sc = _grazing_scene([3.0, 3.0, 3.0, 3.0])
    st = settings(Camera(eye=(0.0, 0.0, 1.0), target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), W=8, H=8,
                         projection=1, ortho_height=0.4), spp=3, max_depth=1)
    spec, _, pb = orc.render(orc.OracleScene(sc), st, prec=(REL, CEPS, EPS))
    # image rows run from the top (+y) down: rows 0..3 see y > 0, rows 4..7 y < 0
    cs = np.sqrt(1 - 0.002 ** 2)
    assert np.allclose(pb[:4] / spec[:4], 3 * REL + CEPS / cs, rtol=1e-9)
    assert np.allclose(pb[4:] / spec[4:], 4 * REL + CEPS / 0.002 + CEPS / cs, rtol=1e-6)


def test_precision_bound_thickness_gradient(orc):
    """The same pane with thickness 2 mm at its bottom edge and 5 mm at its
    top (z = 300 m): gradient 0.01 mm per m, absorption 0.3 per mm.  The
    camera origin (|o| = 1) is rounded (EPS), the floor hit 1 m below is
    reached head-on, so its error is e = 2 EPS + 0.05 EPS; the shadow ray
    then crosses the pane about 25 m up at c = 0.002, so the crossing's
    error is h = (e + 25 EPS) / c + 25 EPS, and the glass factor adds
    0.3 * 0.01 * h / cos_t with cos_t = sqrt(1 - (0.999998 / 1.52)^2)."""
    sc = _grazing_scene([2.0, 2.0, 5.0, 5.0])
    cam = Camera(eye=(0.0, -0.05, 1.0), target=(0.0, -0.05, 0.0), up=(0.0, 1.0, 0.0), W=4, H=4,
                 projection=1, ortho_height=0.001)
    st = settings(cam, spp=2, max_depth=1)
    spec, _, pb = orc.render(orc.OracleScene(sc), st, prec=(0.0, 0.0, EPS))
    c = 0.002
    z = 0.05 * np.sqrt(1 - c * c) / c                  # crossing height
    e = 2.05 * EPS
    h = (e + z * EPS) / c + z * EPS
    ct = np.sqrt(1 - (np.sqrt(1 - c * c) / 1.52) ** 2)
    assert np.allclose(pb / spec, 0.3 * 0.01 * h / ct, rtol=0.02)
