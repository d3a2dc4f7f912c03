"""Pins of the oracle's bubbly-pane rendering: the BF16 rounding, the
surrogate's lobe sampler, the slab frame, the walk's structure without
bubbles, and closed-form renders (an absorption-free bubbly pane is invisible
under a uniform sky; a constant network scales the sky by R + T; the fallback
mode reduces to either pure mode; shadow rays see the ballistic slab)."""
import math

import numpy as np
import pytest

from paper_1912_05494_amd import synth
from scenes_for_tests import LAM, assemble, bubbly, constant_net, glass, ortho_down, quad, settings


def test_bf16_rounding_matches_torch(orc):
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 3, 4000), rng.uniform(-1e-3, 1e-3, 1000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 65504.0, 3e38]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    assert np.array_equal(orc.bf16(x), ref)


def test_bf16_network_within_rounding_of_fp64(orc):
    from paper_1912_05494_amd import surrogate
    rng = np.random.default_rng(1)
    p = surrogate.init_params(3, seed=2).astype(np.float64)
    tup, pane = surrogate.random_tuples(300, 3, synth.LAMBDA_81, seed=3)
    a = orc.mlp_forward(p, 3, tup, pane)
    b = orc.mlp_forward_bf16(p, 3, tup, pane)
    err = np.abs(a - b)
    assert 0 < err.max() < 2e-2           # roundings take effect, within the BF16 bound
    z = np.zeros_like(p)
    z[-(8 * 3 + 3):-8 * 3] = [0.25, -0.125, 0.5]   # output biases only (exact in float)
    assert np.array_equal(orc.mlp_forward(z, 3, tup, pane), orc.mlp_forward_bf16(z, 3, tup, pane))


def test_lobe_sampler_statistics(orc):
    d = np.array([0.3, -0.4, 0.866])
    d /= np.linalg.norm(d)
    assert np.array_equal(orc.lobe_dir(d, 0.0, 0.7, 0.2), d)
    w = 0.02
    u = (np.arange(200) + 0.5) / 200
    th2, mean = [], np.zeros(3)
    for u1 in u:
        for u2 in u[::4]:
            o = orc.lobe_dir(d, w, u1, u2)
            assert abs(np.linalg.norm(o) - 1) < 1e-12
            th2.append(math.acos(min(1.0, float(o @ d))) ** 2)
            mean += o
    # two Gaussian tangent offsets of sd w: E[theta^2] = 2 w^2 (small-angle)
    assert np.mean(th2) == pytest.approx(2 * w * w, rel=0.03)
    mean /= np.linalg.norm(mean)
    assert np.linalg.norm(mean - d) < 1e-4


def test_lobe_transmit_stays_on_far_side(orc):
    """The surrogate's transmitted direction: the lobe sample where it already
    points through the pane, else its mirror image across the pane's plane
    (tangential part kept, normal part negated), so always on the far side."""
    rng = np.random.default_rng(9)
    folded = 0
    for _ in range(400):
        ng = rng.normal(size=3)
        ng /= np.linalg.norm(ng)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        w, u1, u2 = rng.uniform(0.0, 1.2), rng.random(), rng.random()
        lobe = orc.lobe_dir(d, w, u1, u2)
        out = orc.lobe_transmit(d, ng, w, u1, u2)
        assert (out @ ng) * (d @ ng) >= 0.0
        assert abs(np.linalg.norm(out) - 1) < 1e-12
        if (lobe @ ng) * (d @ ng) >= 0.0:
            assert np.array_equal(out, lobe)
        else:
            folded += 1
            tang = lobe - (lobe @ ng) * ng
            assert np.allclose(out - (out @ ng) * ng, tang, atol=1e-14)
            assert out @ ng == pytest.approx(-(lobe @ ng), abs=1e-14)
    assert folded > 20      # wide lobes at grazing incidence do cross the plane


def test_slab_frame(orc):
    rng = np.random.default_rng(4)
    for _ in range(50):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        ng = rng.normal(size=3)
        ng /= np.linalg.norm(ng)
        c = abs(d @ ng)
        s = math.sqrt(1 - c * c)
        # the incident direction itself, and its mirror image
        assert np.allclose(orc.slab_to_world(d, ng, [s, 0, c]), d, atol=1e-12)
        assert np.allclose(orc.slab_to_world(d, ng, [s, 0, -c]), d - 2 * (d @ ng) * ng, atol=1e-12)
    # head-on: the frame falls back to the fixed tangent basis, z still the ray
    assert np.allclose(orc.slab_to_world([0, 0, -1], [0, 0, 1], [0, 0, 1]), [0, 0, -1])


@pytest.mark.parametrize("cos_i", [1.0, 0.6, 0.15])
def test_walk_without_bubbles_is_the_ray_series(orc, cos_i):
    """sigma = 0: the photon bounces between the faces; after m internal
    reflections it leaves the far face (m even) with L = (m + 1) d / cos_t and
    the incident direction, or the entry face (m odd) with the mirror one."""
    n, d = 1.5, 3.0
    ct = orc.snell_cos_t(cos_i, n)
    s = math.sqrt(1 - cos_i * cos_i)
    seen = set()
    for ph in range(400):
        kind, a, L = orc.bubbly_walk(cos_i, d, 0.0, n, ph % 2, seed=5, c0=1, c1=ph)
        m = round(L * ct / d) - 1
        assert L == pytest.approx((m + 1) * d / ct, rel=1e-13)
        assert kind == (2 if m % 2 == 0 else 1)
        assert np.allclose(a, [s, 0, c if (c := cos_i) and kind == 2 else -cos_i], atol=1e-12)
        seen.add(m)
    assert 0 in seen and len(seen) >= 2


def test_walk_draw_counters(orc):
    """Dataset and render counters are the documented Philox words."""
    u = orc.walk_draw(7, 3, 4, 5, 2)
    x = orc.philox(np.array([[3, 4, 5, 0x5EB10002]], np.uint32), np.array([[7, 0]], np.uint32))[0]
    assert np.array_equal(u, (x >> 8) * 2.0 ** -24)
    u = orc.walk_draw(7, 3, 4, 5, 2, render=True, vertex=6, c3=9)
    w2 = 0x80000000 | (6 << 23) | (5 << 5) | 2
    x = orc.philox(np.array([[3, 4, w2, 9]], np.uint32), np.array([[7, 0]], np.uint32))[0]
    assert np.array_equal(u, (x >> 8) * 2.0 ** -24)


def pane_scene(mat, sky=1.0, sun=0.0):
    p, t = quad(0.0, 2.0)
    return assemble([(p, t, 0)], [mat], sun_E=sun, sky_L=sky, vthick=3.0)


def oblique(W=12, H=12):
    return synth.Camera(eye=(0.3, -1.2, 1.5), target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0), W=W, H=H,
                        vfov_deg=50.0)


def test_absorption_free_bubbly_pane_is_invisible(orc):
    """k = 0, no tint: a walk loses no energy, so under a unit sky every path
    ends with weight 1 whatever the bubbles do."""
    sc = pane_scene(bubbly(n=1.5, k=0.0, tint=0.0, density=30.0))
    st = settings(oblique(), spp=6, max_depth=4)
    spec, _ = orc.render(orc.OracleScene(sc), st, btdf={"mode": "exact"})
    assert np.allclose(spec, 1.0, rtol=0, atol=1e-15)


def test_constant_network_scales_the_sky(orc):
    R, T, w = 0.1, 0.6, 0.05
    net = constant_net(1, R, T, w)
    sc = pane_scene(bubbly(density=10.0))
    st = settings(ortho_down(1.0, 1.0, W=8, H=8), spp=3, max_depth=3)
    for bf16 in (False, True):
        spec, _ = orc.render(orc.OracleScene(sc), st,
                             btdf={"mode": "surrogate", "params": net, "n_panes": 1, "bf16": bf16})
        # exp(o) of the biases is exact to rounding: R + T up to 1e-15
        assert np.allclose(spec, R + T, rtol=1e-12)


def test_fallback_reduces_to_either_mode(orc):
    from paper_1912_05494_amd import surrogate
    net = surrogate.init_params(2, seed=7).astype(np.float64)
    sc = pane_scene(bubbly(density=12.0, pane_id=1), sun=1.0)
    st = settings(oblique(10, 10), spp=2, max_depth=3)
    osc = orc.OracleScene(sc)
    base = {"params": net, "n_panes": 2}
    ex, _ = orc.render(osc, st, btdf=dict(base, mode="exact"))
    su, _ = orc.render(osc, st, btdf=dict(base, mode="surrogate"))
    hi = np.full((2, 4, 3, 2), 1.0)
    lo = np.zeros((2, 4, 3, 2))
    fh, _ = orc.render(osc, st, btdf=dict(base, mode="fallback", err_table=hi, bound=1e-3))
    fl, _ = orc.render(osc, st, btdf=dict(base, mode="fallback", err_table=lo, bound=1e-3))
    assert np.array_equal(fh, ex) and np.array_equal(fl, su)
    assert not np.array_equal(ex, su)
    # a table flagging only some cells mixes the two per vertex
    mix = lo.copy()
    mix[1, :2] = 1.0                    # cos(theta) < 0.5 on pane type 1
    fm, _ = orc.render(osc, st, btdf=dict(base, mode="fallback", err_table=mix, bound=1e-3))
    assert not np.array_equal(fm, ex) and not np.array_equal(fm, su)


def test_bubbly_shadow_is_ballistic(orc):
    """Toward the sun a bubbly pane passes the unscattered light only: the
    slab transmittance with the bubbles' extinction added to the absorption."""
    p, t = quad(0.5, 1.0)
    mat = bubbly(n=1.52, k=1e-6, tint=0.1, density=15.0)
    sc = assemble([(p, t, 0)], [mat], sun_dir=(0.2, 0.1, 1.0), sun_E=1.0, sky_L=0.0, vthick=3.0)
    osc = orc.OracleScene(sc)
    sun = np.asarray(sc.sun_dir, np.float64)
    c = abs(sun[2])
    sig = orc.bubble_sigma(15.0, 10.0, 200.0)
    for lam in (450.0, 600.0):
        T = osc.shadow(np.array([[0.0, 0.0, 0.0]]), lam)[0]
        _, Tr = orc.slab(c, lam, 3.0, float(np.float32(1.52)), float(np.float32(1e-6)), float(np.float32(0.1)) + sig)
        assert T == pytest.approx(float(Tr), rel=1e-12)
    assert sig == pytest.approx(15.0 * math.pi * (0.01 ** 2 + 0.01 * 0.2 + 0.2 ** 2) / 3, rel=1e-14)


def test_exact_without_bubbles_matches_clear_glass(orc):
    """rho_b = 0 and a dispersion-free index: the exact walk samples the same
    slab series as the clear-glass vertex, so image means agree within noise."""
    sc_b = pane_scene(bubbly(n=1.5, k=3e-6, tint=0.2, density=0.0), sky=1.0)
    sc_g = pane_scene(glass(n=1.5, k=3e-6, tint=0.2), sky=1.0)
    st = settings(oblique(16, 16), spp=16, max_depth=3)
    a, _ = orc.render(orc.OracleScene(sc_b), st, btdf={"mode": "exact"})
    b, _ = orc.render(orc.OracleScene(sc_g), st)
    sd = np.sqrt(a.var() / a.size) + np.sqrt(b.var() / b.size)
    assert abs(a.mean() - b.mean()) < 4 * sd + 1e-12
