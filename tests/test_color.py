"""Pins of the colour-difference utility: closed-form special cases of
CIEDE2000 and of the CIELAB conversion."""
import numpy as np
import pytest

from paper_1912_05494_amd import color, synth


def test_lab_of_white_and_black():
    wp = np.array([0.95, 1.0, 1.09])
    assert np.allclose(color.xyz_to_lab(wp, wp), [100.0, 0.0, 0.0], atol=1e-12)
    assert np.allclose(color.xyz_to_lab([0, 0, 0], wp), [0.0, 0.0, 0.0], atol=1e-12)
    # a grey is neutral: a = b = 0, and L follows the cube-root law
    lab = color.xyz_to_lab(0.3 * wp, wp)
    assert lab[1] == pytest.approx(0, abs=1e-12) and lab[2] == pytest.approx(0, abs=1e-12)
    assert lab[0] == pytest.approx(116 * 0.3 ** (1 / 3) - 16, rel=1e-12)


def test_delta_e_special_cases():
    rng = np.random.default_rng(0)
    a = np.stack([rng.uniform(0, 100, 200), rng.uniform(-80, 80, 200), rng.uniform(-80, 80, 200)], -1)
    b = a + rng.normal(0, 2, a.shape)
    assert np.all(color.delta_e2000(a, a) == 0)
    assert np.allclose(color.delta_e2000(a, b), color.delta_e2000(b, a), rtol=1e-12)
    # neutral colours around L = 50: S_L = 1 and the chroma terms vanish
    for dl in (0.5, 2.0, 7.0):
        assert color.delta_e2000([50 - dl / 2, 0, 0], [50 + dl / 2, 0, 0]) == pytest.approx(dl, rel=1e-12)
    # lightness weighting away from L = 50: S_L = 1 + 0.015 (L - 50)^2 / sqrt(20 + (L - 50)^2)
    SL = 1 + 0.015 * 400 / np.sqrt(420)
    assert color.delta_e2000([69.9, 0, 0], [70.1, 0, 0]) == pytest.approx(0.2 / SL, rel=1e-9)


def test_white_point_is_flat_spectrum():
    lam = synth.LAMBDA_81.astype(np.float64)
    cmf = synth.cmf_xyz(lam)
    wp = color.white_point(cmf, lam, Y=2.0)
    assert wp[1] == pytest.approx(2.0)
    spec = np.full((3, 4, len(lam)), 5.0)
    from oracle import spec_to_xyz
    xyz = spec_to_xyz(spec, lam, cmf)
    de = color.image_delta_e(xyz, xyz, cmf, lam)
    assert np.all(de == 0)
    lab = color.xyz_to_lab(xyz, color.white_point(cmf, lam, Y=xyz[0, 0, 1]))
    assert np.allclose(lab, [100, 0, 0], atol=1e-9)


def test_delta_e_pure_chroma_difference():
    """Same lightness and hue (b = 0): only the chroma term is left,
    dC' / S_C with a' = (1 + G) a and S_C = 1 + 0.045 C'."""
    a1, a2 = 10.0, 12.0
    cm = 0.5 * (a1 + a2)
    G = 0.5 * (1 - np.sqrt(cm ** 7 / (cm ** 7 + 25.0 ** 7)))
    dc = (1 + G) * (a2 - a1)
    SC = 1 + 0.045 * (1 + G) * cm
    assert color.delta_e2000([50, a1, 0], [50, a2, 0]) == pytest.approx(dc / SC, rel=1e-12)
