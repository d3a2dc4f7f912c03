"""Small hand-built scenes for the closed-form pins (inputs only)."""
import numpy as np

from paper_1912_05494_amd import synth
from paper_1912_05494_amd.synth import GLASS, LAMBERT, Camera, Material, RenderSettings, Scene

LAM = synth.LAMBDA_81


def quad(z, half, x0=0.0, y0=0.0):
    p = np.array([[x0 - half, y0 - half, z], [x0 + half, y0 - half, z],
                  [x0 + half, y0 + half, z], [x0 - half, y0 + half, z]], dtype=np.float32)
    return p, np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)


def assemble(parts, materials, sun_dir=(0.0, 0.0, 1.0), sun_E=1.0, sky_L=1.0, vthick=None):
    pos, idx, mat, base = [], [], [], 0
    for p, t, m in parts:
        pos.append(p)
        idx.append(t + base)
        mat.append(np.full(len(t), m, dtype=np.int32))
        base += len(p)
    n = len(LAM)
    sE = np.full(n, sun_E, dtype=np.float32) if np.isscalar(sun_E) else np.asarray(sun_E, np.float32)
    sL = np.full(n, sky_L, dtype=np.float32) if np.isscalar(sky_L) else np.asarray(sky_L, np.float32)
    sd = np.asarray(sun_dir, dtype=np.float64)
    sd = (sd / np.linalg.norm(sd)).astype(np.float32)
    if pos:
        P, I, M = np.concatenate(pos), np.concatenate(idx), np.concatenate(mat)
    else:
        P, I, M = (np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32),
                   np.zeros(0, np.int32))
    vt = None
    if vthick is not None:
        vt = np.full(len(P), vthick, dtype=np.float32) if np.isscalar(vthick) else vthick
    return Scene(pos=P, idx=I, mat=M, materials=materials, tab_lambda=LAM.copy(),
                 sun_dir=sd, sun_E=sE, sky_L=sL, vthick=vt)


def lambert(rho):
    return Material(LAMBERT, albedo=np.full(len(LAM), rho, dtype=np.float32))


def glass(n=1.52, k=1e-7, tint=0.0, thick=3.0, dispersive=False):
    nn = synth.cauchy_n(LAM, n, 0.0042) if dispersive else np.full(len(LAM), n, np.float32)
    return Material(GLASS, n=nn, k=np.full(len(LAM), k, np.float32),
                    alpha_tint=np.full(len(LAM), tint, np.float32), thick_mm=thick)


def settings(cam, lam=None, spp=4, max_depth=4, n_bands=1, seed=0, thr=0.0):
    lam = (400.0 + 20.0 * np.arange(16)).astype(np.float32) if lam is None else lam
    return RenderSettings(camera=cam, lambda_nm=lam, cmf=synth.cmf_xyz(lam), spp=spp,
                          max_depth=max_depth, seed=seed, n_bands=n_bands, beta_threshold=thr)


def ortho_down(z, height, W=32, H=32):
    return Camera(eye=(0.0, 0.0, z), target=(0.0, 0.0, z - 1.0), up=(0.0, 1.0, 0.0),
                  W=W, H=H, projection=1, ortho_height=height)


def bubbly(n=1.52, k=1e-7, tint=0.0, thick=3.0, density=20.0, rmin=10.0, rmax=200.0, pane_id=0,
           dispersive=False):
    g = glass(n, k, tint, thick, dispersive)
    g.type = synth.GLASS_BUBBLY
    g.bubble_density = density
    g.bubble_rmin_um = rmin
    g.bubble_rmax_um = rmax
    g.pane_id = pane_id
    return g


def constant_net(n_panes, R, T, w):
    """Network parameters whose output is (R, T, w) for every input: zero
    weights and the output biases that give those heads."""
    from paper_1912_05494_amd import surrogate
    p = np.zeros(surrogate.n_params(n_panes), dtype=np.float64)
    s = surrogate.split(p, n_panes)
    rest = 1.0 - R - T
    s["b4"][:] = [np.log(R / rest), np.log(T / rest), np.log(np.expm1(w))]
    return p
