"""Seeded synthetic inputs for the spectral path tracer.

This module only *makes inputs*: procedural geometry, optical-constant tables,
light spectra, colour-matching tables and render settings.  It holds none of
the rendering arithmetic (no intersection, Fresnel, absorption, sampling or
colour conversion), so both the CPU oracle and the HIP path can consume it.

The paper's own scene (the Royaumont abbey church) and its measured glasses
are not available; the generators below stand in for them with the same
structure the paper describes: a naturally lit church interior (sun plus sky,
eq. (3) and Sec. 3.1), glass panes carrying optical constants n + ik (eq. (1))
with per-location thickness and optical-constant maps (Sec. 6), and the
81-sample 380-780 nm spectral grid (Sec. 4).

All geometry and tables are stored as float32 so that the float32 GPU inputs
and the float64 oracle inputs are the same numbers.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

LAMBERT = 0
GLASS = 1
GLASS_BUBBLY = 2

#: The 81-sample visible grid of Sec. 4 (380 to 780 nm, 5 nm step).
LAMBDA_81 = (380.0 + 5.0 * np.arange(81)).astype(np.float32)


# ----------------------------------------------------------------------------
# Spectra (inputs only)
# ----------------------------------------------------------------------------
def planck(lam_nm, temp_k):
    """Black-body spectral radiance shape B(lambda, T) (arbitrary scale)."""
    lam = np.asarray(lam_nm, dtype=np.float64) * 1e-9
    c2 = 1.4387769e-2  # m K
    return 1.0 / (lam ** 5 * np.expm1(c2 / (lam * temp_k)))


def sun_irradiance(lam_nm):
    """Sun spectral irradiance: pi * B(l, 5778 K) / B(560 nm, 5778 K)."""
    return (math.pi * planck(lam_nm, 5778.0) / planck(560.0, 5778.0)).astype(np.float32)


def sky_radiance(lam_nm, scale=0.2):
    """Uniform sky radiance: scale * B(l, 12000 K) / B(560 nm, 12000 K)."""
    return (scale * planck(lam_nm, 12000.0) / planck(560.0, 12000.0)).astype(np.float32)


def _lobe(lam, mu, s1, s2):
    s = np.where(lam < mu, s1, s2)
    return np.exp(-0.5 * ((lam - mu) / s) ** 2)


def cmf_xyz(lam_nm):
    """Observer table (n, 3): the multi-lobe piecewise-Gaussian fit of the CIE
    1931 2-degree colour-matching functions published by Wyman, Sloan and
    Shirley (JCGT 2(2), 2013).  The CIE table itself is not available here;
    the renderer takes the observer as an input, so any smooth table works."""
    lam = np.asarray(lam_nm, dtype=np.float64)
    x = (1.056 * _lobe(lam, 599.8, 37.9, 31.0) + 0.362 * _lobe(lam, 442.0, 16.0, 26.7)
         - 0.065 * _lobe(lam, 501.1, 20.4, 26.2))
    y = 0.821 * _lobe(lam, 568.8, 46.9, 40.5) + 0.286 * _lobe(lam, 530.9, 16.3, 31.1)
    z = 1.217 * _lobe(lam, 437.0, 11.8, 36.0) + 0.681 * _lobe(lam, 459.0, 26.0, 13.8)
    return np.stack([x, y, z], axis=1).astype(np.float32)


def cauchy_n(lam_nm, a, b_um2):
    """n(lambda) = a + b / lambda^2 with lambda in micrometres."""
    lam_um = np.asarray(lam_nm, dtype=np.float64) * 1e-3
    return (a + b_um2 / lam_um ** 2).astype(np.float32)


def direction(elev_deg, azim_deg):
    """Unit vector at elevation/azimuth (azimuth from +y toward +x), float32."""
    e, a = math.radians(elev_deg), math.radians(azim_deg)
    v = np.array([math.cos(e) * math.sin(a), math.cos(e) * math.cos(a), math.sin(e)])
    return (v / np.linalg.norm(v)).astype(np.float32)


# ----------------------------------------------------------------------------
# Containers
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Material:
    type: int
    albedo: Optional[np.ndarray] = None      # [n_tab] (Lambert)
    n: Optional[np.ndarray] = None           # [n_tab] (glass)
    k: Optional[np.ndarray] = None           # [n_tab]
    alpha_tint: Optional[np.ndarray] = None  # [n_tab], mm^-1
    thick_mm: float = 3.0
    bubble_density: float = 0.0              # bubbles per mm^3
    bubble_rmin_um: float = 10.0
    bubble_rmax_um: float = 200.0
    pane_id: int = 0
    dist_map: int = 0                   # clear glass: 1 + index of its distribution map, 0 none


@dataclasses.dataclass
class DistMap:
    """Distribution map (Sec. 6): W x H texels over texture space [0, 1]^2,
    row 0 at t = 0; per texel a clear-glass material index and optionally a
    thickness (mm)."""
    W: int
    H: int
    material: np.ndarray                # (H, W) int32
    thick_mm: Optional[np.ndarray] = None   # (H, W) float32 or None


@dataclasses.dataclass
class Scene:
    pos: np.ndarray            # (nv, 3) float32, metres
    idx: np.ndarray            # (nt, 3) int32
    mat: np.ndarray            # (nt,) int32
    materials: List[Material]
    tab_lambda: np.ndarray     # (n_tab,) float32, nm
    sun_dir: np.ndarray        # (3,) float32, unit vector toward the sun
    sun_E: np.ndarray          # (n_tab,) float32
    sky_L: np.ndarray          # (n_tab,) float32
    vthick: Optional[np.ndarray] = None  # (nv,) float32 mm, or None
    uv: Optional[np.ndarray] = None      # (nv, 2) float32 texture coordinates, or None
    maps: list = dataclasses.field(default_factory=list)   # DistMap

    @property
    def nt(self):
        return int(self.idx.shape[0])


@dataclasses.dataclass
class Camera:
    eye: tuple
    target: tuple
    up: tuple = (0.0, 0.0, 1.0)
    vfov_deg: float = 40.0
    W: int = 64
    H: int = 64
    projection: int = 0        # 0 = pinhole, 1 = orthographic
    ortho_height: float = 1.0  # view height in metres for orthographic

    def __post_init__(self):
        # the library's camera is single precision: hold the values it will
        # see, so that every consumer (the library in FP32 or FP64, a
        # reference in double) starts from the same camera
        f32 = lambda v: float(np.float32(v))
        self.eye = tuple(f32(v) for v in self.eye)
        self.target = tuple(f32(v) for v in self.target)
        self.up = tuple(f32(v) for v in self.up)
        self.vfov_deg = f32(self.vfov_deg)
        self.ortho_height = f32(self.ortho_height)


@dataclasses.dataclass
class RenderSettings:
    camera: Camera
    lambda_nm: np.ndarray      # (n_lambda,) float32
    cmf: np.ndarray            # (n_lambda, 3) float32
    spp: int = 4
    max_depth: int = 4
    seed: int = 0
    n_bands: int = 1
    beta_threshold: float = 0.0
    job_id: int = 0


def flat_table(value, n=81):
    return np.full(n, value, dtype=np.float32)


# ----------------------------------------------------------------------------
# Mesh helpers
# ----------------------------------------------------------------------------
class _Mesh:
    def __init__(self):
        self.pos, self.idx, self.mat, self.uv = [], [], [], []
        self.nv = 0

    def grid(self, origin, ax_u, ax_v, nu, nv_, material, keep=None):
        """Quad grid origin + i/nu*ax_u + j/nv*ax_v; keep(i, j) filters cells."""
        o, a, b = (np.asarray(x, dtype=np.float64) for x in (origin, ax_u, ax_v))
        ii, jj = np.meshgrid(np.arange(nu + 1), np.arange(nv_ + 1), indexing="ij")
        p = o + ii[..., None] / nu * a + jj[..., None] / nv_ * b
        base = self.nv
        self.pos.append(p.reshape(-1, 3))
        self.uv.append(np.stack([ii / nu, jj / nv_], -1).reshape(-1, 2))
        self.nv += (nu + 1) * (nv_ + 1)
        vid = lambda i, j: base + i * (nv_ + 1) + j
        tris = []
        for i in range(nu):
            for j in range(nv_):
                if keep is not None and not keep(i, j):
                    continue
                a0, a1, a2, a3 = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
                tris.append((a0, a1, a2))
                tris.append((a0, a2, a3))
        if tris:
            self.idx.append(np.asarray(tris, dtype=np.int64))
            self.mat.append(np.full(len(tris), material, dtype=np.int64))
        return base

    def param(self, fn, nu, nv_, material):
        """Parametric surface fn(s, t) -> xyz over s, t in [0, 1]."""
        s = np.arange(nu + 1) / nu
        t = np.arange(nv_ + 1) / nv_
        ss, tt = np.meshgrid(s, t, indexing="ij")
        p = fn(ss, tt)
        base = self.nv
        self.pos.append(p.reshape(-1, 3))
        self.uv.append(np.stack([ss, tt], -1).reshape(-1, 2))
        self.nv += (nu + 1) * (nv_ + 1)
        i, j = np.meshgrid(np.arange(nu), np.arange(nv_), indexing="ij")
        a0 = base + i * (nv_ + 1) + j
        a1 = a0 + (nv_ + 1)
        a2 = a1 + 1
        a3 = a0 + 1
        t1 = np.stack([a0, a1, a2], -1).reshape(-1, 3)
        t2 = np.stack([a0, a2, a3], -1).reshape(-1, 3)
        tri = np.stack([t1, t2], 1).reshape(-1, 3)
        self.idx.append(tri)
        self.mat.append(np.full(len(tri), material, dtype=np.int64))

    def arrays(self):
        pos = np.concatenate(self.pos).astype(np.float32)
        idx = np.concatenate(self.idx).astype(np.int32)
        mat = np.concatenate(self.mat).astype(np.int32)
        return pos, idx, mat

    def uv_array(self):
        """Texture coordinates of every vertex: a grid's or a parametric
        surface's own (s, t) in [0, 1]^2."""
        return np.concatenate(self.uv).astype(np.float32)


# ----------------------------------------------------------------------------
# Configurations
# ----------------------------------------------------------------------------
def tiny_scene(bubbly=False, bubble_density=20.0):
    """Floor quad (Lambert 0.5) at z = 0, x, y in [-1, 1]; glass quad at
    z = 0.5, x, y in [-0.5, 0.5], 3 mm, n = 1.52 + 0.0042/l^2, k = 1e-7.
    Sun at elevation 60 deg, azimuth 30 deg; uniform sky."""
    lam = LAMBDA_81
    pos = np.array([[-1, -1, 0], [1, -1, 0], [1, 1, 0], [-1, 1, 0],
                    [-.5, -.5, .5], [.5, -.5, .5], [.5, .5, .5], [-.5, .5, .5]],
                   dtype=np.float32)
    idx = np.array([[0, 1, 2], [0, 2, 3], [4, 5, 6], [4, 6, 7]], dtype=np.int32)
    mat = np.array([0, 0, 1, 1], dtype=np.int32)
    floor = Material(LAMBERT, albedo=flat_table(0.5))
    glass = Material(GLASS_BUBBLY if bubbly else GLASS,
                     n=cauchy_n(lam, 1.52, 0.0042), k=flat_table(1e-7),
                     alpha_tint=flat_table(0.0), thick_mm=3.0,
                     bubble_density=bubble_density if bubbly else 0.0, pane_id=0)
    return Scene(pos=pos, idx=idx, mat=mat, materials=[floor, glass], tab_lambda=lam.copy(),
                 sun_dir=direction(60.0, 30.0), sun_E=sun_irradiance(lam),
                 sky_L=sky_radiance(lam), vthick=np.full(8, 3.0, dtype=np.float32))


def tiny_settings(spp=4, W=64, H=64, max_depth=4, n_bands=1, seed=0):
    lam = (400.0 + 20.0 * np.arange(16)).astype(np.float32)
    cam = Camera(eye=(0.0, -2.5, 1.8), target=(0.0, 0.0, 0.2), vfov_deg=40.0, W=W, H=H)
    return RenderSettings(camera=cam, lambda_nm=lam, cmf=cmf_xyz(lam), spp=spp,
                          max_depth=max_depth, seed=seed, n_bands=n_bands)


def random_glass(rng, lam):
    """Per-pane optical constants: smooth Cauchy n(l) within [1.50, 1.58],
    k log-uniform in [1e-7, 1e-5], Gaussian tint absorption band."""
    n0 = rng.uniform(1.50, 1.56)
    b = rng.uniform(0.0, (1.58 - n0) * 0.38 ** 2)
    k = 10.0 ** rng.uniform(-7.0, -5.0)
    a = rng.uniform(0.0, 0.5)
    mu = rng.uniform(400.0, 700.0)
    sg = rng.uniform(20.0, 80.0)
    lam64 = lam.astype(np.float64)
    tint = (a * np.exp(-0.5 * ((lam64 - mu) / sg) ** 2)).astype(np.float32)
    return cauchy_n(lam, n0, b), flat_table(k, len(lam)), tint


def stained_glass_palette(rng, lam, n_tiles=6):
    """Glasses of a Cistercian window (Sec. 6): nearly clear tile glasses (n0
    in [1.50, 1.56], weak tints) and one yellow glass for the edgings (a
    strong absorption band at 440 nm).  Returns a list of (n, k, tint)."""
    lam64 = lam.astype(np.float64)
    out = []
    for _ in range(n_tiles):
        n0 = rng.uniform(1.50, 1.56)
        k = 10.0 ** rng.uniform(-7.0, -6.0)
        a, mu, sg = rng.uniform(0.0, 0.15), rng.uniform(400.0, 700.0), rng.uniform(40.0, 120.0)
        out.append((cauchy_n(lam, n0, 0.0042), flat_table(k, len(lam)),
                    (a * np.exp(-0.5 * ((lam64 - mu) / sg) ** 2)).astype(np.float32)))
    yellow = (2.5 * np.exp(-0.5 * ((lam64 - 440.0) / 45.0) ** 2)).astype(np.float32)
    out.append((cauchy_n(lam, 1.53, 0.0042), flat_table(1e-6, len(lam)), yellow))
    return out


def stained_glass_map(rng, first_material, n_tiles, W=6, H=16, thick=(2.0, 5.0)):
    """One pane's distribution map: a border of yellow-edging texels around
    tiles drawn from the n_tiles tile glasses (materials first_material ..
    first_material + n_tiles - 1; the yellow glass follows them), each texel
    with its own thickness."""
    mat = first_material + rng.integers(0, n_tiles, size=(H, W))
    mat[0, :] = mat[-1, :] = first_material + n_tiles
    mat[:, 0] = mat[:, -1] = first_material + n_tiles
    th = rng.uniform(*thick, size=(H, W)).astype(np.float32)
    return DistMap(W=W, H=H, material=mat.astype(np.int32), thick_mm=th)


def nave_scene(seed=1, target_tris=40000, windows_per_side=12, panes_per_window=1,
               pane_grid=10, bubbly=False, rho_max=34.0, sun_elev=35.0, sun_azim=15.0, rho_min=0.0,
               bubble_free=False, glass_types=None, dist_maps=False):
    """Procedural church nave, 60 x 12 x 20 m: floor, side walls with window
    openings (1.5 x 4 m), semicircular barrel vault, end walls and two rows of
    ten cylindrical columns; glass panes fill the openings.  Opaque parts are
    gray Lambert groups with albedo in [0.3, 0.7].  Panes are quad grids with
    per-vertex thickness in [2, 5] mm and per-pane optical constants.
    bubbly: panes carry air bubbles of density U(rho_min, rho_max) per mm^3;
    bubble_free (with bubbly): the same scene with every pane a clear slab
    (the draws are the same, the bubbles are left out).  glass_types: None
    gives every pane its own glass (n, k, tint); an integer draws that many
    glasses and pane p takes glass p mod glass_types (its pane type), keeping
    its own density and thickness map.  Each pane is a pane_grid x pane_grid
    quad grid.  dist_maps (clear glass): every pane takes its optical
    constants and thickness from its own stained-glass distribution map
    (tiles of six nearly clear glasses with a yellow edging, Sec. 6), looked
    up through the pane's texture coordinates; the other draws are unchanged."""
    rng = np.random.default_rng(seed)
    lam = LAMBDA_81
    L, Wd, Hw, R = 60.0, 12.0, 14.0, 6.0
    f = math.sqrt(target_tris / 40000.0)
    mx = max(1, int(round(f)))                      # x subdivisions per 0.25 m
    rz = max(2, int(round(14 * f)))                 # wall rows
    wall_rows = rz
    spacing = L / windows_per_side
    win_w, win_z0, win_z1 = 1.5, 6.0, 10.0
    mesh = _Mesh()
    # materials: 0 floor, 1 walls, 2 vault, 3 end walls, 4 columns, then panes
    mats = [Material(LAMBERT, albedo=flat_table(rng.uniform(0.3, 0.7))) for _ in range(5)]
    # floor
    nfx, nfy = max(2, int(round(120 * f))), max(2, int(round(24 * f)))
    mesh.grid((0, 0, 0), (L, 0, 0), (0, Wd, 0), nfx, nfy, 0)
    # side walls with openings.  The wall is cut into columns of width 0.25/mx.
    ncx = int(round(L / 0.25)) * mx
    cx = L / ncx
    z_edges = np.unique(np.concatenate([np.linspace(0, Hw, wall_rows + 1), [win_z0, win_z1]]))
    centres = spacing * (np.arange(windows_per_side) + 0.5)

    def in_window(x0, x1, z0, z1):
        xm, zm = 0.5 * (x0 + x1), 0.5 * (z0 + z1)
        if not (win_z0 < zm < win_z1):
            return False
        return bool(np.any(np.abs(xm - centres) < win_w / 2))

    for y in (0.0, Wd):
        tris_pos = []
        for i in range(ncx):
            x0, x1 = i * cx, (i + 1) * cx
            for j in range(len(z_edges) - 1):
                z0, z1 = z_edges[j], z_edges[j + 1]
                if in_window(x0, x1, z0, z1):
                    continue
                tris_pos.append(((x0, y, z0), (x1, y, z0), (x1, y, z1)))
                tris_pos.append(((x0, y, z0), (x1, y, z1), (x0, y, z1)))
        tp = np.asarray(tris_pos, dtype=np.float64).reshape(-1, 3)
        base = mesh.nv
        mesh.pos.append(tp)
        mesh.uv.append(np.zeros((len(tp), 2)))      # opaque walls carry no map
        mesh.nv += len(tp)
        mesh.idx.append(base + np.arange(len(tp)).reshape(-1, 3))
        mesh.mat.append(np.full(len(tp) // 3, 1))
    # barrel vault
    nvx, nva = max(2, int(round(120 * f))), max(4, int(round(32 * f)))
    mesh.param(lambda s, t: np.stack([L * s, Wd / 2 - R * np.cos(math.pi * t),
                                      Hw + R * np.sin(math.pi * t)], -1), nvx, nva, 2)
    # end walls
    ney, nez = max(2, int(round(24 * f))), max(2, int(round(40 * f)))
    for x in (0.0, L):
        mesh.grid((x, 0, 0), (0, Wd, 0), (0, 0, Hw + R), ney, nez, 3)
    # columns
    nseg, nring = max(6, int(round(24 * f))), max(2, int(round(10 * f)))
    for row_y in (3.0, 9.0):
        for c in range(10):
            xc = 3.5 + 5.5 * c
            mesh.param(lambda s, t, xc=xc, yc=row_y: np.stack(
                [xc + 0.4 * np.cos(2 * math.pi * s), yc + 0.4 * np.sin(2 * math.pi * s),
                 Hw * t], -1), nseg, nring, 4)
    # panes
    pane_mat0 = len(mats)
    n_opaque = sum(len(t) for t in mesh.idx)
    vthick_parts = [np.zeros(mesh.nv)]
    pane = 0
    glasses = [random_glass(rng, lam) for _ in range(glass_types)] if glass_types else None
    for y in (0.0, Wd):
        for xc in centres:
            h = (win_z1 - win_z0) / panes_per_window
            for q in range(panes_per_window):
                if glasses is None:
                    nn, kk, tint = random_glass(rng, lam)
                    ptype = pane
                else:
                    ptype = pane % glass_types
                    nn, kk, tint = glasses[ptype]
                rho = float(rng.uniform(rho_min, rho_max)) if bubbly else 0.0
                m = Material(GLASS_BUBBLY if bubbly and not bubble_free else GLASS, n=nn, k=kk,
                             alpha_tint=tint, thick_mm=3.5, pane_id=ptype,
                             bubble_density=0.0 if bubble_free else rho)
                mats.append(m)
                v0 = mesh.nv
                gu = gv = pane_grid
                mesh.grid((xc - win_w / 2, y, win_z0 + q * h), (win_w, 0, 0), (0, 0, h),
                          gu, gv, pane_mat0 + pane)
                vthick_parts.append(rng.uniform(2.0, 5.0, size=mesh.nv - v0))
                pane += 1
    pos, idx, mat = mesh.arrays()
    vthick = np.concatenate(vthick_parts).astype(np.float32)
    assert vthick.shape[0] == pos.shape[0]
    scene = Scene(pos=pos, idx=idx, mat=mat, materials=mats, tab_lambda=lam.copy(),
                  sun_dir=direction(sun_elev, 180.0 - sun_azim), sun_E=sun_irradiance(lam),
                  sky_L=sky_radiance(lam), vthick=vthick)
    if dist_maps and not bubbly:
        # a separate stream, so that the scene's other draws stay as they are
        mrng = np.random.default_rng(seed + 7919)
        first = len(mats)
        palette = stained_glass_palette(mrng, lam)
        for nn, kk, tint in palette:
            mats.append(Material(GLASS, n=nn, k=kk, alpha_tint=tint, thick_mm=3.5))
        for q in range(pane):
            scene.maps.append(stained_glass_map(mrng, first, len(palette) - 1))
            mats[pane_mat0 + q].dist_map = q + 1
        scene.uv = mesh.uv_array()
    scene.n_opaque = n_opaque
    return scene


def large_scene(seed=5, bubbly=True, bubble_free=False):
    """The large nave: about 1 M triangles; 25 windows a side of 4 panes,
    200 bubbly panes of 200 triangles (10 x 10 quads) with per-vertex
    thickness in [2, 5] mm, each with its own bubble density U(0, 34) per
    mm^3 and one of 40 glass types."""
    return nave_scene(seed=seed, target_tris=1_000_000, windows_per_side=25, panes_per_window=4, pane_grid=10,
                      bubbly=bubbly, bubble_free=bubble_free, glass_types=40)


def large_settings(spp=256, max_depth=12, seed=0):
    """1920 x 1080, 81 wavelengths, 256 spp, depth 12."""
    return nave_settings(W=1920, H=1080, spp=spp, max_depth=max_depth, seed=seed)


def nave_settings(W=512, H=512, spp=64, max_depth=8, n_bands=1, seed=0, n_lambda=81):
    lam = np.linspace(380.0, 780.0, n_lambda).astype(np.float32)
    cam = Camera(eye=(2.0, 6.0, 1.7), target=(40.0, 6.0, 7.0), vfov_deg=60.0, W=W, H=H)
    return RenderSettings(camera=cam, lambda_nm=lam, cmf=cmf_xyz(lam), spp=spp,
                          max_depth=max_depth, seed=seed, n_bands=n_bands)


def batch_jobs(n_jobs=32, seed=2, scale=1.0):
    """Uneven batch: square side in [128, 1024], 10k-200k triangles, 8-81
    wavelengths evenly spaced in 380-780 nm, 16-128 spp.  ``scale`` shrinks
    image sides and triangle counts for small test batches."""
    rng = np.random.default_rng(seed)
    jobs = []
    for j in range(n_jobs):
        side = int(rng.integers(128, 1025) * scale)
        tris = int(rng.integers(10000, 200001) * scale * scale)
        nl = int(rng.integers(8, 82))
        spp = int(rng.integers(16, 129))
        sc = nave_scene(seed=2 + j, target_tris=max(2000, tris))
        st = nave_settings(W=max(8, side), H=max(8, side), spp=spp, n_lambda=nl)
        st.job_id = j
        jobs.append((sc, st))
    return jobs


def random_soup(seed, n_tris=32, n_glass=8, extent=1.0):
    """Random triangle soup for intersection tests (float32 vertices)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-extent, extent, size=(n_tris, 1, 3))
    pos = (c + rng.normal(scale=0.3 * extent, size=(n_tris, 3, 3))).reshape(-1, 3)
    idx = np.arange(3 * n_tris, dtype=np.int32).reshape(-1, 3)
    mat = np.zeros(n_tris, dtype=np.int32)
    mat[:n_glass] = 1
    lam = LAMBDA_81
    mats = [Material(LAMBERT, albedo=flat_table(0.6)),
            Material(GLASS, n=cauchy_n(lam, 1.52, 0.0042), k=flat_table(1e-6),
                     alpha_tint=flat_table(0.05), thick_mm=3.0)]
    return Scene(pos=pos.astype(np.float32), idx=idx, mat=mat, materials=mats,
                 tab_lambda=lam.copy(), sun_dir=direction(50.0, 20.0),
                 sun_E=sun_irradiance(lam), sky_L=sky_radiance(lam),
                 vthick=rng.uniform(2.0, 5.0, size=3 * n_tris).astype(np.float32))


def random_rays(seed, n, extent=1.5):
    """Random ray origins in a box and unit directions (float32)."""
    rng = np.random.default_rng(seed)
    o = rng.uniform(-extent, extent, size=(n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)
