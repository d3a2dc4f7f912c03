"""ctypes binding of the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import ensure_built

__all__ = ["lib", "OracleScene", "philox", "u01", "fresnel", "slab", "snell_cos_t",
           "render", "render_pixels", "spec_to_xyz", "camera_ray", "cosine_dir", "slab_mc",
           "fresnel_real", "bubble_dir", "mlp_nparams", "mlp_forward", "mlp_loss_grad", "walk_draw",
           "bubbly_walk", "bubble_sigma", "bf16", "mlp_forward_bf16", "lobe_dir", "lobe_transmit", "mlp_bf16_bound", "pane_at", "photon_map", "slab_to_world",
           "BTDF_MODES"]

_lib = None


class _Material(C.Structure):
    _fields_ = [("type", C.c_int32), ("thick_mm", C.c_double), ("bubble_density", C.c_double),
                ("bubble_rmin_um", C.c_double), ("bubble_rmax_um", C.c_double),
                ("pane_id", C.c_int32),
                ("albedo", C.POINTER(C.c_double)), ("n", C.POINTER(C.c_double)),
                ("k", C.POINTER(C.c_double)), ("alpha_tint", C.POINTER(C.c_double)),
                ("dist_map", C.c_int32)]


class _DistMap(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("material", C.POINTER(C.c_int32)),
                ("thick_mm", C.POINTER(C.c_double))]


class _SceneDesc(C.Structure):
    _fields_ = [("nv", C.c_int32), ("pos", C.POINTER(C.c_double)),
                ("vthick_mm", C.POINTER(C.c_double)), ("nt", C.c_int32),
                ("idx", C.POINTER(C.c_int32)), ("mat", C.POINTER(C.c_int32)),
                ("n_mat", C.c_int32), ("mats", C.POINTER(_Material)), ("n_tab", C.c_int32),
                ("tab_lambda_nm", C.POINTER(C.c_double)), ("sun_dir", C.c_double * 3),
                ("sun_E", C.POINTER(C.c_double)), ("sky_L", C.POINTER(C.c_double)),
                ("uv", C.POINTER(C.c_double)), ("n_maps", C.c_int32), ("maps", C.POINTER(_DistMap))]


class _Params(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("spp", C.c_int32), ("max_depth", C.c_int32),
                ("projection", C.c_int32), ("eye", C.c_double * 3), ("target", C.c_double * 3),
                ("up", C.c_double * 3), ("vfov_deg", C.c_double), ("ortho_height", C.c_double),
                ("seed", C.c_uint64), ("job_id", C.c_uint32), ("n_lambda", C.c_int32),
                ("lambda_nm", C.POINTER(C.c_double)), ("cmf_xyz", C.POINTER(C.c_double)),
                ("n_bands", C.c_int32), ("tile", C.c_int32), ("beta_threshold", C.c_double),
                ("use_bvh", C.c_int32), ("n_threads", C.c_int32),
                ("btdf_mode", C.c_int32), ("mlp_n_panes", C.c_int32), ("mlp_bf16", C.c_int32),
                ("err_dims", C.c_int32 * 3), ("mlp_params", C.POINTER(C.c_double)),
                ("err_table", C.POINTER(C.c_double)), ("err_bound", C.c_double),
                ("item_begin", C.c_int64), ("max_items", C.c_int64), ("events", C.c_void_p),
                ("prec_bound", C.c_void_p), ("prec_rel", C.c_double), ("prec_ceps", C.c_double),
                ("prec_eps", C.c_double), ("photons", C.c_int64), ("photon_radius", C.c_double)]


class _WalkStream(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("c0", C.c_uint32), ("c1", C.c_uint32), ("c3", C.c_uint32),
                ("vertex", C.c_uint32), ("render", C.c_int32)]


class _WalkOut(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dir", C.c_double * 3), ("L", C.c_double), ("n_events", C.c_int32),
                ("bubbles", C.c_int32)]


BTDF_MODES = {"exact": 0, "surrogate": 1, "fallback": 2}


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32)) if a is not None else None


def lib():
    global _lib
    if _lib is None:
        so = ensure_built()
        L = C.CDLL(so)
        L.orc_philox_batch.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_u01.restype = C.c_double
        L.orc_u01.argtypes = [C.c_uint32]
        L.orc_fresnel.argtypes = [C.c_double] * 3 + [C.POINTER(C.c_double)] * 2
        L.orc_slab_batch.argtypes = [C.c_int64] + [C.c_void_p] * 8
        L.orc_snell_cos_t.restype = C.c_double
        L.orc_snell_cos_t.argtypes = [C.c_double, C.c_double]
        L.orc_scene_create.restype = C.c_void_p
        L.orc_scene_create.argtypes = [C.POINTER(_SceneDesc)]
        L.orc_scene_destroy.argtypes = [C.c_void_p]
        L.orc_scene_teps.restype = C.c_double
        L.orc_scene_teps.argtypes = [C.c_void_p]
        L.orc_bvh_depth.restype = C.c_int32
        L.orc_bvh_depth.argtypes = [C.c_void_p]
        L.orc_intersect.argtypes = [C.c_void_p, C.c_int32, C.c_int64] + [C.c_void_p] * 7
        L.orc_shadow.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p,
                                 C.c_double, C.c_void_p]
        L.orc_render.restype = C.c_int
        L.orc_render.argtypes = [C.c_void_p, C.POINTER(_Params), C.c_void_p, C.c_void_p]
        L.orc_render_pixels.restype = C.c_int
        L.orc_render_pixels.argtypes = [C.c_void_p, C.POINTER(_Params), C.c_int64, C.c_void_p,
                                        C.c_void_p]
        L.orc_camera_ray.argtypes = [C.POINTER(_Params), C.c_int32, C.c_int32, C.c_double,
                                     C.c_double, C.c_void_p, C.c_void_p]
        L.orc_cosine_dir.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_void_p]
        L.orc_spec_to_xyz.argtypes = [C.c_int64, C.c_int32] + [C.c_void_p] * 4
        L.orc_slab_mc.argtypes = ([C.c_int64] + [C.c_void_p] * 4 + [C.c_double] * 2 + [C.c_void_p] * 4
                                  + [C.c_uint64, C.c_uint32, C.c_int32] + [C.c_void_p] * 4)
        L.orc_walk_draw.argtypes = [C.POINTER(_WalkStream), C.c_uint32, C.c_uint32, C.c_void_p]
        L.orc_bubbly_walk.argtypes = [C.POINTER(_WalkStream)] + [C.c_double] * 4 + [C.c_int,
                                                                                  C.POINTER(_WalkOut)]
        L.orc_bubble_sigma.restype = C.c_double
        L.orc_bubble_sigma.argtypes = [C.c_double] * 3
        L.orc_mlp_forward_bf16.argtypes = [C.c_void_p, C.c_int32, C.c_int64] + [C.c_void_p] * 3
        L.orc_bf16.restype = C.c_double
        L.orc_bf16.argtypes = [C.c_double]
        L.orc_lobe_dir.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_void_p]
        L.orc_lobe_transmit.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_void_p]
        L.orc_pane_at.argtypes = [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_void_p, C.c_void_p]
        L.orc_photon_map.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_photon_map.restype = C.c_int64
        L.orc_mlp_bf16_bound.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_void_p,
                                         C.c_void_p]
        L.orc_slab_to_world.argtypes = [C.c_void_p] * 4
        L.orc_fresnel_real.restype = C.c_double
        L.orc_fresnel_real.argtypes = [C.c_double] * 3 + [C.c_int]
        L.orc_bubble_dir.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_int, C.c_void_p]
        L.orc_mlp_nparams.restype = C.c_int64
        L.orc_mlp_nparams.argtypes = [C.c_int32]
        L.orc_mlp_forward.argtypes = [C.c_void_p, C.c_int32, C.c_int64] + [C.c_void_p] * 3
        L.orc_mlp_loss_grad.restype = C.c_double
        L.orc_mlp_loss_grad.argtypes = [C.c_void_p, C.c_int32, C.c_int64] + [C.c_void_p] * 4
        _lib = L
    return _lib


# ----------------------------------------------------------------------------
def philox(ctr, key):
    """ctr: (n, 4) uint32, key: (n, 2) uint32 -> (n, 4) uint32."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    out = np.empty_like(ctr)
    lib().orc_philox_batch(len(ctr), ctr.ctypes.data, key.ctypes.data, out.ctypes.data)
    return out


def u01(x):
    return lib().orc_u01(int(x))


def fresnel(cos_i, n, k):
    rs, rp = C.c_double(), C.c_double()
    lib().orc_fresnel(float(cos_i), float(n), float(k), C.byref(rs), C.byref(rp))
    return rs.value, rp.value


def snell_cos_t(cos_i, n):
    return lib().orc_snell_cos_t(float(cos_i), float(n))


def slab(cos_i, lambda_nm, d_mm, n, k, alpha_tint):
    """Vectorised thin-slab (R, T); arguments broadcast."""
    arrs = np.broadcast_arrays(*[np.asarray(a, dtype=np.float64) for a in
                                 (cos_i, lambda_nm, d_mm, n, k, alpha_tint)])
    shape = arrs[0].shape
    flat = [np.ascontiguousarray(a.reshape(-1)) for a in arrs]
    R = np.empty(flat[0].size)
    T = np.empty(flat[0].size)
    lib().orc_slab_batch(flat[0].size, *[a.ctypes.data for a in flat], R.ctypes.data, T.ctypes.data)
    return R.reshape(shape), T.reshape(shape)


class OracleScene:
    """Owns the C scene; arrays are converted to float64 (exact for float32)."""

    def __init__(self, scene):
        self._keep = []
        f64 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
        pos = f64(scene.pos.reshape(-1))
        vth = f64(scene.vthick)
        idx = np.ascontiguousarray(scene.idx.reshape(-1), dtype=np.int32)
        mat = np.ascontiguousarray(scene.mat, dtype=np.int32)
        tab = f64(scene.tab_lambda)
        mats = (_Material * max(1, len(scene.materials)))()
        for i, m in enumerate(scene.materials):
            arrs = [f64(m.albedo), f64(m.n), f64(m.k), f64(m.alpha_tint)]
            self._keep += arrs
            mats[i] = _Material(m.type, float(m.thick_mm), float(m.bubble_density),
                                float(m.bubble_rmin_um), float(m.bubble_rmax_um), int(m.pane_id),
                                *[_dp(a) for a in arrs], int(getattr(m, "dist_map", 0)))
        sunE, skyL = f64(scene.sun_E), f64(scene.sky_L)
        uv = f64(None if getattr(scene, "uv", None) is None else np.asarray(scene.uv).reshape(-1))
        smaps = list(getattr(scene, "maps", []) or [])
        maps = (_DistMap * max(1, len(smaps)))()
        for i, dm in enumerate(smaps):
            tm = np.ascontiguousarray(np.asarray(dm.material).reshape(-1), dtype=np.int32)
            th = f64(None if dm.thick_mm is None else np.asarray(dm.thick_mm).reshape(-1))
            self._keep += [tm, th]
            maps[i] = _DistMap(int(dm.W), int(dm.H), _ip(tm), _dp(th))
        self._keep += [pos, vth, idx, mat, tab, mats, sunE, skyL, uv, maps]
        d = _SceneDesc(len(scene.pos), _dp(pos), _dp(vth), int(scene.idx.shape[0]), _ip(idx),
                       _ip(mat), len(scene.materials), mats, len(tab), _dp(tab),
                       (C.c_double * 3)(*[float(x) for x in scene.sun_dir]), _dp(sunE), _dp(skyL),
                       _dp(uv), len(smaps), maps)
        self.ptr = lib().orc_scene_create(C.byref(d))
        if not self.ptr:
            raise ValueError("oracle rejected the scene description")
        self.nt = int(scene.idx.shape[0])

    def __del__(self):
        if getattr(self, "ptr", None):
            lib().orc_scene_destroy(self.ptr)
            self.ptr = None

    @property
    def teps(self):
        return lib().orc_scene_teps(self.ptr)

    @property
    def bvh_depth(self):
        return lib().orc_bvh_depth(self.ptr)

    def intersect(self, o, d, skip=None, use_bvh=True):
        o = np.ascontiguousarray(o, dtype=np.float64).reshape(-1, 3)
        d = np.ascontiguousarray(d, dtype=np.float64).reshape(-1, 3)
        m = len(o)
        sk = None if skip is None else np.ascontiguousarray(skip, dtype=np.int32)
        t = np.empty(m)
        tri = np.empty(m, dtype=np.int32)
        u = np.empty(m)
        v = np.empty(m)
        lib().orc_intersect(self.ptr, int(use_bvh), m, o.ctypes.data, d.ctypes.data,
                            None if sk is None else sk.ctypes.data, t.ctypes.data,
                            tri.ctypes.data, u.ctypes.data, v.ctypes.data)
        return t, tri, u, v

    def shadow(self, o, lambda_nm, skip=None, use_bvh=True):
        o = np.ascontiguousarray(o, dtype=np.float64).reshape(-1, 3)
        sk = None if skip is None else np.ascontiguousarray(skip, dtype=np.int32)
        T = np.empty(len(o))
        lib().orc_shadow(self.ptr, int(use_bvh), len(o), o.ctypes.data,
                         None if sk is None else sk.ctypes.data, float(lambda_nm), T.ctypes.data)
        return T


def _params(settings, use_bvh=True, tile=16, n_threads=0, n_bands=None, btdf=None, photons=0, photon_radius=0.05):
    """btdf: None (exact walks on bubbly panes) or a dict with keys mode
    ("exact" / "surrogate" / "fallback"), params, n_panes, bf16 (bool) and,
    for "fallback", err_table (n_panes, n_cos, n_d, n_rho) and bound."""
    cam = settings.camera
    lam = np.ascontiguousarray(settings.lambda_nm, dtype=np.float64)
    cmf = np.ascontiguousarray(settings.cmf, dtype=np.float64).reshape(-1)
    p = _Params(cam.W, cam.H, settings.spp, settings.max_depth, cam.projection,
                (C.c_double * 3)(*cam.eye), (C.c_double * 3)(*cam.target),
                (C.c_double * 3)(*cam.up), float(cam.vfov_deg), float(cam.ortho_height),
                int(settings.seed), int(settings.job_id), len(lam), _dp(lam), _dp(cmf),
                int(settings.n_bands if n_bands is None else n_bands), int(tile),
                float(settings.beta_threshold), int(use_bvh), int(n_threads))
    keep = [lam, cmf]
    p.photons = int(photons)
    p.photon_radius = float(photon_radius)
    if btdf is not None:
        p.btdf_mode = BTDF_MODES[btdf.get("mode", "exact")]
        if btdf.get("params") is not None:
            prm = np.ascontiguousarray(btdf["params"], dtype=np.float64)
            keep.append(prm)
            p.mlp_params = _dp(prm)
            p.mlp_n_panes = int(btdf["n_panes"])
            p.mlp_bf16 = int(bool(btdf.get("bf16", False)))
        if btdf.get("err_table") is not None:
            tab = np.ascontiguousarray(btdf["err_table"], dtype=np.float64)
            keep.append(tab)
            p.err_table = _dp(tab)
            p.err_dims = (C.c_int32 * 3)(*tab.shape[1:4])
            p.err_bound = float(btdf.get("bound", 1e-3))
    return p, keep


def render(oscene, settings, use_bvh=True, tile=16, n_threads=0, n_bands=None, btdf=None, items=None,
           events=False, spec=None, prec=None, photons=0, photon_radius=0.05):
    """Full image -> (spec (H, W, nl) float64, xyz (H, W, 3) float64), plus the
    event signatures (H, W, nl) uint64 when events is True, plus the
    single-precision error bound (H, W, nl) float64 when prec = (rel,
    cos_eps, pos_eps) is given (see orc_render_params).  items: (begin,
    count) of the work
    items to render (count 0: to the end); the others keep the values of
    spec (zeros when spec is None)."""
    p, keep = _params(settings, use_bvh, tile, n_threads, n_bands, btdf, photons, photon_radius)
    W, H, nl = settings.camera.W, settings.camera.H, len(settings.lambda_nm)
    spec = np.zeros((H, W, nl)) if spec is None else np.ascontiguousarray(spec, dtype=np.float64)
    xyz = np.empty((H, W, 3))
    ev = np.zeros((H, W, nl), dtype=np.uint64) if events else None
    pb = np.zeros((H, W, nl)) if prec is not None else None
    if items is not None:
        p.item_begin, p.max_items = int(items[0]), int(items[1])
    if ev is not None:
        p.events = ev.ctypes.data
    if pb is not None:
        p.prec_bound = pb.ctypes.data
        p.prec_rel, p.prec_ceps, p.prec_eps = (float(x) for x in prec)
    rc = lib().orc_render(oscene.ptr, C.byref(p), spec.ctypes.data, xyz.ctypes.data)
    if rc != 0:
        raise ValueError("oracle render rejected the parameters")
    return (spec, xyz) + ((ev,) if events else ()) + ((pb,) if pb is not None else ())


def render_pixels(oscene, settings, pixels, use_bvh=True, n_threads=0, btdf=None, events=False, prec=None,
                  photons=0, photon_radius=0.05):
    """Selected linear pixel indices -> spec (m, nl) float64, plus the event
    signatures (m, nl) uint64 when events is True and the single-precision
    error bound (m, nl) float64 when prec is given (as for render)."""
    p, keep = _params(settings, use_bvh, 16, n_threads, btdf=btdf, photons=photons, photon_radius=photon_radius)
    px = np.ascontiguousarray(pixels, dtype=np.int32)
    nl = len(settings.lambda_nm)
    spec = np.empty((len(px), nl))
    ev = np.zeros((len(px), nl), dtype=np.uint64) if events else None
    pb = np.zeros((len(px), nl)) if prec is not None else None
    if ev is not None:
        p.events = ev.ctypes.data
    if pb is not None:
        p.prec_bound = pb.ctypes.data
        p.prec_rel, p.prec_ceps, p.prec_eps = (float(x) for x in prec)
    rc = lib().orc_render_pixels(oscene.ptr, C.byref(p), len(px), px.ctypes.data, spec.ctypes.data)
    if rc != 0:
        raise ValueError("oracle render rejected the parameters")
    extra = ((ev,) if events else ()) + ((pb,) if pb is not None else ())
    return (spec,) + extra if extra else spec


def camera_ray(settings, i, j, u0, u1):
    p, keep = _params(settings)
    o = np.empty(3)
    d = np.empty(3)
    lib().orc_camera_ray(C.byref(p), int(i), int(j), float(u0), float(u1), o.ctypes.data,
                         d.ctypes.data)
    return o, d


def cosine_dir(n, u1, u2):
    n = np.ascontiguousarray(n, dtype=np.float64)
    d = np.empty(3)
    lib().orc_cosine_dir(n.ctypes.data, float(u1), float(u2), d.ctypes.data)
    return d


def slab_mc(cos_i, lambda_nm, d_mm, rho_b, n, k, alpha_tint, seed=0, tuple0=0, n_photons=64,
            rmin_um=10.0, rmax_um=200.0, n_ref=None):
    """Bubbly-slab Monte Carlo per tuple -> (R, T, A, w_lobe) float64 arrays.
    n_ref: index used inside the slab (default: n)."""
    arrs = np.broadcast_arrays(*[np.asarray(a, dtype=np.float64) for a in
                                 (cos_i, lambda_nm, d_mm, rho_b, n, k, alpha_tint,
                                  n if n_ref is None else n_ref)])
    flat = [np.ascontiguousarray(a.reshape(-1)) for a in arrs]
    m = flat[0].size
    R, T, A, W = (np.empty(m) for _ in range(4))
    lib().orc_slab_mc(m, *[a.ctypes.data for a in flat[:4]], float(rmin_um), float(rmax_um),
                      *[a.ctypes.data for a in flat[4:]], int(seed), int(tuple0), int(n_photons),
                      R.ctypes.data, T.ctypes.data, A.ctypes.data, W.ctypes.data)
    return R, T, A, W


def walk_draw(seed, c0, c1, event, sub, render=False, vertex=0, c3=0):
    st = _WalkStream(int(seed), int(c0), int(c1), int(c3), int(vertex), int(bool(render)))
    u = np.empty(4)
    lib().orc_walk_draw(C.byref(st), int(event), int(sub), u.ctypes.data)
    return u


def bubbly_walk(cos_i, d_mm, sigma, n_ref, pol, seed=0, c0=0, c1=0, render=False, vertex=0, c3=0):
    """One walk inside a bubbly slab -> (kind, direction (3,), length in glass)."""
    st = _WalkStream(int(seed), int(c0), int(c1), int(c3), int(vertex), int(bool(render)))
    out = _WalkOut()
    lib().orc_bubbly_walk(C.byref(st), float(cos_i), float(d_mm), float(sigma), float(n_ref), int(pol),
                          C.byref(out))
    return out.kind, np.array(out.dir[:]), out.L


def bubble_sigma(rho_b, rmin_um=10.0, rmax_um=200.0):
    return lib().orc_bubble_sigma(float(rho_b), float(rmin_um), float(rmax_um))


def bf16(x):
    return np.array([lib().orc_bf16(float(v)) for v in np.asarray(x, dtype=np.float64).reshape(-1)])


def mlp_forward_bf16(params, n_panes, tuples, panes):
    """The network with BF16 operands (inputs, weights, hidden activations)."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(tuples, dtype=np.float64).reshape(-1, 4)
    pn = np.ascontiguousarray(panes, dtype=np.int32)
    out = np.empty((len(x), 3))
    lib().orc_mlp_forward_bf16(p.ctypes.data, int(n_panes), len(x), x.ctypes.data, pn.ctypes.data,
                               out.ctypes.data)
    return out


def lobe_dir(d, w, u1, u2):
    d = np.ascontiguousarray(d, dtype=np.float64)
    out = np.empty(3)
    lib().orc_lobe_dir(d.ctypes.data, float(w), float(u1), float(u2), out.ctypes.data)
    return out


def mlp_bf16_bound(params, tup, pane, e_cos=0.0, e_d=0.0):
    """One tuple's BF16-operand outputs (R, T, w) and the bound on their
    distance from an FP32-sum evaluation with inputs off by e_cos, e_d."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    t = np.ascontiguousarray(tup, dtype=np.float64)
    out, bnd = np.empty(3), np.empty(3)
    lib().orc_mlp_bf16_bound(p.ctypes.data, t.ctypes.data, int(pane), float(e_cos), float(e_d), out.ctypes.data,
                             bnd.ctypes.data)
    return out, bnd


def photon_map(oscene, settings, photons, photon_radius=0.05, use_bvh=True):
    """Stored photons of the caustic map: (n, 8) rows (x, y, z, nx, ny, nz,
    power, wavelength index)."""
    p, keep = _params(settings, use_bvh, photons=photons, photon_radius=photon_radius)
    n = lib().orc_photon_map(oscene.ptr, C.byref(p), None)
    if n < 0:
        raise ValueError("oracle rejected the parameters")
    out = np.empty((max(n, 0), 8))
    lib().orc_photon_map(oscene.ptr, C.byref(p), out.ctypes.data if n > 0 else None)
    return out


def pane_at(oscene, t, u, v):
    """(material, thickness mm) of the pane of triangle t at barycentric (u, v)."""
    m = C.c_int32()
    d = C.c_double()
    lib().orc_pane_at(oscene.ptr, int(t), float(u), float(v), C.byref(m), C.byref(d))
    return int(m.value), float(d.value)


def lobe_transmit(d, ng, w, u1, u2):
    d = np.ascontiguousarray(d, dtype=np.float64)
    ng = np.ascontiguousarray(ng, dtype=np.float64)
    out = np.empty(3)
    lib().orc_lobe_transmit(d.ctypes.data, ng.ctypes.data, float(w), float(u1), float(u2), out.ctypes.data)
    return out


def slab_to_world(d, ng, a):
    d = np.ascontiguousarray(d, dtype=np.float64)
    ng = np.ascontiguousarray(ng, dtype=np.float64)
    a = np.ascontiguousarray(a, dtype=np.float64)
    out = np.empty(3)
    lib().orc_slab_to_world(d.ctypes.data, ng.ctypes.data, a.ctypes.data, out.ctypes.data)
    return out


def fresnel_real(n1, n2, c, pol):
    return lib().orc_fresnel_real(float(n1), float(n2), float(c), int(pol))


def bubble_dir(d, e_perp, sin_i, n, p):
    d = np.ascontiguousarray(d, dtype=np.float64)
    e = np.ascontiguousarray(e_perp, dtype=np.float64)
    out = np.empty(3)
    lib().orc_bubble_dir(d.ctypes.data, e.ctypes.data, float(sin_i), float(n), int(p), out.ctypes.data)
    return out


def mlp_nparams(n_panes):
    return int(lib().orc_mlp_nparams(int(n_panes)))


def mlp_forward(params, n_panes, tuples, panes):
    """tuples (m, 4): cos, lambda_nm, d_mm, rho_b -> (m, 3): R, T, w."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(tuples, dtype=np.float64).reshape(-1, 4)
    pn = np.ascontiguousarray(panes, dtype=np.int32)
    out = np.empty((len(x), 3))
    lib().orc_mlp_forward(p.ctypes.data, int(n_panes), len(x), x.ctypes.data, pn.ctypes.data,
                          out.ctypes.data)
    return out


def mlp_loss_grad(params, n_panes, tuples, panes, target):
    p = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(tuples, dtype=np.float64).reshape(-1, 4)
    pn = np.ascontiguousarray(panes, dtype=np.int32)
    t = np.ascontiguousarray(target, dtype=np.float64).reshape(-1, 3)
    g = np.empty_like(p)
    loss = lib().orc_mlp_loss_grad(p.ctypes.data, int(n_panes), len(x), x.ctypes.data, pn.ctypes.data,
                                   t.ctypes.data, g.ctypes.data)
    return loss, g


def spec_to_xyz(spec, lambda_nm, cmf):
    spec = np.ascontiguousarray(spec, dtype=np.float64)
    nl = spec.shape[-1]
    lam = np.ascontiguousarray(lambda_nm, dtype=np.float64)
    cm = np.ascontiguousarray(cmf, dtype=np.float64).reshape(-1)
    out = np.empty(spec.shape[:-1] + (3,))
    lib().orc_spec_to_xyz(spec.size // nl, nl, lam.ctypes.data, cm.ctypes.data, spec.ctypes.data,
                          out.ctypes.data)
    return out
