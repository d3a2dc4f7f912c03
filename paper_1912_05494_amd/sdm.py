"""Python binding of ``libsdm.so`` (include/sdm.h): argument marshalling only.

PyTorch provides device memory and streams; every step of the render runs in
the library's HIP kernels.  There is no CPU fallback: if the library or a GPU
is missing, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsdm.so")

SDM_OK = 0
SDM_MEM_HOST, SDM_MEM_DEVICE = 0, 1
SDM_PREC_FP32, SDM_PREC_FP64 = 0, 1
KERNELS = ("generate", "trace", "shade", "shadow", "finalize", "shadow_accum", "shade_glass", "bubbly_eval",
           "shade_bubbly", "photon", "caustic")
BTDF_MODES = {"exact": 0, "surrogate": 1, "fallback": 2}
SHADOW_WALKS = {"auto": 0, "bvh": 1}

_FP = C.POINTER(C.c_float)


class Material(C.Structure):
    _fields_ = [("type", C.c_int32), ("albedo", _FP), ("n", _FP), ("k", _FP), ("alpha_tint", _FP),
                ("thick_mm", C.c_float), ("bubble_density_mm3", C.c_float),
                ("bubble_rmin_um", C.c_float), ("bubble_rmax_um", C.c_float),
                ("pane_id", C.c_int32), ("dist_map", C.c_int32)]


class DistMapDesc(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("material", C.POINTER(C.c_int32)), ("thick_mm", _FP)]


class SceneDesc(C.Structure):
    _fields_ = [("nv", C.c_int32), ("pos", _FP), ("vthick_mm", _FP), ("nt", C.c_int32),
                ("idx", C.POINTER(C.c_int32)), ("mat", C.POINTER(C.c_int32)),
                ("n_mat", C.c_int32), ("mats", C.POINTER(Material)), ("n_tab", C.c_int32),
                ("tab_lambda_nm", _FP), ("sun_dir", C.c_float * 3), ("sun_E", _FP),
                ("sky_L", _FP), ("shadow_walk", C.c_int32), ("uv", _FP), ("n_maps", C.c_int32),
                ("maps", C.POINTER(DistMapDesc)), ("subdomains", C.c_int32 * 3),
                ("subdomain_handoff", C.c_int32)]


class Camera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("target", C.c_float * 3), ("up", C.c_float * 3),
                ("vfov_deg", C.c_float), ("ortho_height", C.c_float), ("W", C.c_int32),
                ("H", C.c_int32), ("projection", C.c_int32)]


class RenderParams(C.Structure):
    _fields_ = [("camera", Camera), ("n_lambda", C.c_int32), ("lambda_nm", _FP),
                ("cmf_xyz", _FP), ("spp", C.c_int32), ("max_depth", C.c_int32),
                ("seed", C.c_uint64), ("job_id", C.c_uint32), ("n_bands", C.c_int32),
                ("band_edges", C.POINTER(C.c_int32)), ("tile_w", C.c_int32),
                ("tile_h", C.c_int32), ("beta_threshold", C.c_float), ("precision", C.c_int32),
                ("chunk_paths", C.c_int64), ("timing", C.c_int32), ("btdf_mode", C.c_int32),
                ("err_dims", C.c_int32 * 3), ("mlp", C.c_void_p), ("err_table", _FP),
                ("err_bound", C.c_float), ("graph", C.c_int32), ("max_items", C.c_int64),
                ("photons", C.c_int64), ("photon_radius", C.c_float),
                ("trace_blocks_per_cu", C.c_int32), ("shadow_blocks_per_cu", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("spectral_samples", C.c_uint64), ("paths", C.c_uint64),
                ("closest_segments", C.c_uint64), ("shadow_segments", C.c_uint64),
                ("forks", C.c_uint64), ("chunks", C.c_uint64), ("nodes_visited", C.c_uint64 * 2),
                ("tris_tested", C.c_uint64 * 2), ("bubbly_vertices", C.c_uint64),
                ("spectral_paths", C.c_uint64), ("spectral_records", C.c_uint64),
                ("glass_vertices", C.c_uint64 * 2), ("ms_render", C.c_double), ("kernel_ms", C.c_double * 11),
                ("kernel_launches", C.c_uint64 * 11), ("items_done", C.c_uint64), ("items_total", C.c_uint64),
                ("interface_rays", C.c_uint64), ("photons_stored", C.c_uint64)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_[:6]}
        d["ms_render"] = self.ms_render
        d["nodes_visited"] = {"closest": int(self.nodes_visited[0]), "shadow": int(self.nodes_visited[1])}
        d["tris_tested"] = {"closest": int(self.tris_tested[0]), "shadow": int(self.tris_tested[1])}
        d["bubbly_vertices"] = int(self.bubbly_vertices)
        d["spectral_paths"] = int(self.spectral_paths)
        d["spectral_records"] = int(self.spectral_records)
        d["glass_vertices"] = {"all": int(self.glass_vertices[0]), "spectral": int(self.glass_vertices[1])}
        d["kernel_ms"] = {k: self.kernel_ms[i] for i, k in enumerate(KERNELS)}
        d["kernel_launches"] = {k: int(self.kernel_launches[i]) for i, k in enumerate(KERNELS)}
        d["items_done"] = int(self.items_done)
        d["items_total"] = int(self.items_total)
        d["interface_rays"] = int(self.interface_rays)
        d["photons_stored"] = int(self.photons_stored)
        return d


class Outputs(C.Structure):
    _fields_ = [("spectral", C.c_void_p), ("xyz", C.c_void_p), ("spectral_mem", C.c_int32),
                ("xyz_mem", C.c_int32), ("stats", C.POINTER(Stats)), ("events", C.c_void_p)]


class Job(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("params", C.POINTER(RenderParams)), ("out", C.POINTER(Outputs))]


class TuneResult(C.Structure):
    _fields_ = [("chunk_paths", C.c_int64), ("tile_w", C.c_int32), ("tile_h", C.c_int32), ("ms", C.c_double),
                ("from_cache", C.c_int32), ("trace_blocks_per_cu", C.c_int32), ("shadow_blocks_per_cu", C.c_int32)]


class TrainParams(C.Structure):
    _fields_ = [("steps", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float)]


class SdmError(RuntimeError):
    """A call of the library failed; code is its return value (SDM_E_*), or
    None for errors raised by the binding itself."""

    def __init__(self, msg, code=None):
        super().__init__(msg)
        self.code = code


_lib = None


def lib():
    """Load libsdm.so; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SdmError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.sdm_context_create.argtypes = [C.c_int, C.POINTER(vp)]
        L.sdm_context_destroy.argtypes = [vp]
        L.sdm_last_error.restype = C.c_char_p
        L.sdm_last_error.argtypes = [vp]
        L.sdm_scene_create.argtypes = [vp, C.POINTER(SceneDesc), C.POINTER(vp)]
        L.sdm_scene_destroy.argtypes = [vp]
        L.sdm_scene_subdomains.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.sdm_scene_info.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.sdm_render.argtypes = [vp, vp, C.POINTER(RenderParams), C.POINTER(Outputs), vp]
        L.sdm_slab_eval.argtypes = [vp, C.c_int64] + [vp] * 9
        L.sdm_debug_intersect.argtypes = [vp, vp, C.c_int64] + [vp] * 7
        L.sdm_debug_shadow.argtypes = [vp, vp, C.c_int64, vp, vp, C.c_float, vp, vp]
        L.sdm_slab_mc.argtypes = ([vp, C.c_int64] + [vp] * 8 + [C.c_float, C.c_float, C.c_int32, C.c_uint64,
                                                                 C.c_uint32, C.c_int32] + [vp] * 5)
        L.sdm_slab_mc_noalloc.argtypes = L.sdm_slab_mc.argtypes
        L.sdm_mlp_nparams.restype = C.c_int64
        L.sdm_mlp_nparams.argtypes = [C.c_int32]
        L.sdm_mlp_create.argtypes = [vp, C.c_int32, vp, C.POINTER(vp)]
        L.sdm_mlp_destroy.argtypes = [vp]
        L.sdm_mlp_get_params.argtypes = [vp, vp]
        L.sdm_mlp_grad.argtypes = [vp, C.c_int64] + [vp] * 6
        L.sdm_mlp_train.argtypes = [vp, C.c_int64] + [vp] * 3 + [C.POINTER(TrainParams), vp, vp]
        L.sdm_mlp_infer.argtypes = [vp, C.c_int64] + [vp] * 4
        L.sdm_debug_mfma.argtypes = [vp] * 8
        L.sdm_mlp_error_table.argtypes = [vp, C.c_int64] + [vp] * 6
        L.sdm_render_batch.argtypes = [vp, C.c_int32, C.POINTER(Job), C.POINTER(Stats), vp]
        L.sdm_autotune.argtypes = [vp, vp, C.POINTER(RenderParams), C.c_char_p, C.POINTER(TuneResult), vp]
        L.sdm_render_checkpoint.argtypes = [vp, C.c_char_p]
        L.sdm_render_resume.argtypes = [vp, C.c_char_p, vp, C.POINTER(RenderParams), C.POINTER(Outputs), vp]
        L.sdm_mlp_save.argtypes = [vp, C.c_char_p]
        L.sdm_mlp_load.argtypes = [vp, C.c_char_p, C.POINTER(vp)]
        L.sdm_mlp_info.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        _lib = L
    return _lib


EXPORTED = ("sdm_context_create", "sdm_context_destroy", "sdm_last_error", "sdm_scene_create",
            "sdm_scene_destroy", "sdm_scene_info", "sdm_scene_subdomains", "sdm_render", "sdm_slab_eval",
            "sdm_debug_intersect", "sdm_debug_shadow", "sdm_slab_mc", "sdm_mlp_nparams",
            "sdm_mlp_create", "sdm_mlp_destroy", "sdm_mlp_get_params", "sdm_mlp_grad",
            "sdm_mlp_train", "sdm_mlp_infer", "sdm_debug_mfma", "sdm_mlp_error_table",
            "sdm_render_batch", "sdm_autotune", "sdm_render_checkpoint", "sdm_render_resume", "sdm_mlp_save",
            "sdm_mlp_load", "sdm_mlp_info", "sdm_slab_mc_noalloc")
SDM_E_INVALID, SDM_E_NOMEM, SDM_E_DEVICE = -1, -2, -3
SDM_E_UNSUPPORTED = -4
SDM_E_ABORTED = -5


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _f32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32)


class Context:
    def __init__(self, device=0):
        import torch
        if not torch.cuda.is_available():
            raise SdmError("no GPU available")
        self.device = device
        self.ptr = C.c_void_p()
        # scenes and networks of this context, destroyed before it (the C ABI
        # requires that order)
        self._owned = weakref.WeakSet()
        rc = lib().sdm_context_create(device, C.byref(self.ptr))
        if rc != SDM_OK:
            raise SdmError(f"sdm_context_create failed ({rc})", code=rc)

    def check(self, rc, what):
        if rc != SDM_OK:
            msg = lib().sdm_last_error(self.ptr).decode(errors="replace")
            raise SdmError(f"{what} failed ({rc}): {msg}", code=rc)

    def close(self):
        if self.ptr:
            for obj in list(self._owned):
                obj.close()
            lib().sdm_context_destroy(self.ptr)
            self.ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Scene:
    """Uploads a ``synth.Scene``-like object (pos, idx, mat, materials, tables)."""

    def __init__(self, ctx: Context, scene, shadow_walk="auto", subdomains=None, handoff="queue"):
        """shadow_walk: "auto" (sun grid where it is compact) or "bvh".
        subdomains: (nx, ny, nz) cells of geometric sub-domains, or None;
        handoff: "queue" (interface queues, one pass per cell crossed) or
        "march" (the thread goes on in the next cell)."""
        self.ctx = ctx
        keep = []
        pos = _f32(scene.pos.reshape(-1))
        vth = _f32(scene.vthick)
        idx = np.ascontiguousarray(scene.idx.reshape(-1), dtype=np.int32)
        mat = np.ascontiguousarray(scene.mat, dtype=np.int32)
        tab = _f32(scene.tab_lambda)
        fp = lambda a: a.ctypes.data_as(_FP) if a is not None else None
        mats = (Material * max(1, len(scene.materials)))()
        for i, m in enumerate(scene.materials):
            arrs = [_f32(m.albedo), _f32(m.n), _f32(m.k), _f32(m.alpha_tint)]
            keep += arrs
            mats[i] = Material(int(m.type), *[fp(a) for a in arrs], float(m.thick_mm),
                               float(m.bubble_density), float(m.bubble_rmin_um),
                               float(m.bubble_rmax_um), int(m.pane_id), int(getattr(m, "dist_map", 0)))
        sE, sL = _f32(scene.sun_E), _f32(scene.sky_L)
        uv = _f32(None if getattr(scene, "uv", None) is None else np.asarray(scene.uv).reshape(-1))
        smaps = list(getattr(scene, "maps", []) or [])
        maps = (DistMapDesc * max(1, len(smaps)))()
        for i, dm in enumerate(smaps):
            tm = np.ascontiguousarray(np.asarray(dm.material).reshape(-1), dtype=np.int32)
            th = _f32(None if dm.thick_mm is None else np.asarray(dm.thick_mm).reshape(-1))
            keep += [tm, th]
            maps[i] = DistMapDesc(int(dm.W), int(dm.H), tm.ctypes.data_as(C.POINTER(C.c_int32)), fp(th))
        keep += [pos, vth, idx, mat, tab, sE, sL, uv, maps]
        d = SceneDesc(len(scene.pos), fp(pos), fp(vth), int(scene.idx.shape[0]),
                      idx.ctypes.data_as(C.POINTER(C.c_int32)),
                      mat.ctypes.data_as(C.POINTER(C.c_int32)), len(scene.materials), mats,
                      len(tab), fp(tab), (C.c_float * 3)(*[float(x) for x in scene.sun_dir]),
                      fp(sE), fp(sL), SHADOW_WALKS[shadow_walk], fp(uv), len(smaps), maps,
                      (C.c_int32 * 3)(*[int(x) for x in (subdomains or (0, 0, 0))]),
                      {"queue": 0, "march": 1}[handoff])
        self.ptr = C.c_void_p()
        ctx.check(lib().sdm_scene_create(ctx.ptr, C.byref(d), C.byref(self.ptr)), "sdm_scene_create")
        ctx._owned.add(self)
        self.nt = int(scene.idx.shape[0])

    def info(self):
        n, dep, stk = C.c_int32(), C.c_int32(), C.c_int32()
        cells, cands = C.c_int64(), C.c_int64()
        lib().sdm_scene_info(self.ptr, C.byref(n), C.byref(dep), C.byref(stk), C.byref(cells), C.byref(cands))
        return {"n_nodes": n.value, "depth": dep.value, "stack": stk.value, "grid_cells": cells.value,
                "grid_candidates": cands.value}

    def subdomains(self):
        """(cells along x, y, z; triangle references of the cells; their BVH nodes)."""
        n = (C.c_int32 * 3)()
        refs, nodes = C.c_int64(), C.c_int64()
        self.ctx.check(lib().sdm_scene_subdomains(self.ptr, n, C.byref(refs), C.byref(nodes)), "sdm_scene_subdomains")
        return tuple(int(x) for x in n), int(refs.value), int(nodes.value)

    def close(self):
        if self.ptr:
            lib().sdm_scene_destroy(self.ptr)
            self.ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_params(settings, n_bands=None, band_edges=None, tile=(0, 0), precision="fp32",
                chunk_paths=0, timing=False, btdf=None, graph=False, max_items=0, photons=0, photon_radius=0.05,
                blocks_per_cu=(0, 0)):
    """btdf: None (exact walks on bubbly panes) or a dict with mode ("exact",
    "surrogate", "fallback"), mlp (an MLP) and, for "fallback", err_table
    (array (n_panes, n_cos, n_d, n_rho)) and bound."""
    cam = settings.camera
    lam = _f32(settings.lambda_nm)
    cmf = _f32(np.asarray(settings.cmf).reshape(-1))
    keep = [lam, cmf]
    be = None
    nb = int(settings.n_bands if n_bands is None else n_bands)
    if band_edges is not None:
        be = np.ascontiguousarray(band_edges, dtype=np.int32)
        keep.append(be)
        nb = len(be) - 1
    p = RenderParams(
        Camera((C.c_float * 3)(*cam.eye), (C.c_float * 3)(*cam.target), (C.c_float * 3)(*cam.up),
               float(cam.vfov_deg), float(cam.ortho_height), int(cam.W), int(cam.H),
               int(cam.projection)),
        len(lam), lam.ctypes.data_as(_FP), cmf.ctypes.data_as(_FP), int(settings.spp),
        int(settings.max_depth), int(settings.seed), int(settings.job_id), nb,
        be.ctypes.data_as(C.POINTER(C.c_int32)) if be is not None else None,
        int(tile[0]), int(tile[1]), float(settings.beta_threshold),
        SDM_PREC_FP64 if precision == "fp64" else SDM_PREC_FP32, int(chunk_paths), int(timing))
    p.graph = int(bool(graph))
    p.max_items = int(max_items)
    p.photons = int(photons)
    p.photon_radius = float(photon_radius)
    p.trace_blocks_per_cu, p.shadow_blocks_per_cu = int(blocks_per_cu[0]), int(blocks_per_cu[1])
    if btdf is not None:
        p.btdf_mode = BTDF_MODES[btdf.get("mode", "exact")]
        if btdf.get("mlp") is not None:
            p.mlp = btdf["mlp"].ptr
            keep.append(btdf["mlp"])
        if btdf.get("err_table") is not None:
            tab = _f32(btdf["err_table"])
            keep.append(tab)
            p.err_table = tab.ctypes.data_as(_FP)
            p.err_dims = (C.c_int32 * 3)(*tab.shape[1:4])
            p.err_bound = float(btdf.get("bound", 1e-3))
    return p, keep


def render(ctx: Context, scene: Scene, settings, n_bands=None, band_edges=None, tile=(0, 0),
           precision="fp32", chunk_paths=0, timing=False, stream=None, spectral=True, xyz=True,
           btdf=None, graph=False, max_items=0, events=None, resume=None, photons=0, photon_radius=0.05):
    """Render into new device tensors: (spectral (H, W, nl) float32, xyz (H, W, 3) float64,
    stats dict).

    max_items > 0: at most that many work items this call; when items remain,
    stats["aborted"] is True and the images hold the items done so far.
    events: a device int64 tensor (H, W, nl) that receives the event
    signatures (bit patterns of the library's uint64 values).
    resume: continue a partial render -- True for the context's own state, or
    the path of a checkpoint file."""
    import torch
    cam = settings.camera
    nl = len(settings.lambda_nm)
    dev = torch.device("cuda", ctx.device)
    spec_t = torch.empty((cam.H, cam.W, nl), dtype=torch.float32, device=dev) if spectral else None
    xyz_t = torch.empty((cam.H, cam.W, 3), dtype=torch.float64, device=dev) if xyz else None
    p, keep = make_params(settings, n_bands, band_edges, tile, precision, chunk_paths, timing, btdf, graph,
                          max_items, photons, photon_radius)
    st = Stats()
    out = Outputs(_ptr(spec_t), _ptr(xyz_t), SDM_MEM_DEVICE, SDM_MEM_DEVICE, C.pointer(st), _ptr(events))
    if resume is None:
        rc = lib().sdm_render(ctx.ptr, scene.ptr, C.byref(p), C.byref(out), _stream(stream))
    else:
        path = None if resume is True else str(resume).encode()
        rc = lib().sdm_render_resume(ctx.ptr, path, scene.ptr, C.byref(p), C.byref(out), _stream(stream))
    aborted = rc == SDM_E_ABORTED
    if not aborted:
        ctx.check(rc, "sdm_render" if resume is None else "sdm_render_resume")
    d = st.as_dict()
    d["aborted"] = aborted
    return spec_t, xyz_t, d


def checkpoint(ctx: Context, path):
    """Saves the context's partial render (after an aborted render) to path."""
    ctx.check(lib().sdm_render_checkpoint(ctx.ptr, str(path).encode()), "sdm_render_checkpoint")


def render_into(ctx: Context, scene: Scene, params, spec_t, xyz_t, stream=None):
    """Render with prepared params into existing device tensors; returns stats."""
    st = Stats()
    out = Outputs(_ptr(spec_t), _ptr(xyz_t), SDM_MEM_DEVICE, SDM_MEM_DEVICE, C.pointer(st))
    ctx.check(lib().sdm_render(ctx.ptr, scene.ptr, C.byref(params), C.byref(out), _stream(stream)),
              "sdm_render")
    return st.as_dict()


def slab_eval(ctx: Context, cos_i, lambda_nm, d_mm, n, k, alpha_tint, stream=None):
    """Device float32 tensors of equal length -> (R, T) device tensors."""
    import torch
    m = cos_i.numel()
    R = torch.empty_like(cos_i)
    T = torch.empty_like(cos_i)
    ctx.check(lib().sdm_slab_eval(ctx.ptr, m, _ptr(cos_i), _ptr(lambda_nm), _ptr(d_mm), _ptr(n),
                                  _ptr(k), _ptr(alpha_tint), _ptr(R), _ptr(T), _stream(stream)),
              "sdm_slab_eval")
    return R, T


def debug_intersect(ctx: Context, scene: Scene, o, d, skip=None, stream=None):
    import torch
    m = o.shape[0]
    t = torch.empty(m, dtype=torch.float32, device=o.device)
    tri = torch.empty(m, dtype=torch.int32, device=o.device)
    uv = torch.empty((m, 2), dtype=torch.float32, device=o.device)
    ctx.check(lib().sdm_debug_intersect(ctx.ptr, scene.ptr, m, _ptr(o), _ptr(d), _ptr(skip), _ptr(t),
                                        _ptr(tri), _ptr(uv), _stream(stream)), "sdm_debug_intersect")
    return t, tri, uv


def debug_shadow(ctx: Context, scene: Scene, o, lambda_nm, skip=None, stream=None):
    import torch
    m = o.shape[0]
    T = torch.empty(m, dtype=torch.float32, device=o.device)
    ctx.check(lib().sdm_debug_shadow(ctx.ptr, scene.ptr, m, _ptr(o), _ptr(skip), float(lambda_nm),
                                     _ptr(T), _stream(stream)), "sdm_debug_shadow")
    return T


PRECISION = {"fp32": 0, "fp64": 1}


def slab_mc(ctx: Context, cos_i, lambda_nm, d_mm, rho_b, n, k, alpha_tint=None, rmin_um=10.0,
            rmax_um=200.0, n_photons=64, seed=0, tuple0=0, precision="fp32", n_ref=None, stream=None,
            noalloc=False, out=None):
    """Bubbly-slab Monte Carlo on device float32 tensors of length m ->
    (R, T, A, w_lobe) device tensors.  noalloc: the allocation-free entry
    point (m <= 65536, outputs valid once the stream is synchronised); out:
    four preallocated output tensors."""
    import torch
    m = cos_i.numel()
    out = list(out) if out is not None else [torch.empty_like(cos_i) for _ in range(4)]
    fn = lib().sdm_slab_mc_noalloc if noalloc else lib().sdm_slab_mc
    ctx.check(fn(ctx.ptr, m, _ptr(cos_i), _ptr(lambda_nm), _ptr(d_mm), _ptr(rho_b), _ptr(n),
                 _ptr(k), _ptr(alpha_tint), _ptr(n_ref), float(rmin_um), float(rmax_um),
                 int(n_photons),
                 int(seed), int(tuple0), PRECISION[precision], *[_ptr(o) for o in out],
                 _stream(stream)), "sdm_slab_mc_noalloc" if noalloc else "sdm_slab_mc")
    return tuple(out)


def mlp_nparams(n_panes):
    return int(lib().sdm_mlp_nparams(int(n_panes)))


class MLP:
    """Surrogate network held by the library (FP32 master weights, BF16 copy,
    Adam state)."""

    def __init__(self, ctx: Context, n_panes, params):
        self.ctx = ctx
        self.n_panes = int(n_panes)
        p = _f32(params).reshape(-1)
        if p.size != mlp_nparams(n_panes):
            raise SdmError(f"expected {mlp_nparams(n_panes)} parameters, got {p.size}")
        h = C.c_void_p()
        ctx.check(lib().sdm_mlp_create(ctx.ptr, self.n_panes, p.ctypes.data, C.byref(h)), "sdm_mlp_create")
        self.ptr = h
        ctx._owned.add(self)

    def params(self):
        p = np.empty(mlp_nparams(self.n_panes), dtype=np.float32)
        self.ctx.check(lib().sdm_mlp_get_params(self.ptr, p.ctypes.data), "sdm_mlp_get_params")
        return p

    def grad(self, tuples, panes, target, stream=None):
        """Device tensors tuples [m,4] f32, panes [m] i32, target [m,3] f32 ->
        (gradient device tensor, mean loss)."""
        import torch
        g = torch.empty(mlp_nparams(self.n_panes), dtype=torch.float32, device=tuples.device)
        loss = C.c_float()
        self.ctx.check(lib().sdm_mlp_grad(self.ptr, tuples.shape[0], _ptr(tuples), _ptr(panes), _ptr(target),
                                          _ptr(g), C.byref(loss), _stream(stream)), "sdm_mlp_grad")
        return g, float(loss.value)

    def train(self, tuples, panes, target, steps, batch, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
              stream=None):
        """Adam steps; returns the loss before each step (numpy)."""
        tp = TrainParams(int(steps), int(batch), float(lr), float(beta1), float(beta2), float(eps))
        curve = np.zeros(max(int(steps), 1), dtype=np.float32)
        self.ctx.check(lib().sdm_mlp_train(self.ptr, tuples.shape[0], _ptr(tuples), _ptr(panes), _ptr(target),
                                           C.byref(tp), curve.ctypes.data, _stream(stream)), "sdm_mlp_train")
        return curve[:int(steps)]

    def infer(self, tuples, panes, stream=None):
        import torch
        out = torch.empty((tuples.shape[0], 3), dtype=torch.float32, device=tuples.device)
        self.ctx.check(lib().sdm_mlp_infer(self.ptr, tuples.shape[0], _ptr(tuples), _ptr(panes), _ptr(out),
                                           _stream(stream)), "sdm_mlp_infer")
        return out

    def error_table(self, tuples, panes, target, dims=(8, 3, 4), stream=None):
        """Largest |R - R*| or |T - T*| per cell -> device tensor
        (n_panes, *dims)."""
        import torch
        d = np.ascontiguousarray(dims, dtype=np.int32)
        tab = torch.empty((self.n_panes, *[int(x) for x in dims]), dtype=torch.float32, device=tuples.device)
        self.ctx.check(lib().sdm_mlp_error_table(self.ptr, tuples.shape[0], _ptr(tuples), _ptr(panes),
                                                 _ptr(target), d.ctypes.data, _ptr(tab), _stream(stream)),
                       "sdm_mlp_error_table")
        return tab

    def save(self, path):
        """Parameters and optimiser state to a file."""
        self.ctx.check(lib().sdm_mlp_save(self.ptr, str(path).encode()), "sdm_mlp_save")

    @classmethod
    def load(cls, ctx: Context, path):
        """A network created from a file written by save()."""
        h = C.c_void_p()
        ctx.check(lib().sdm_mlp_load(ctx.ptr, str(path).encode(), C.byref(h)), "sdm_mlp_load")
        net = cls.__new__(cls)
        net.ctx = ctx
        net.ptr = h
        ctx._owned.add(net)
        n, t = C.c_int32(), C.c_int64()
        ctx.check(lib().sdm_mlp_info(h, C.byref(n), C.byref(t)), "sdm_mlp_info")
        net.n_panes = int(n.value)
        return net

    def steps(self):
        """Adam steps taken so far."""
        n, t = C.c_int32(), C.c_int64()
        self.ctx.check(lib().sdm_mlp_info(self.ptr, C.byref(n), C.byref(t)), "sdm_mlp_info")
        return int(t.value)

    def close(self):
        if getattr(self, "ptr", None):
            lib().sdm_mlp_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def debug_mfma(ctx: Context, A32, B32, A16, B16, stream=None):
    """Device float32 [16,32] x [32,16] and [16,16] x [16,16] products on the
    matrix cores (inputs rounded to BF16)."""
    import torch
    C32 = torch.empty((16, 16), dtype=torch.float32, device=A32.device)
    C16 = torch.empty((16, 16), dtype=torch.float32, device=A32.device)
    ctx.check(lib().sdm_debug_mfma(ctx.ptr, _ptr(A32), _ptr(B32), _ptr(C32), _ptr(A16), _ptr(B16), _ptr(C16),
                                   _stream(stream)), "sdm_debug_mfma")
    return C32, C16


def render_batch(ctx: Context, jobs, precision="fp32", chunk_paths=0, graph=False, timing=False, stream=None,
                 max_items=0):
    """jobs: list of (Scene, settings) or (Scene, settings, btdf); renders them
    in one wavefront.  Returns ([(spectral, xyz) device tensors], stats)."""
    import torch
    dev = torch.device("cuda", ctx.device)
    arr = (Job * len(jobs))()
    keep, outs, images = [], [], []
    for i, jb in enumerate(jobs):
        scene, settings = jb[0], jb[1]
        btdf = jb[2] if len(jb) > 2 else None
        cam = settings.camera
        nl = len(settings.lambda_nm)
        spec_t = torch.empty((cam.H, cam.W, nl), dtype=torch.float32, device=dev)
        xyz_t = torch.empty((cam.H, cam.W, 3), dtype=torch.float64, device=dev)
        p, k = make_params(settings, precision=precision, chunk_paths=chunk_paths if i == 0 else 0,
                           timing=timing, btdf=btdf, graph=graph, max_items=max_items)
        o = Outputs(_ptr(spec_t), _ptr(xyz_t), SDM_MEM_DEVICE, SDM_MEM_DEVICE, None)
        keep += [p, k, o, scene]
        arr[i] = Job(scene.ptr, C.pointer(p), C.pointer(o))
        images.append((spec_t, xyz_t))
    st = Stats()
    ctx.check(lib().sdm_render_batch(ctx.ptr, len(jobs), arr, C.byref(st), _stream(stream)), "sdm_render_batch")
    return images, st.as_dict()


def autotune(ctx: Context, scene: Scene, settings, precision="fp32", cache_path=None, n_bands=None, stream=None):
    """Chooses chunk size and pixel tile for (scene, settings); later renders
    with default chunk/tile use it.  Returns a dict of the choice."""
    p, keep = make_params(settings, n_bands=n_bands, precision=precision)
    r = TuneResult()
    ctx.check(lib().sdm_autotune(ctx.ptr, scene.ptr, C.byref(p),
                                 None if cache_path is None else str(cache_path).encode(), C.byref(r),
                                 _stream(stream)), "sdm_autotune")
    return {"chunk_paths": int(r.chunk_paths), "tile": (int(r.tile_w), int(r.tile_h)), "ms": r.ms,
            "from_cache": bool(r.from_cache), "trace_blocks_per_cu": int(r.trace_blocks_per_cu),
            "shadow_blocks_per_cu": int(r.shadow_blocks_per_cu)}
