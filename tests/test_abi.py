"""The C ABI library: it loads, exports every function the public headers
declare, and the Python binding's structures have the C layouts.  No compute
call is made (no GPU here)."""
import ctypes as C
import glob
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1912_05494_amd", "libsdm.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"^\s*(?:int64_t|int|const\s+char\s*\*|void)\s*\**\s*(sdm_\w+)\s*\(", text, re.M))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1912_05494_amd.build import build
        build()
    return C.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 19
    for n in names:
        assert hasattr(lib, n), n
    from paper_1912_05494_amd import sdm
    assert set(sdm.EXPORTED) <= set(names)


def declared_arity():
    """Parameter count of every prototype in the public headers."""
    out = {}
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        for m in re.finditer(r"^\s*(?:int64_t|int|const\s+char\s*\*|void)\s*\**\s*(sdm_\w+)\s*\(([^)]*)\)\s*;",
                             text, re.M):
            args = [a for a in m.group(2).split(",") if a.strip() and a.strip() != "void"]
            out[m.group(1)] = len(args)
    return out


def test_binding_argument_counts_match_header():
    from paper_1912_05494_amd import sdm
    if not os.path.exists(sdm.LIB_PATH):
        pytest.skip("library not built")
    L = sdm.lib()
    arity = declared_arity()
    assert set(sdm.EXPORTED) <= set(arity)
    for name in sdm.EXPORTED:
        assert len(getattr(L, name).argtypes) == arity[name], name


def test_binding_layouts_match_header():
    from paper_1912_05494_amd import sdm
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "sdm.h"
#define P(T, F) printf(#T "." #F " %zu\n", offsetof(T, F))
int main(void) {
  printf("sdm_material %zu\n", sizeof(sdm_material));
  printf("sdm_scene_desc %zu\n", sizeof(sdm_scene_desc));
  printf("sdm_camera %zu\n", sizeof(sdm_camera));
  printf("sdm_render_params %zu\n", sizeof(sdm_render_params));
  printf("sdm_stats %zu\n", sizeof(sdm_stats));
  printf("sdm_outputs %zu\n", sizeof(sdm_outputs));
  printf("sdm_train_params %zu\n", sizeof(sdm_train_params));
  P(sdm_train_params, lr); P(sdm_train_params, eps);
  P(sdm_material, thick_mm); P(sdm_material, pane_id);
  P(sdm_scene_desc, mats); P(sdm_scene_desc, sun_dir); P(sdm_scene_desc, sky_L); P(sdm_scene_desc, shadow_walk);
  P(sdm_render_params, seed); P(sdm_render_params, band_edges);
  P(sdm_render_params, chunk_paths); P(sdm_render_params, timing);
  P(sdm_render_params, btdf_mode); P(sdm_render_params, err_dims); P(sdm_render_params, mlp);
  P(sdm_render_params, err_table); P(sdm_render_params, err_bound);
  P(sdm_stats, bubbly_vertices); P(sdm_stats, kernel_ms); P(sdm_stats, spectral_records); P(sdm_stats, glass_vertices);
  P(sdm_render_params, graph);
  P(sdm_render_params, trace_blocks_per_cu); P(sdm_render_params, shadow_blocks_per_cu);
  printf("sdm_job %zu\n", sizeof(sdm_job));
  printf("sdm_tune_result %zu\n", sizeof(sdm_tune_result));
  P(sdm_tune_result, ms); P(sdm_tune_result, from_cache);
  P(sdm_tune_result, trace_blocks_per_cu); P(sdm_tune_result, shadow_blocks_per_cu);
  P(sdm_stats, ms_render); P(sdm_stats, kernel_launches);
  P(sdm_outputs, stats);
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "l.c")
        open(c, "w").write(src)
        exe = os.path.join(td, "l")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    got = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    m = {"sdm_material": sdm.Material, "sdm_scene_desc": sdm.SceneDesc, "sdm_camera": sdm.Camera,
         "sdm_render_params": sdm.RenderParams, "sdm_stats": sdm.Stats, "sdm_outputs": sdm.Outputs,
         "sdm_train_params": sdm.TrainParams, "sdm_job": sdm.Job, "sdm_tune_result": sdm.TuneResult}
    for key, val in got.items():
        if "." in key:
            t, f = key.split(".")
            assert getattr(m[t], f).offset == int(val), key
        else:
            assert C.sizeof(m[key]) == int(val), key


def test_binding_refuses_without_library(monkeypatch, tmp_path):
    from paper_1912_05494_amd import sdm
    monkeypatch.setattr(sdm, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(sdm, "_lib", None)
    with pytest.raises(sdm.SdmError):
        sdm.lib()
