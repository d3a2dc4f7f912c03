"""Bounces overlapped on two streams against the serial order, through the C
ABI.  A bounce's shadow walk, accumulation and caustic gather run on the
context's second stream beside the next bounce's closest-hit pass; a context
created with SDM_SERIAL=1 keeps every pass on the caller's stream.  The same
paths do the same arithmetic either way, so the images agree to the order
of the FP64 accumulation (1e-9 relative) and the path, segment, fork and
record counts are equal -- eagerly with per-kernel events, and replayed as
graphs (the capture takes the same fork and join).
"""
import os

import numpy as np
import pytest

from paper_1912_05494_amd import synth

pytestmark = pytest.mark.gpu

COUNTS = ("paths", "closest_segments", "shadow_segments", "forks", "spectral_paths", "spectral_records",
          "glass_vertices", "photons_stored")


@pytest.fixture(scope="module")
def contexts():
    import torch
    from paper_1912_05494_amd import sdm
    assert torch.cuda.is_available()
    ov = sdm.Context(0)
    old = os.environ.get("SDM_SERIAL")
    os.environ["SDM_SERIAL"] = "1"
    try:
        ser = sdm.Context(0)
    finally:
        if old is None:
            del os.environ["SDM_SERIAL"]
        else:
            os.environ["SDM_SERIAL"] = old
    yield sdm, ov, ser
    ov.close()
    ser.close()


def np64(t):
    return t.cpu().numpy().astype(np.float64)


def close(a, b, rtol=1e-9):
    return np.allclose(a, b, rtol=rtol, atol=rtol * max(1e-30, np.abs(b).max()))


@pytest.mark.parametrize("precision,photons,walk", [("fp32", 0, "auto"), ("fp64", 0, "auto"), ("fp32", 0, "bvh"),
                                                    ("fp32", 0, "cells"), ("fp32", 1 << 16, "auto")])
def test_overlap_matches_serial(contexts, precision, photons, walk):
    """walk: shadow rays on the sun grid ("auto") or the BVH (with its own
    overflow stack beside the closest-hit pass's), or closest hits by
    geometric sub-domains ("cells")."""
    sdm, ov, ser = contexts
    opts = {"auto": {}, "bvh": {"shadow_walk": "bvh"}, "cells": {"subdomains": (2, 2, 1)}}[walk]
    # bubbly panes scatter sunlight onto the floor, so the photon map is not empty
    scene = synth.nave_scene(seed=3, target_tris=6000, windows_per_side=4, bubbly=photons > 0)
    st = synth.nave_settings(W=96, H=64, spp=4, max_depth=6, n_lambda=16)
    runs = {}
    for name, ctx, graph in (("serial", ser, False), ("overlap", ov, False), ("overlap-graph", ov, True),
                             ("serial-graph", ser, True)):
        g = sdm.Scene(ctx, scene, **opts)
        # chunks of 2^13 paths: several chunks, each joined back before the next
        spec, xyz, stats = sdm.render(ctx, g, st, precision=precision, chunk_paths=1 << 13, graph=graph,
                                      timing=not graph, photons=photons, photon_radius=0.1)
        runs[name] = (np64(spec), np64(xyz), stats)
    ref_spec, ref_xyz, ref_st = runs["serial"]
    assert ref_st["chunks"] >= 3 and ref_st["shadow_segments"] > 0
    if photons:
        assert ref_st["photons_stored"] > 0
    for name, (spec, xyz, stats) in runs.items():
        assert close(spec, ref_spec), name
        assert close(xyz, ref_xyz), name
        for k in COUNTS:
            assert stats[k] == ref_st[k], (name, k)
    # per-kernel events are taken on the stream each pass ran on
    ks = runs["overlap"][2]
    assert ks["kernel_launches"]["shadow"] == ks["kernel_launches"]["trace"] > 0
    assert ks["kernel_ms"]["shadow"] > 0 and ks["kernel_ms"]["shadow_accum"] > 0
