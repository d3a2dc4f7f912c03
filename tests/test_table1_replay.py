"""The CPU replay of the shape of the paper's Table 1 (speedup against
threads x spectral sub-domains) on a small image: every cell renders the same
image and reports a positive time."""
import os

import numpy as np

import bench
from paper_1912_05494_amd import synth


def test_table1_replay_small():
    st = synth.nave_settings(W=32, H=24, spp=1, max_depth=3, n_lambda=8)
    sc = synth.nave_scene(seed=1, target_tris=4000)
    out = bench.cpu_table1(threads=(1, 2), bands=(1, 2, 4), reps=1, scene=sc, settings=st)
    assert set(out["speedup"]) == {"1", "2", "4"}
    assert out["speedup"]["1"]["1"] == 1.0
    for nb, row in out["seconds"].items():
        for t, s in row.items():
            assert s > 0.0
