"""Structure of the wide BVH built on the host (CPU only): the builder is run
through a small driver compiled with hipcc, and its nodes are checked here
against properties any correct tree has.  Closest-hit results that follow
from these properties are checked against brute force in the GPU tests."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1912_05494_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1912_05494_amd", "csrc")
NODE = np.dtype([("lox", "<f4", 4), ("hix", "<f4", 4), ("loy", "<f4", 4), ("hiy", "<f4", 4),
                 ("loz", "<f4", 4), ("hiz", "<f4", 4), ("child", "<i4", 4), ("pad", "<i4", 4)])


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("bvh")
    exe = d / "bvh_dump"
    subprocess.run(["hipcc", "-O2", "-std=c++17", os.path.join(HERE, "bvh_dump.cpp"),
                    os.path.join(CSRC, "bvh_build.cpp"), "-o", str(exe)], check=True,
                   stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return d, exe


def build(driver, pos, idx):
    d, exe = driver
    pos = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)
    idx = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1, 3)
    src, dst = d / "mesh.bin", d / "bvh.bin"
    with open(src, "wb") as f:
        np.array([len(pos), len(idx)], np.int32).tofile(f)
        pos.tofile(f)
        idx.tofile(f)
    subprocess.run([str(exe), str(src), str(dst)], check=True)
    raw = np.fromfile(dst, dtype=np.uint8)
    depth, stack, n_nodes, ok = np.frombuffer(raw[:16], np.int32)
    nodes = np.frombuffer(raw[16:16 + 128 * n_nodes], NODE)
    order = np.frombuffer(raw[16 + 128 * n_nodes:], np.int32)
    return dict(depth=int(depth), stack=int(stack), nodes=nodes, order=order, ok=bool(ok), pos=pos, idx=idx)


def decode(e):
    """Child entry -> ('inner', index) | ('leaf', first, count) | None."""
    if e == -1:
        return None
    if e >= 0:
        return ("inner", int(e))
    x = -1 - int(e)
    return ("leaf", x >> 8, x & 255)


def check_tree(b):
    nodes, order, pos, idx = b["nodes"], b["order"], b["pos"], b["idx"]
    nt = len(idx)
    assert b["ok"]
    assert sorted(order.tolist()) == list(range(nt))
    covered = np.zeros(nt, np.int32)
    parent = {0: None}
    level = {0: 0}
    for i, nd in enumerate(nodes):
        n_kids = 0
        for c in range(4):
            e = decode(nd["child"][c])
            if e is None:
                # empty slot: an empty box that no slab test can accept
                assert nd["lox"][c] == np.inf and nd["hix"][c] == -np.inf
                continue
            n_kids += 1
            lo = np.array([nd["lox"][c], nd["loy"][c], nd["loz"][c]])
            hi = np.array([nd["hix"][c], nd["hiy"][c], nd["hiz"][c]])
            if e[0] == "inner":
                j = e[1]
                assert j > i and j not in parent, "breadth-first order, one parent"
                parent[j] = i
                level[j] = level[i] + 1
                tris = subtree_tris(nodes, j)
            else:
                _, first, cnt = e
                assert 1 <= cnt <= 255
                covered[first:first + cnt] += 1
                tris = list(range(first, first + cnt))
            v = pos[idx[order[tris]].reshape(-1)]
            # padded boxes hold every vertex strictly
            assert (v > lo).all() and (v < hi).all()
        assert 1 <= n_kids <= 4
        assert n_kids >= 2 or len(nodes) == 1
    assert (covered == 1).all(), "leaf ranges partition the triangles"
    assert sorted(parent) == list(range(len(nodes)))
    lv = [level[i] for i in range(len(nodes))]
    assert lv == sorted(lv), "levels never decrease along the node array"
    assert b["depth"] == max(lv) + 2


def subtree_tris(nodes, j):
    out = []
    for c in range(4):
        e = decode(nodes[j]["child"][c])
        if e is None:
            continue
        if e[0] == "inner":
            out += subtree_tris(nodes, e[1])
        else:
            out += list(range(e[1], e[1] + e[2]))
    return out


def stack_bound(nodes, i=0):
    """Most entries a depth-first walk can hold on its stack: at each node it
    keeps the other children while it descends into one."""
    kids = [decode(e) for e in nodes[i]["child"]]
    kids = [k for k in kids if k is not None]
    deeper = max([stack_bound(nodes, k[1]) for k in kids if k[0] == "inner"], default=0)
    return len(kids) - 1 + deeper


def random_soup(n, seed):
    rng = np.random.default_rng(seed)
    c = rng.uniform(-5, 5, (n, 1, 3))
    v = c + rng.normal(0, 0.3, (n, 3, 3))
    return v.reshape(-1, 3), np.arange(3 * n, dtype=np.int32).reshape(-1, 3)


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (5, 2), (37, 3), (1000, 4)])
def test_random_soups(driver, n, seed):
    pos, idx = random_soup(n, seed)
    b = build(driver, pos, idx)
    check_tree(b)
    assert b["stack"] == stack_bound(b["nodes"])
    if n > 100:
        # wide nodes: about half the levels of a binary tree with small leaves
        assert b["depth"] <= int(np.ceil(np.log2(n / 4) / 2)) + 4


def test_nave_scene(driver):
    sc = synth.nave_scene(seed=0, target_tris=20000)
    b = build(driver, sc.pos, sc.idx)
    check_tree(b)
    assert b["stack"] == stack_bound(b["nodes"])
    n2 = sc.nt
    # most nodes are full
    fill = np.mean([(nd["child"] != -1).sum() for nd in b["nodes"]])
    assert fill > 3.0, fill
    assert len(b["nodes"]) < n2 / 4


def test_coincident_centroids(driver):
    """All triangles share one centroid: split by count, still a valid tree."""
    n = 300
    rng = np.random.default_rng(7)
    d = rng.normal(0, 1, (n, 3))
    v = np.stack([d, -d, np.zeros_like(d)], 1).reshape(-1, 3)
    b = build(driver, v, np.arange(3 * n, dtype=np.int32).reshape(-1, 3))
    check_tree(b)
    assert b["stack"] == stack_bound(b["nodes"])
