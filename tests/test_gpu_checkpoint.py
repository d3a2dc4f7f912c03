"""Work-item budgets, checkpoints and resumption of a render, and saved
networks, through the C ABI.

The spectral and ray-set sub-domains are independent, so a render may stop
after any number of (pixel tile x band) items and continue later, in the
same process or from a file in another context.  A run that stops returns
SDM_E_ABORTED with the items done so far in its outputs; the finished image
equals one uninterrupted render up to the order of the FP64 additions
(1e-12 relative in the FP64 accumulator; the spectral output is float32).
"""
import os

import numpy as np
import pytest

from paper_1912_05494_amd import surrogate, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    from paper_1912_05494_amd import sdm
    assert torch.cuda.is_available()
    ctx = sdm.Context(0)
    yield sdm, ctx, torch
    ctx.close()


def tol_ok(g, o):
    return np.abs(g - o) <= 1e-4 * np.maximum(np.abs(o), 1e-3 * np.abs(o).mean())


def np64(t):
    return t.cpu().numpy().astype(np.float64)


def test_abort_then_resume_in_memory(gpu, orc):
    sdm, ctx, torch = gpu
    sc = synth.tiny_scene()
    st = synth.tiny_settings(W=40, H=24, spp=3)
    st.n_bands = 3
    gs = sdm.Scene(ctx, sc)
    full, fx, fst = sdm.render(ctx, gs, st, tile=(8, 8), precision="fp64")
    n_items = 5 * 3 * 3
    assert fst["items_done"] == fst["items_total"] == n_items and not fst["aborted"]
    # 7 items, then 20, then the rest
    a, ax, s1 = sdm.render(ctx, gs, st, tile=(8, 8), precision="fp64", max_items=7)
    assert s1["aborted"] and s1["items_done"] == 7 and s1["items_total"] == n_items
    # the partial image is the oracle's first 7 items, zero elsewhere
    part, _ = orc.render(orc.OracleScene(sc), st, tile=8, items=(0, 7))
    a = np64(a)
    assert tol_ok(a, part).all()
    assert np.all(a[part == 0] == 0)
    b, _, s2 = sdm.render(ctx, gs, st, tile=(8, 8), precision="fp64", max_items=20, resume=True)
    assert s2["aborted"] and s2["items_done"] == 27
    c, cx, s3 = sdm.render(ctx, gs, st, tile=(8, 8), precision="fp64", resume=True)
    assert not s3["aborted"] and s3["items_done"] == n_items
    assert np.allclose(np64(c), np64(full), rtol=1e-6, atol=0)     # float32 spectral output
    assert np.allclose(cx.cpu().numpy(), fx.cpu().numpy(), rtol=1e-12, atol=0)
    # nothing left: a further resume has no partial render
    with pytest.raises(sdm.SdmError):
        sdm.render(ctx, gs, st, tile=(8, 8), precision="fp64", resume=True)


def test_checkpoint_file_resumes_in_another_context(gpu, tmp_path):
    sdm, ctx, torch = gpu
    sc = synth.nave_scene(seed=3, target_tris=6000)
    st = synth.nave_settings(W=96, H=64, spp=4, max_depth=5, n_lambda=24)
    gs = sdm.Scene(ctx, sc)
    full, fx, _ = sdm.render(ctx, gs, st)
    _, _, s1 = sdm.render(ctx, gs, st, max_items=5)
    assert s1["aborted"]
    path = tmp_path / "render.ckpt"
    sdm.checkpoint(ctx, path)
    assert os.path.getsize(path) > 96 * 64 * 24 * 8
    ctx2 = sdm.Context(0)
    try:
        gs2 = sdm.Scene(ctx2, sc)
        _, _, s2 = sdm.render(ctx2, gs2, st, max_items=3, resume=path)
        assert s2["aborted"] and s2["items_done"] == 8
        sdm.checkpoint(ctx2, path)
        c, cx, s3 = sdm.render(ctx2, gs2, st, resume=path)
        assert not s3["aborted"] and s3["items_done"] == s3["items_total"]
        assert np.allclose(np64(c), np64(full), rtol=1e-6, atol=0)
        assert np.allclose(cx.cpu().numpy(), fx.cpu().numpy(), rtol=1e-9, atol=0)
        # a checkpoint of other parameters is refused
        st2 = synth.nave_settings(W=96, H=64, spp=5, max_depth=5, n_lambda=24)
        with pytest.raises(sdm.SdmError, match="another render"):
            sdm.render(ctx2, gs2, st2, resume=path)
    finally:
        gs2.close()          # a scene is destroyed before its context
        ctx2.close()


def test_budget_errors(gpu, tmp_path):
    sdm, ctx, torch = gpu
    sc = synth.tiny_scene()
    st = synth.tiny_settings(W=16, H=16, spp=1)
    gs = sdm.Scene(ctx, sc)
    sdm.render(ctx, gs, st)      # a complete render leaves no partial state
    with pytest.raises(sdm.SdmError, match="no partial"):
        sdm.checkpoint(ctx, tmp_path / "x.ckpt")
    with pytest.raises(sdm.SdmError):
        sdm.render(ctx, gs, st, resume=True)
    ev = torch.zeros((16, 16, len(st.lambda_nm)), dtype=torch.int64, device="cuda")
    with pytest.raises(sdm.SdmError, match="uninterrupted"):
        sdm.render(ctx, gs, st, max_items=1, events=ev)
    with pytest.raises(sdm.SdmError, match="single renders"):
        sdm.render_batch(ctx, [(gs, st), (gs, st)], max_items=1)
    (tmp_path / "junk.ckpt").write_bytes(b"not a checkpoint")
    with pytest.raises(sdm.SdmError):
        sdm.render(ctx, gs, st, resume=tmp_path / "junk.ckpt")
    # max_items larger than the plan: one complete call
    _, _, s = sdm.render(ctx, gs, st, max_items=10 ** 6)
    assert not s["aborted"] and s["items_done"] == s["items_total"]


def test_mlp_save_load_continues_training(gpu, tmp_path):
    sdm, ctx, torch = gpu
    n_panes, m = 3, 2048
    rng = np.random.default_rng(3)
    tup, pane = surrogate.random_tuples(m, n_panes, synth.LAMBDA_81, seed=4)
    target = np.stack([rng.uniform(0, 0.2, m), rng.uniform(0.5, 0.9, m), rng.uniform(0, 0.3, m)], 1)
    t, pn, tg = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in
                 (tup, pane, target.astype(np.float32))]
    net = sdm.MLP(ctx, n_panes, surrogate.init_params(n_panes, seed=9))
    net.train(t, pn, tg, steps=20, batch=512, lr=1e-3)
    path = tmp_path / "net.bin"
    net.save(path)
    net2 = sdm.MLP.load(ctx, path)
    assert net2.n_panes == n_panes and net2.steps() == net.steps() == 20
    assert np.array_equal(net2.params(), net.params())
    # the same next steps from the same state (moments and step count saved)
    net.train(t, pn, tg, steps=5, batch=512, lr=1e-3)
    net2.train(t, pn, tg, steps=5, batch=512, lr=1e-3)
    assert np.allclose(net2.params(), net.params(), rtol=1e-6, atol=1e-7)
    (tmp_path / "bad.bin").write_bytes(b"SDMMLP01" + b"\0" * 8)
    with pytest.raises(sdm.SdmError):
        sdm.MLP.load(ctx, tmp_path / "bad.bin")
    net.close()
    net2.close()
