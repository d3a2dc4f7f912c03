"""Bubbly-glass Monte Carlo and the surrogate network: HIP path vs the FP64
oracle, through the C ABI.

Tolerances:
- MC walk, FP64 kernels: the same Philox draws drive the same decisions as
  the oracle; the FP64 sums agree to rounding, and the FP32 outputs to their
  own rounding (2e-7 relative), except where a comparison of a draw with a
  probability lands within rounding of it (not expected at these sizes; at
  most 2% of tuples may differ, each by at most 3 photons).
- MC walk, FP32 kernels: decisions flip where FP32 rounding crosses a draw;
  R and T must agree within 4 binomial sigmas (+1e-4).
- Network: operands are rounded to BF16 (relative 2^-9) and accumulated in
  FP32 through four layers, so outputs may differ from FP64 by a few 1e-3;
  against the oracle's BF16-operand definition (operands rounded, sums in
  FP64) they differ only by FP32 summation and the BF16 re-roundings it
  causes, held to a bound carried through the layers;
  the gradient vector must have cosine >= 0.999 with the oracle's and a
  relative L2 error <= 3e-2 per weight or bias tensor.  The embedding rows'
  gradient is the network's input gradient, a sum over 64 hidden units with
  terms of both signs: the cancellation raises its relative error (bounded
  by about 3 * 2^-9 * sum |terms| / |sum|), so it gets 6e-2.
"""
import math

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


def f32(a):
    return np.asarray(a, dtype=np.float32)


def mc_inputs(rng, m, rho_max=34.0):
    return dict(cos_i=f32(rng.uniform(0.05, 1.0, m)), lambda_nm=f32(rng.uniform(380, 780, m)),
                d_mm=f32(rng.uniform(2, 5, m)), rho_b=f32(rng.uniform(0, rho_max, m)),
                n=f32(rng.uniform(1.5, 1.58, m)), k=f32(10 ** rng.uniform(-7, -5, m)),
                alpha_tint=f32(rng.uniform(0, 0.5, m)))


def run_mc(gpu, inp, **kw):
    sdm, ctx, torch = gpu
    dev = {k: torch.from_numpy(v).cuda() for k, v in inp.items()}
    out = sdm.slab_mc(ctx, dev["cos_i"], dev["lambda_nm"], dev["d_mm"], dev["rho_b"], dev["n"], dev["k"],
                      dev["alpha_tint"], **kw)
    torch.cuda.synchronize()
    return [o.cpu().numpy().astype(np.float64) for o in out]


def run_mc_oracle(orc, inp, **kw):
    a = {k: v.astype(np.float64) for k, v in inp.items()}
    return orc.slab_mc(a["cos_i"], a["lambda_nm"], a["d_mm"], a["rho_b"], a["n"], a["k"], a["alpha_tint"], **kw)


# --------------------------------------------------------------------------
# Matrix-core lane layout
# --------------------------------------------------------------------------
def test_mfma_layout(gpu):
    """Small integers are exact in BF16 and their products and sums in FP32,
    so both products must equal numpy exactly."""
    sdm, ctx, torch = gpu
    rng = np.random.default_rng(0)
    A32 = rng.integers(-8, 9, (16, 32)).astype(np.float32)
    B32 = rng.integers(-8, 9, (32, 16)).astype(np.float32)
    A16 = rng.integers(-8, 9, (16, 16)).astype(np.float32)
    B16 = rng.integers(-8, 9, (16, 16)).astype(np.float32)
    t = [torch.from_numpy(x).cuda() for x in (A32, B32, A16, B16)]
    C32, C16 = sdm.debug_mfma(ctx, *t)
    torch.cuda.synchronize()
    assert np.array_equal(C32.cpu().numpy(), A32 @ B32)
    assert np.array_equal(C16.cpu().numpy(), A16 @ B16)


# --------------------------------------------------------------------------
# Bubbly-slab Monte Carlo
# --------------------------------------------------------------------------
def test_slab_mc_fp64_matches_oracle(gpu, orc):
    rng = np.random.default_rng(1)
    m, nph = 300, 97                 # 97 photons: runs of a tuple straddle waves
    inp = mc_inputs(rng, m)
    g = run_mc(gpu, inp, n_photons=nph, seed=123, tuple0=7, precision="fp64")
    o = run_mc_oracle(orc, inp, n_photons=nph, seed=123, tuple0=7)
    close = np.ones(m, dtype=bool)
    for gv, ov in zip(g, o):
        close &= np.abs(gv - ov) <= 2e-7 * np.abs(ov) + 1e-12
    bad = np.flatnonzero(~close)[:5]
    assert close.mean() >= 0.98, [(i, [float(x[i]) for x in g], [float(x[i]) for x in o]) for i in bad]
    for gv, ov in zip(g[:3], o[:3]):
        assert np.all(np.abs(gv - ov) <= 3.0 / nph)


def test_slab_mc_fp32_within_binomial_noise(gpu, orc):
    rng = np.random.default_rng(2)
    m, nph = 200, 512
    inp = mc_inputs(rng, m)
    g = run_mc(gpu, inp, n_photons=nph, seed=5, precision="fp32")
    o = run_mc_oracle(orc, inp, n_photons=nph, seed=5)
    for gv, ov in zip(g[:2], o[:2]):
        sig = np.sqrt(np.maximum(ov * (1 - ov), 1e-4) / nph)
        assert np.all(np.abs(gv - ov) <= 4 * sig + 1e-4)
    assert np.allclose(g[0] + g[1] + g[2], 1.0, atol=1e-5)


def test_slab_mc_edge_cases(gpu, orc):
    sdm, ctx, torch = gpu
    # no bubbles: the walk reduces to the closed-form slab (within MC noise)
    inp = dict(cos_i=f32([1.0, 0.3]), lambda_nm=f32([550, 700]), d_mm=f32([3, 2]), rho_b=f32([0, 0]),
               n=f32([1.52, 1.5]), k=f32([1e-7, 3e-6]), alpha_tint=f32([0, 0.1]))
    N = 100000
    R, T, A, W = run_mc(gpu, inp, n_photons=N, seed=9, precision="fp32")
    for i in range(2):
        Rr, Tr = orc.slab(*(float(inp[k][i]) for k in ("cos_i", "lambda_nm", "d_mm", "n", "k", "alpha_tint")))
        assert abs(R[i] - Rr) < 4 * math.sqrt(Rr * (1 - Rr) / N)
        assert abs(T[i] - Tr) < 4 * math.sqrt(Tr * (1 - Tr) / N)
        assert W[i] < 1e-3
    # single photon, single tuple; empty input; invalid arguments
    one = {k: v[:1] for k, v in inp.items()}
    g = run_mc(gpu, one, n_photons=1, seed=3, precision="fp64")
    o = run_mc_oracle(orc, one, n_photons=1, seed=3)
    assert all(abs(a[0] - b[0]) <= 2e-7 * abs(b[0]) + 1e-12 for a, b in zip(g, o))
    e = torch.empty(0, device="cuda")
    out = sdm.slab_mc(ctx, e, e, e, e, e, e)
    assert all(x.numel() == 0 for x in out)
    c = torch.ones(4, device="cuda")
    with pytest.raises(sdm.SdmError):
        sdm.slab_mc(ctx, c, c, c, c, c, c, n_photons=0)
    with pytest.raises(sdm.SdmError):
        sdm.slab_mc(ctx, c, c, c, c, c, c, rmin_um=50, rmax_um=10)
    with pytest.raises(sdm.SdmError):
        sdm.slab_mc(ctx, c, c, c, c, c, c, tuple0=2 ** 32 - 2)


# --------------------------------------------------------------------------
# Surrogate network
# --------------------------------------------------------------------------
def net_case(seed, m, n_panes, scale=1.0):
    rng = np.random.default_rng(seed)
    p = surrogate.init_params(n_panes, seed=seed)
    sp = surrogate.split(p, n_panes)
    sp["b1"][:] = rng.normal(0, 0.1, 64)
    sp["b4"][:] = [-2.0, 0.5, -1.0]
    sp["E"][:] *= 5.0
    p *= np.float32(scale)
    tup, pane = surrogate.random_tuples(m, n_panes, synth.LAMBDA_81, seed=seed + 1)
    target = np.stack([rng.uniform(0, 0.2, m), rng.uniform(0.4, 0.95, m), rng.uniform(0, 0.3, m)], 1)
    return p, tup, pane, target.astype(np.float32)


def to_dev(torch, *arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def test_mlp_forward_matches_oracle(gpu, orc):
    sdm, ctx, torch = gpu
    n_panes = 5
    p, tup, pane, _ = net_case(3, 1000, n_panes)
    net = sdm.MLP(ctx, n_panes, p)
    assert np.array_equal(net.params(), p)
    t, pn = to_dev(torch, tup, pane)
    y = net.infer(t, pn).cpu().numpy().astype(np.float64)
    yo = orc.mlp_forward(p.astype(np.float64), n_panes, tup.astype(np.float64), pane)
    err = np.abs(y - yo)
    assert err.max() < 1e-2 and err.mean() < 2e-3, (err.max(), err.mean())
    net.close()


def _bf16_forward_bound(p, n_panes, tup, pane, orc):
    """Per-sample bound on |GPU - oracle BF16 mode| for (R, T, w).

    Both sides take BF16 operands; the matrix cores sum the exact BF16
    products in FP32, which moves a pre-activation z by at most
    E = |W| D + gamma (|b| + |W| (|h| + D)), gamma = 65 u / (1 - 65 u),
    u = 2^-24, where D bounds how far the layer's inputs h already differ.
    After the ReLU the activation is rounded to BF16 again.  Rounding is
    monotone, so both sides' activations lie in
    [bf16(max(z - E, 0)), bf16(max(z + E, 0))]: D of the next layer is that
    interval's width, zero unless a BF16 rounding boundary falls within E of
    z.  The features start the chain the same way (the kernel scales them in
    FP32, within 4 ulp of the exact value; cos and the embedding are taken
    as they are).  The output bound is carried through the heads by their
    derivatives (R(1 - R), RT, T(1 - T); the softplus slope), with 5 % for
    second-order terms and 2e-6 for the heads' own FP32 rounding."""
    from paper_1912_05494_amd import surrogate as sg

    def rb(a):
        return orc.bf16(a).reshape(np.shape(a))

    v = sg.split(p.astype(np.float64), n_panes)
    gam = 65 * 2.0 ** -24 / (1 - 65 * 2.0 ** -24)
    x = np.concatenate([tup[:, :1], (tup[:, 1:2] - 580) / 200, (tup[:, 2:3] - 3.5) / 1.5, tup[:, 3:4] / 34,
                        v["E"][pane]], 1)
    ex = np.zeros_like(x)
    ex[:, 1:4] = 4 * 2.0 ** -24 * np.abs(x[:, 1:4])
    h = rb(x)
    D = rb(x + ex) - rb(x - ex)
    for k in (1, 2, 3, 4):
        Wb = rb(v[f"W{k}"])
        b = v[f"b{k}"]
        z = h @ Wb.T + b
        E = D @ np.abs(Wb).T + gam * (np.abs(b) + (np.abs(h) + D) @ np.abs(Wb).T)
        if k == 4:
            break
        h = rb(np.maximum(z, 0.0))
        D = rb(np.maximum(z + E, 0.0)) - rb(np.maximum(z - E, 0.0))
    o, do = z, E
    ea, eb = np.exp(o[:, 0]), np.exp(o[:, 1])
    R, T = ea / (ea + eb + 1), eb / (ea + eb + 1)
    bR = R * (1 - R) * do[:, 0] + R * T * do[:, 1]
    bT = R * T * do[:, 0] + T * (1 - T) * do[:, 1]
    bw = do[:, 2] / (1 + np.exp(-o[:, 2]))
    return 1.05 * np.stack([bR, bT, bw], 1) + 2e-6


def test_mlp_forward_within_bf16_bound(gpu, orc):
    """The matrix-core network against the oracle's plain BF16-operand
    definition: every output within the bound carried from FP32 summation
    and BF16 re-rounding (see _bf16_forward_bound)."""
    sdm, ctx, torch = gpu
    n_panes = 5
    p, tup, pane, _ = net_case(3, 1000, n_panes)
    net = sdm.MLP(ctx, n_panes, p)
    t, pn = to_dev(torch, tup, pane)
    y = net.infer(t, pn).cpu().numpy().astype(np.float64)
    yb = orc.mlp_forward_bf16(p.astype(np.float64), n_panes, tup.astype(np.float64), pane)
    bound = _bf16_forward_bound(p, n_panes, tup.astype(np.float64), pane, orc)
    err = np.abs(y - yb)
    print(f"bf16 forward: max err {err.max():.3e}, mean err {err.mean():.3e}, mean bound {bound.mean():.3e}, "
          f"max err/bound {(err / bound).max():.3f}")
    assert np.all(err <= bound), (err / bound).max()
    net.close()


def test_mlp_gradient_matches_oracle(gpu, orc):
    sdm, ctx, torch = gpu
    n_panes = 5
    for m in (1000, 37, 16):         # ragged tiles, one partial tile, one full tile
        p, tup, pane, target = net_case(4 + m, m, n_panes)
        net = sdm.MLP(ctx, n_panes, p)
        t, pn, tg = to_dev(torch, tup, pane, target)
        g, loss = net.grad(t, pn, tg)
        g = g.cpu().numpy().astype(np.float64)
        lo, go = orc.mlp_loss_grad(p.astype(np.float64), n_panes, tup.astype(np.float64), pane,
                                   target.astype(np.float64))
        assert loss == pytest.approx(lo, rel=2e-2)
        cos = g @ go / (np.linalg.norm(g) * np.linalg.norm(go))
        assert cos >= 0.999, (m, cos)
        gs, os_ = surrogate.split(g, n_panes), surrogate.split(go, n_panes)
        for name in gs:
            ref = os_[name]
            used = np.linalg.norm(ref)
            if used == 0.0:          # embedding rows of panes absent from the batch
                assert np.all(gs[name] == 0.0)
                continue
            rel = np.linalg.norm(gs[name] - ref) / used
            assert rel <= (6e-2 if name == "E" else 3e-2), (m, name, rel)
        net.close()


def test_mlp_training_is_reproducible(gpu):
    """The gradient pass writes each block's sums without atomics and the
    step sums the blocks in a fixed order: two trainings from the same state
    give the same parameters bit for bit, at a batch with one 64-sample group
    per block and at one with several groups per block and a ragged tail."""
    sdm, ctx, torch = gpu
    n_panes = 7
    p, tup, pane, target = net_case(21, 1 << 16, n_panes)
    t, pn, tg = to_dev(torch, tup, pane, target)
    for batch in (8192, 40000 + 37):
        runs = []
        for _ in range(2):
            net = sdm.MLP(ctx, n_panes, p)
            curve = net.train(t, pn, tg, steps=12, batch=batch, lr=2e-3)
            runs.append((net.params(), curve))
            net.close()
        assert np.array_equal(runs[0][0], runs[1][0]), batch
        assert np.array_equal(runs[0][1], runs[1][1]), batch
        assert not np.array_equal(runs[0][0], p)


def test_mlp_adam_first_step(gpu, orc):
    """With zero moments, Adam's first step is lr * g / (|g| + eps): each
    parameter with a clear gradient moves by lr against the gradient's sign."""
    sdm, ctx, torch = gpu
    n_panes = 3
    p, tup, pane, target = net_case(11, 512, n_panes)
    net = sdm.MLP(ctx, n_panes, p)
    t, pn, tg = to_dev(torch, tup, pane, target)
    lr = 1e-3
    net.train(t, pn, tg, steps=1, batch=512, lr=lr)
    step = net.params().astype(np.float64) - p
    _, go = orc.mlp_loss_grad(p.astype(np.float64), n_panes, tup.astype(np.float64), pane,
                              target.astype(np.float64))
    clear = np.abs(go) > 1e-2 * np.abs(go).max()
    assert clear.sum() > 100
    agree = np.sign(step[clear]) == -np.sign(go[clear])
    assert agree.mean() >= 0.99
    assert np.allclose(np.abs(step[clear][agree]), lr, rtol=1e-3)
    net.close()


def test_mlp_training_fits_mc_data(gpu, orc):
    """End to end: MC targets from the GPU walk, Adam on the matrix cores; the
    fitted network must beat the best constant predictor by a wide margin."""
    sdm, ctx, torch = gpu
    n_panes, m = 2, 8192
    rng = np.random.default_rng(21)
    tup, pane = surrogate.random_tuples(m, n_panes, synth.LAMBDA_81, seed=22)
    nk = np.array([[1.52, 2e-7, 0.05], [1.55, 4e-6, 0.3]], dtype=np.float32)[pane]
    dev = to_dev(torch, *(np.ascontiguousarray(x) for x in (tup[:, 0], tup[:, 1], tup[:, 2], tup[:, 3],
                                                           nk[:, 0], nk[:, 1], nk[:, 2])))
    R, T, A, W = sdm.slab_mc(ctx, *dev, n_photons=256, seed=4)
    target = torch.stack([R, T, W], 1).contiguous()
    p = surrogate.init_params(n_panes, seed=5)
    net = sdm.MLP(ctx, n_panes, p)
    t, pn = to_dev(torch, tup, pane)
    curve = net.train(t, pn, target, steps=1500, batch=1024, lr=2e-3)
    assert np.all(np.isfinite(curve))
    y = net.infer(t, pn)
    mse = float(((y - target) ** 2).sum(1).mean())
    const = float(((target - target.mean(0)) ** 2).sum(1).mean())
    assert mse < 0.2 * const, (mse, const)
    assert curve[-50:].mean() < 0.5 * curve[:10].mean()
    net.close()


def test_mlp_invalid_inputs(gpu):
    sdm, ctx, torch = gpu
    p = surrogate.init_params(2, seed=0)
    with pytest.raises(sdm.SdmError):
        sdm.MLP(ctx, 0, surrogate.init_params(0, seed=0))
    with pytest.raises(sdm.SdmError):
        sdm.MLP(ctx, 65, surrogate.init_params(65, seed=0))
    net = sdm.MLP(ctx, 2, p)
    tup, pane = surrogate.random_tuples(40, 2, synth.LAMBDA_81, seed=1)
    pane[17] = 2                     # out of range
    t, pn = to_dev(torch, tup, pane)
    with pytest.raises(sdm.SdmError):
        net.infer(t, pn)
    tg = torch.zeros((40, 3), device="cuda")
    with pytest.raises(sdm.SdmError):
        net.grad(t, pn, tg)
    pane[17] = 1
    t, pn = to_dev(torch, tup, pane)
    assert net.infer(t, pn).shape == (40, 3)
    with pytest.raises(sdm.SdmError):
        net.train(t, pn, tg, steps=1, batch=41)
    net.close()


def test_mlp_error_table_matches_oracle(gpu, orc):
    """Per-cell largest |R - R*| or |T - T*|: the GPU network against targets,
    compared with the oracle's BF16-operand network binned the same way."""
    sdm, ctx, torch = gpu
    n_panes, m, dims = 3, 6000, (8, 3, 4)
    p, tup, pane, _ = net_case(31, m, n_panes)
    y = orc.mlp_forward_bf16(p.astype(np.float64), n_panes, tup.astype(np.float64), pane)
    rng = np.random.default_rng(5)
    target = (y + rng.normal(0, 0.01, y.shape)).astype(np.float32)
    net = sdm.MLP(ctx, n_panes, p)
    t, pn, tg = to_dev(torch, tup, pane, target)
    tab = net.error_table(t, pn, tg, dims=dims).cpu().numpy()
    f = np.float32
    ic = np.clip((tup[:, 0] * f(dims[0])).astype(np.int64), 0, dims[0] - 1)
    idd = np.clip(((tup[:, 2] - f(2)) / f(3) * f(dims[1])).astype(np.int64), 0, dims[1] - 1)
    ir = np.clip((tup[:, 3] / f(34) * f(dims[2])).astype(np.int64), 0, dims[2] - 1)
    e = np.maximum(np.abs(y[:, 0] - target[:, 0]), np.abs(y[:, 1] - target[:, 1]))
    ref = np.zeros((n_panes,) + dims)
    np.maximum.at(ref, (pane, ic, idd, ir), e)
    assert np.array_equal(tab > 0, ref > 0)
    assert np.allclose(tab, ref, atol=1e-3)
    pane[0] = n_panes
    t, pn = to_dev(torch, tup, pane)
    with pytest.raises(sdm.SdmError):
        net.error_table(t, pn, tg, dims=dims)
    net.close()
