"""Pins of the oracle's surrogate network: the analytic gradient against
central finite differences, the output heads' constraints, the forward pass
against a numpy network written from the parameter layout and against one
path worked out by hand, and the BF16 mode as operand rounding only (BF16
rounding straight from the double, pinned on midpoint cases)."""
import math

import numpy as np
import pytest

from paper_1912_05494_amd import surrogate


def _batch(rng, m, n_panes):
    tup = np.stack([rng.uniform(0.05, 1, m), rng.uniform(380, 780, m), rng.uniform(2, 5, m),
                    rng.uniform(0, 34, m)], axis=1)
    return tup, rng.integers(0, n_panes, m).astype(np.int32)


def test_parameter_count(orc):
    assert orc.mlp_nparams(0) == 9347
    assert orc.mlp_nparams(3) == 9347 + 24
    assert surrogate.n_params(3) == orc.mlp_nparams(3)


def test_gradient_matches_finite_differences(orc):
    rng = np.random.default_rng(0)
    n_panes = 3
    p = surrogate.init_params(n_panes, seed=1).astype(np.float64)
    tup, pane = _batch(rng, 16, n_panes)
    target = np.stack([rng.uniform(0, 0.2, 16), rng.uniform(0.5, 0.95, 16), rng.uniform(0, 0.3, 16)], 1)
    loss, g = orc.mlp_loss_grad(p, n_panes, tup, pane, target)
    h = 1e-6
    idx = np.concatenate([rng.choice(len(p), 300, replace=False), np.arange(len(p) - 24, len(p))])
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (orc.mlp_loss_grad(pp, n_panes, tup, pane, target)[0] -
              orc.mlp_loss_grad(pm, n_panes, tup, pane, target)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-9), i


def test_heads_constraints(orc):
    rng = np.random.default_rng(2)
    p = surrogate.init_params(2, seed=3).astype(np.float64) * 3.0
    tup, pane = _batch(rng, 500, 2)
    y = orc.mlp_forward(p, 2, tup, pane)
    assert np.all(y[:, 0] > 0) and np.all(y[:, 1] > 0) and np.all(y[:, 0] + y[:, 1] < 1)
    assert np.all(y[:, 2] > 0)
    # softmax over (o0, o1, 0): R / (1 - R - T) = exp(o0) cannot be checked
    # without o, but the third share is positive and the shares sum to 1
    assert np.all(1 - y[:, 0] - y[:, 1] > 0)


def test_loss_is_mean_squared_error(orc):
    rng = np.random.default_rng(4)
    p = surrogate.init_params(1, seed=5).astype(np.float64)
    tup, pane = _batch(rng, 37, 1)
    y = orc.mlp_forward(p, 1, tup, pane)
    target = rng.uniform(0, 1, (37, 3))
    loss, _ = orc.mlp_loss_grad(p, 1, tup, pane, target)
    assert loss == pytest.approx(np.mean(np.sum((y - target) ** 2, axis=1)), rel=1e-13)


# --------------------------------------------------------------------------
# The forward pass, pinned outside the oracle's own loss and gradient
# --------------------------------------------------------------------------
def _numpy_forward(params, n_panes, tup, pane, rnd=None):
    """The network written out with numpy on the named parameter views:
    features, three ReLU layers of 64, the (R, T) shares of a softmax over
    (o0, o1, 0) and a softplus width.  rnd (optional) rounds every operand
    that enters a product."""
    r = rnd if rnd is not None else (lambda a: a)
    v = surrogate.split(np.asarray(params, dtype=np.float64), n_panes)
    x = np.concatenate([tup[:, 0:1], (tup[:, 1:2] - 580.0) / 200.0, (tup[:, 2:3] - 3.5) / 1.5,
                        tup[:, 3:4] / 34.0, v["E"][pane]], axis=1)
    h = r(x)
    for k in (1, 2, 3):
        h = r(np.maximum(h @ r(v[f"W{k}"]).T + v[f"b{k}"], 0.0))
    o = h @ r(v["W4"]).T + v["b4"]
    den = np.exp(o[:, 0]) + np.exp(o[:, 1]) + 1.0
    return np.stack([np.exp(o[:, 0]) / den, np.exp(o[:, 1]) / den, np.log1p(np.exp(o[:, 2]))], axis=1)


def _bf16_round(a):
    """Nearest value with an 8-bit significand, ties to even (numpy's round
    is half-to-even, and scaling by powers of two is exact)."""
    f, e = np.frexp(np.asarray(a, dtype=np.float64))
    return np.ldexp(np.round(np.ldexp(f, 8)), e - 8)


def test_forward_matches_numpy_network(orc):
    rng = np.random.default_rng(7)
    n_panes = 4
    p = surrogate.init_params(n_panes, seed=8).astype(np.float64)
    sp = surrogate.split(p, n_panes)
    for k in (1, 2, 3):
        sp[f"b{k}"][:] = rng.normal(0, 0.2, 64)      # nonzero biases: a dropped bias would show
    sp["b4"][:] = [-1.5, 0.7, -0.3]
    sp["E"][:] *= 4.0
    tup, pane = _batch(rng, 400, n_panes)
    y = orc.mlp_forward(p, n_panes, tup, pane)
    ref = _numpy_forward(p, n_panes, tup, pane)
    assert np.allclose(y, ref, rtol=1e-12, atol=1e-14)
    # the ReLUs are active: a sizeable share of hidden units is cut
    x = np.concatenate([tup[:, :1], (tup[:, 1:2] - 580) / 200, (tup[:, 2:3] - 3.5) / 1.5, tup[:, 3:4] / 34,
                        sp["E"][pane]], 1)
    z1 = x @ sp["W1"].T + sp["b1"]
    assert 0.2 < np.mean(z1 < 0) < 0.8


def test_forward_hand_computed_path(orc):
    """One path through the network by hand.  Pane 1's embedding is one-hot
    at its third value (feature 6); W1[5][6] = 2, W2[9][5] = 3, W3[4][9] = 0.5,
    W4[0][4] = 1, W4[2][4] = -1, every other weight 0; biases b1[5] = -0.5,
    b1[7] = -1 (unit 7 stays cut by its ReLU, as it has no input), b4 =
    (0, ln 2, 0).  With cos = 0.3, lambda = 780, d = 5, rho = 34:
    z1[5] = 2 * 1 - 0.5 = 1.5, z2[9] = 3 * 1.5 = 4.5, z3[4] = 2.25,
    o = (2.25, ln 2, -2.25), so R = e^2.25 / (e^2.25 + 2 + 1), T = 2 / (same),
    w = ln(1 + e^-2.25).  A transposed weight matrix, a dropped ReLU or a
    dropped bias changes these."""
    n_panes = 2
    p = np.zeros(orc.mlp_nparams(n_panes))
    v = surrogate.split(p, n_panes)
    v["E"][1, 2] = 1.0
    v["W1"][5, 6] = 2.0
    v["b1"][5] = -0.5
    v["b1"][7] = -1.0
    v["W1"][3, 0] = -4.0                  # unit 3: -4 cos < 0, cut by the ReLU
    v["W2"][9, 5] = 3.0
    v["W2"][9, 3] = 100.0                 # would add 100 * (-1.2) if the ReLU were missing
    v["W2"][9, 7] = 50.0                  # would add 50 * (-1) if the ReLU were missing
    v["W3"][4, 9] = 0.5
    v["W4"][0, 4] = 1.0
    v["W4"][2, 4] = -1.0
    v["b4"][:] = [0.0, math.log(2.0), 0.0]
    tup = np.array([[0.3, 780.0, 5.0, 34.0], [0.3, 780.0, 5.0, 34.0]])
    pane = np.array([1, 0], dtype=np.int32)
    y = orc.mlp_forward(p, n_panes, tup, pane)
    e = math.exp(2.25)
    assert y[0, 0] == pytest.approx(e / (e + 3.0), rel=1e-14)
    assert y[0, 1] == pytest.approx(2.0 / (e + 3.0), rel=1e-14)
    assert y[0, 2] == pytest.approx(math.log1p(math.exp(-2.25)), rel=1e-14)
    # pane 0 has a zero embedding: only b4 remains, o = (0, ln 2, 0)
    assert y[1, 0] == pytest.approx(1.0 / 4.0, rel=1e-14)
    assert y[1, 1] == pytest.approx(2.0 / 4.0, rel=1e-14)
    assert y[1, 2] == pytest.approx(math.log(2.0), rel=1e-14)
    # the feature scaling: lambda = 780 -> 1, d = 5 -> 1, rho = 34 -> 1 carry
    # W1 columns 1, 2, 3 into unit 5 (+1 each), and cos = 0.3 through column 0
    v["W1"][5, 0:4] = [1.0, 1.0, 1.0, 1.0]
    y2 = orc.mlp_forward(p, n_panes, tup[:1], pane[:1])
    z3 = 0.5 * 3.0 * (1.5 + 0.3 + 1.0 + 1.0 + 1.0)
    e2 = math.exp(z3)
    assert y2[0, 0] == pytest.approx(e2 / (e2 + 3.0), rel=1e-14)
    assert y2[0, 2] == pytest.approx(math.log1p(math.exp(-z3)), rel=1e-14)


def test_bf16_rounding_direct_from_double(orc):
    """Rounding a double straight to 8 significant bits: 1 + 2^-8 + 2^-30 lies
    above the midpoint between 1 and 1 + 2^-7 and rounds up (going through
    float32 first would land on the midpoint and round to 1); exact
    midpoints go to the even significand."""
    assert orc.bf16(1 + 2 ** -8 + 2 ** -30) == 1 + 2 ** -7
    assert orc.bf16(1 + 2 ** -8) == 1.0
    assert orc.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6
    assert orc.bf16(-(1 + 3 * 2 ** -8)) == -(1 + 2 ** -6)
    assert orc.bf16(3 * 2 ** -140) == 3 * 2 ** -140
    rng = np.random.default_rng(11)
    x = rng.normal(0, 10, 3000) * np.exp2(rng.integers(-40, 40, 3000))
    assert np.array_equal(orc.bf16(x), _bf16_round(x))


def test_bf16_forward_is_operand_rounding_only(orc):
    """The BF16 mode rounds the features, the weights and the hidden
    activations where they enter a product, and computes everything else in
    FP64: the numpy network with the same roundings agrees to 1e-12."""
    rng = np.random.default_rng(12)
    n_panes = 3
    p = surrogate.init_params(n_panes, seed=13).astype(np.float64)
    sp = surrogate.split(p, n_panes)
    for k in (1, 2, 3):
        sp[f"b{k}"][:] = rng.normal(0, 0.2, 64)
    sp["b4"][:] = [-2.0, 0.5, -1.0]
    tup, pane = _batch(rng, 300, n_panes)
    y = orc.mlp_forward_bf16(p, n_panes, tup, pane)
    ref = _numpy_forward(p, n_panes, tup, pane, rnd=_bf16_round)
    assert np.allclose(y, ref, rtol=1e-12, atol=1e-14)
    # and the rounding matters: the FP64 network differs by more than that
    assert np.abs(orc.mlp_forward(p, n_panes, tup, pane) - y).max() > 1e-5


def _fp32_sum_forward(orc, p, n_panes, tup, pane, perm):
    """The network as a matrix-core evaluation computes it, emulated: features
    scaled in FP32, BF16 operands, each dot product summed in FP32 in the
    order `perm` (a permutation of the inputs, bias first), ReLU, BF16
    re-rounding; heads in FP64."""
    sp = surrogate.split(p.astype(np.float64), n_panes)
    f32 = np.float32
    x = [f32(tup[0]), (f32(tup[1]) - f32(580)) * f32(0.005), (f32(tup[2]) - f32(3.5)) / f32(1.5),
         f32(tup[3]) / f32(34)] + [f32(e) for e in sp["E"][pane]]
    h = np.asarray(orc.bf16(np.array([float(v) for v in x])), dtype=np.float64).reshape(-1)
    for k in (1, 2, 3, 4):
        W = orc.bf16(sp[f"W{k}"].ravel()).reshape(sp[f"W{k}"].shape)
        b = sp[f"b{k}"].astype(np.float32)
        z = np.empty(W.shape[0])
        order = [int(i) for i in perm if i < W.shape[1]]
        for o in range(W.shape[0]):
            s = f32(b[o])
            for i in order:
                s = f32(s + f32(W[o, i] * h[i]))
            z[o] = s
        if k < 4:
            h = np.asarray(orc.bf16(np.maximum(z, 0.0)), dtype=np.float64).reshape(-1)
    ea, eb = math.exp(z[0]), math.exp(z[1])
    return np.array([ea / (ea + eb + 1), eb / (ea + eb + 1), z[2] if z[2] > 30 else math.log1p(math.exp(z[2]))])


def test_bf16_bound_covers_fp32_summation(orc):
    """orc_mlp_bf16_bound: its outputs are the BF16-mode forward's exactly,
    and an FP32-sum evaluation (emulated in numpy, two summation orders, with
    the cos and thickness inputs moved by up to the stated input errors) lies
    within the bound; the bound is not vacuous (typically a few 1e-6; larger
    only where a BF16 re-rounding may go either way)."""
    rng = np.random.default_rng(12)
    n_panes = 3
    p = surrogate.init_params(n_panes, seed=4).astype(np.float64)
    sp = surrogate.split(p, n_panes)
    sp["b4"][:] = [-1.0, 0.5, -2.0]
    sp["E"][:] *= 8.0
    tup, pane = _batch(rng, 40, n_panes)
    worst, bounds = 0.0, []
    for s in range(len(tup)):
        e_cos, e_d = 3e-7, 2e-6
        out, bnd = orc.mlp_bf16_bound(p, tup[s], pane[s], e_cos, e_d)
        ref = orc.mlp_forward_bf16(p, n_panes, tup[s:s + 1], pane[s:s + 1])[0]
        assert np.array_equal(out, ref)
        bounds.append(bnd)
        for perm in (np.arange(64), rng.permutation(64)):
            for dc, dd in ((0.0, 0.0), (e_cos, -e_d), (-e_cos, e_d)):
                t = tup[s].copy()
                t[0] += dc
                t[2] += dd
                got = _fp32_sum_forward(orc, p, n_panes, t, pane[s], perm)
                err = np.abs(got - out)
                assert np.all(err <= bnd), (s, err, bnd)
                worst = max(worst, float((err / bnd).max()))
    assert worst > 1e-3        # the emulation does differ from the FP64 sums
    assert np.median(bounds) < 1e-4
