"""Pins of the oracle's surrogate network: the analytic gradient against
central finite differences, and the output heads' constraints."""
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
