"""Surrogate BTDF of bubbly glass: parameter layout and seeded initial
weights (inputs of the training), plus thin wrappers of the library's
training and inference entry points.

Network: 12 -> 64 -> 64 -> 64 -> 3 with ReLU; inputs (cos(theta), lambda,
thickness, bubble density, 8-value pane embedding); outputs (R, T, lobe width).
The forward/backward passes, the loss and the optimiser run in the HIP
library (BF16 MFMA with FP32 accumulation); this module only lays out and
initialises parameters and marshals arguments.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT, N_EMB = 12, 64, 3, 8
#: (name, shape) in the order of the flat parameter vector
LAYOUT = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_HID, N_HID)), ("b3", (N_HID,)), ("W4", (N_OUT, N_HID)), ("b4", (N_OUT,))]
RHO_MAX = 34.0   # bubbles per mm^3 at a volume fraction of 0.3 for r in [10, 200] um


def n_params(n_panes):
    return sum(int(np.prod(s)) for _, s in LAYOUT) + N_EMB * n_panes


def init_params(n_panes, seed=0):
    """He-uniform weights, zero biases, N(0, 0.1) embeddings (float32)."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in LAYOUT:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shape[1]) * (0.1 if name == "W4" else 1.0)
            parts.append(rng.uniform(-lim, lim, size=shape).reshape(-1))
        else:
            parts.append(np.zeros(shape).reshape(-1))
    parts.append(rng.normal(0.0, 0.1, size=N_EMB * n_panes))
    return np.concatenate(parts).astype(np.float32)


def split(params, n_panes):
    """Views of the flat vector by name (plus 'E' for the embeddings)."""
    out, o = {}, 0
    for name, shape in LAYOUT:
        k = int(np.prod(shape))
        out[name] = params[o:o + k].reshape(shape)
        o += k
    out["E"] = params[o:o + N_EMB * n_panes].reshape(n_panes, N_EMB)
    return out


def random_tuples(n, n_panes, lambdas, seed=0, rho_max=RHO_MAX, d_range=(2.0, 5.0)):
    """Training inputs: cos(theta) ~ U(0, 1], lambda on the grid, thickness ~
    U(2, 5) mm, bubble density ~ U(0, rho_max), pane ~ U{0..n_panes-1}."""
    rng = np.random.default_rng(seed)
    tup = np.empty((n, 4), dtype=np.float32)
    tup[:, 0] = 1.0 - rng.random(n)
    tup[:, 1] = rng.choice(np.asarray(lambdas, dtype=np.float32), n)
    tup[:, 2] = rng.uniform(*d_range, n)
    tup[:, 3] = rng.uniform(0.0, rho_max, n)
    pane = rng.integers(0, n_panes, n).astype(np.int32)
    return tup, pane


def scene_tuples(materials, tab_lambda, n, lambdas, seed=0, own=0.0, n_ref_nm=560.0):
    """Training or validation inputs for the bubbly materials of a scene, by
    pane type (a material's pane_id; the materials of one type share n, k and
    tint): tuples (cos, lambda, d, rho) and pane types from random_tuples,
    and per tuple the type's (n, k, tint) at lambda and its n at n_ref_nm,
    interpolated linearly in the material tables.  A fraction `own` of the
    tuples is moved to the density of one of its type's panes."""
    from .synth import GLASS_BUBBLY
    by_type = {}
    for m in materials:
        if m.type == GLASS_BUBBLY:
            by_type.setdefault(int(m.pane_id), []).append(m)
    n_types = max(by_type) + 1
    if sorted(by_type) != list(range(n_types)):
        raise ValueError("pane types of the bubbly materials must be 0 .. n-1")
    tup, pane = random_tuples(n, n_types, lambdas, seed=seed)
    if own > 0.0:
        sel = np.flatnonzero(np.random.default_rng(seed + 1).random(n) < own)
        pick = np.random.default_rng(seed + 2).random(len(sel))
        for q in range(n_types):
            dq = np.array([m.bubble_density for m in by_type[q]], dtype=np.float32)
            s = sel[pane[sel] == q]
            tup[s, 3] = dq[np.minimum((pick[pane[sel] == q] * len(dq)).astype(np.int64), len(dq) - 1)]
    tab = np.asarray(tab_lambda, dtype=np.float64)
    nk = np.empty((n, 4), dtype=np.float32)
    for q in range(n_types):
        m = by_type[q][0]
        sel = pane == q
        lam = tup[sel, 1].astype(np.float64)
        nk[sel, 0] = np.interp(lam, tab, m.n)
        nk[sel, 1] = np.interp(lam, tab, m.k)
        nk[sel, 2] = np.interp(lam, tab, m.alpha_tint)
        nk[sel, 3] = np.interp(n_ref_nm, tab, m.n)
    return tup, pane, nk


def mc_targets(ctx, tup, nk, n_photons, seed, device):
    """(R, T, lobe width) of each tuple from the library's slab Monte Carlo:
    a device tensor [m, 3]."""
    import torch
    from . import sdm
    t = [torch.from_numpy(np.ascontiguousarray(a)).to(device) for a in
         (tup[:, 0], tup[:, 1], tup[:, 2], tup[:, 3], nk[:, 0], nk[:, 1], nk[:, 2], nk[:, 3])]
    R, T, A, Wl = sdm.slab_mc(ctx, *t[:7], n_ref=t[7], n_photons=n_photons, seed=seed)
    return torch.stack([R, T, Wl], 1).contiguous()


def train_stepped(net, tuples, panes, target, steps, batch=8192):
    """Adam at a stepped learning rate: half the steps at 2e-3, a third at
    5e-4, the rest at 1e-4.  Returns the loss curve."""
    n1, n2 = steps // 2, steps // 3
    curves = [net.train(tuples, panes, target, steps=s, batch=batch, lr=lr)
              for s, lr in ((n1, 2e-3), (n2, 5e-4), (steps - n1 - n2, 1e-4)) if s > 0]
    return np.concatenate(curves) if curves else np.zeros(0, dtype=np.float32)
