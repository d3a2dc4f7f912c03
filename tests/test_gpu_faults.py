"""Injected allocation failures: with SDM_FAIL_ALLOC=n in the environment
when a context is created, the n-th device allocation of the library from
then on fails once.  For every n that falls inside a scene upload or a
render (FP64, tiny scene; a network creation), the failing call reports
SDM_E_NOMEM and leaves the library usable: the same calls made again
succeed, and the image equals the one rendered without a fault (to the
order of the FP64 accumulation).
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


def armed_context(sdm, n):
    """A context created with SDM_FAIL_ALLOC=n (n = 0 disarms)."""
    os.environ["SDM_FAIL_ALLOC"] = str(n)
    try:
        return sdm.Context(0)
    finally:
        del os.environ["SDM_FAIL_ALLOC"]


def render64(sdm, ctx, scene, st):
    gs = sdm.Scene(ctx, scene)
    try:
        spec, _, _ = sdm.render(ctx, gs, st, precision="fp64")
        return spec.cpu().numpy().astype(np.float64)
    finally:
        gs.close()


def test_injected_allocation_failures(gpu):
    sdm, ctx0, torch = gpu
    scene = synth.tiny_scene()
    st = synth.tiny_settings(spp=4, W=32, H=32)
    ref = render64(sdm, ctx0, scene, st)
    failed_at = []
    try:
        for n in range(1, 64):
            ctx = armed_context(sdm, n)
            try:
                try:
                    render64(sdm, ctx, scene, st)
                except sdm.SdmError as e:
                    assert e.code == sdm.SDM_E_NOMEM, e
                    failed_at.append(n)
                # the fault has fired, or n lies past the calls' allocations
                # (then disarm it before the calls are made again)
                armed_context(sdm, 0).close()
                out = render64(sdm, ctx, scene, st)
                assert np.allclose(out, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
            finally:
                ctx.close()
            if not failed_at or failed_at[-1] != n:
                break
    finally:
        armed_context(sdm, 0).close()
    print(f"allocations that failed and recovered: {failed_at}")
    assert len(failed_at) >= 5 and failed_at == list(range(1, len(failed_at) + 1))


def test_injected_failure_in_network_creation(gpu):
    sdm, _, torch = gpu
    try:
        ctx = armed_context(sdm, 1)
        try:
            with pytest.raises(sdm.SdmError) as ei:
                sdm.MLP(ctx, 3, surrogate.init_params(3, seed=0))
            assert ei.value.code == sdm.SDM_E_NOMEM
            net = sdm.MLP(ctx, 3, surrogate.init_params(3, seed=0))
            assert net.params().shape[0] == surrogate.init_params(3, seed=0).shape[0]
            net.close()
        finally:
            ctx.close()
    finally:
        armed_context(sdm, 0).close()
