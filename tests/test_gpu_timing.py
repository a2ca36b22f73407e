"""GPU test of the kernel-timing entry points (gbd_ctx_set_kernel_timing,
gbd_ctx_kernel_times): one duration per evaluation while enabled, none while
disabled or on the allocation-free path, fields unchanged bit for bit."""
import numpy as np
import pytest
import torch

import paper_2404_12454_amd as gbd
from paper_2404_12454_amd import scenes
from gbd_testutil import ensure_library

pytestmark = pytest.mark.gpu


def test_kernel_timing_counts_and_leaves_fields_unchanged():
    ensure_library()
    ctx = gbd.Context(0)
    sc = scenes.airy_scene(32, npix=96, npix_y=80, half_span_lamF=8.0)
    plan = gbd.Plan(ctx, sc.n).setup(gbd.beamlets_from_scene(ctx, sc), gbd.plane_from_scene(ctx, sc))
    ref = {v: plan.eval(gbd.GBD_MIXED, opts=dict(variant=v)).cpu().numpy() for v in (3, 4, 5)}
    assert ctx.kernel_times() == []  # timing off: nothing recorded
    ctx.set_kernel_timing(True)
    got = {v: plan.eval(gbd.GBD_MIXED, opts=dict(variant=v)).cpu().numpy() for v in (3, 4, 5)}
    E64 = plan.eval(gbd.GBD_FP64)
    plan.eval_noalloc(gbd.GBD_MIXED)  # the allocation-free path records nothing
    ctx.set_kernel_timing(False)
    plan.eval(gbd.GBD_MIXED)
    torch.cuda.synchronize()
    t = ctx.kernel_times()
    print("kernel ms", t, flush=True)
    assert len(t) == 4 and all(0.0 < x < 1000.0 for x in t)
    assert ctx.kernel_times() == []  # taken once
    for v in (3, 4, 5):
        assert np.array_equal(ref[v], got[v]), v
    assert E64.dtype == torch.complex128
