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


def test_issue_probe_overlap_class():
    """The issue probe's class 9 (class 5's MFMA chains and class 0's FMA
    chains in one loop) counts its MFMA instructions like class 5; classes
    outside 0 ... 9 are refused."""
    ctx = gbd.Context(0)
    ms5, n5 = gbd.gbd_issue_probe(ctx, 5, 64)
    ms9, n9 = gbd.gbd_issue_probe(ctx, 9, 64)
    ms0, _ = gbd.gbd_issue_probe(ctx, 0, 64)
    assert n9 == n5 and ms9 > 0 and ms5 > 0 and ms0 > 0
    with pytest.raises(gbd.GbdError):
        gbd.gbd_issue_probe(ctx, 10, 64)
