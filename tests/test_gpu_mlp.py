"""GPU tests of the surrogate network kernels against the FP64 reference
network (oracle/mlp.py, itself pinned by finite differences).

FP32 mode: forward and gradients within 1e-5 (relative L2); BF16 MFMA mode
(hidden products with BF16 operands): within 1e-2 and cosine >= 0.999 against
the reference evaluated with the same BF16-rounded hidden weights.  This also
checks the MFMA operand / result lane layout the kernel assumes."""
import numpy as np
import pytest

import paper_2404_12454_amd as gbd
from oracle import mlp as ref
from gbd_testutil import ensure_library

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    ensure_library()
    return gbd.Context(0)


def bf16_round(a):
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32)


def hidden_rounded(params, shapes):
    """Round the hidden layers' weight matrices to BF16 (biases and head stay FP32)."""
    p = np.array(params, np.float64)
    k = 0
    for li, (o, i) in enumerate(shapes):
        if li < len(shapes) - 1:
            p[k:k + o * i] = bf16_round(p[k:k + o * i])
        k += o * i + o
    return p


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def setup(ctx, mode, B=200, width=128, seed=0):
    import torch
    shapes = ref.layer_shapes(5, width, 3)
    p = ref.init_params(shapes, seed=seed).astype(np.float32)
    net = gbd.Mlp(ctx, 5, width, 3, 256, mode)
    assert net.num_params == ref.num_params(shapes)
    net.set_params(p)
    rng = np.random.default_rng(seed + 1)
    X = rng.normal(size=(B, 5)).astype(np.float32)
    y = rng.normal(size=B).astype(np.float32)
    return shapes, p, net, X, y, torch.tensor(X, device="cuda"), torch.tensor(y, device="cuda")


def test_forward_fp32_and_bf16(ctx):
    import torch
    for mode, tol in ((gbd.GBD_MLP_FP32, 1e-5), (gbd.GBD_MLP_BF16, 1e-2)):
        shapes, p, net, X, y, Xd, yd = setup(ctx, mode)
        out = net.forward(Xd)
        torch.cuda.synchronize()
        pr = p.astype(np.float64) if mode == gbd.GBD_MLP_FP32 else hidden_rounded(p, shapes)
        want, _ = ref.forward(pr, X.astype(np.float64), shapes)
        e = rel(out.cpu().numpy(), want)
        print("forward mode", mode, e, flush=True)
        assert e < tol


def test_gradients_fp32_mode(ctx):
    import torch
    shapes, p, net, X, y, Xd, yd = setup(ctx, gbd.GBD_MLP_FP32, seed=4)
    loss = torch.zeros(1, device="cuda")
    net.backward(Xd, yd, loss_out=loss)
    torch.cuda.synchronize()
    L, g = ref.loss_and_grad(p.astype(np.float64), X.astype(np.float64), y.astype(np.float64), shapes)
    gg = net.get_grads()
    print("fp32 grad rel", rel(gg, g), "loss", float(loss.cpu()), L, flush=True)
    assert rel(gg, g) < 1e-5
    assert abs(float(loss.cpu()) - L) <= 1e-5 * L


def test_gradients_bf16_mode(ctx):
    shapes, p, net, X, y, Xd, yd = setup(ctx, gbd.GBD_MLP_BF16, seed=5)
    net.backward(Xd, yd)
    L, g = ref.loss_and_grad(hidden_rounded(p, shapes), X.astype(np.float64), y.astype(np.float64), shapes)
    gg = net.get_grads().astype(np.float64)
    cos = float(gg @ g / np.linalg.norm(gg) / np.linalg.norm(g))
    print("bf16 grad rel", rel(gg, g), "cos", cos, flush=True)
    assert rel(gg, g) < 1e-2 and cos > 0.999


def test_row_gather_equals_contiguous(ctx):
    import torch
    shapes, p, net, X, y, Xd, yd = setup(ctx, gbd.GBD_MLP_FP32, B=64)
    rows = torch.tensor(np.arange(63, -1, -1, dtype=np.int32), device="cuda")
    a = net.forward(Xd, rows=rows).cpu().numpy()
    b = net.forward(Xd).cpu().numpy()
    assert np.array_equal(a, b[::-1])


def test_adamw_matches_reference(ctx):
    shapes, p, net, X, y, Xd, yd = setup(ctx, gbd.GBD_MLP_FP32, seed=6)
    net.backward(Xd, yd)
    g = net.get_grads().astype(np.float64)
    net.adamw(1e-3, 0.9, 0.999, 1e-8, 1e-2)
    want, m, v = ref.adamw_step(p.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, 1e-3, 0.9, 0.999,
                                1e-8, 1e-2)
    got = net.get_params().astype(np.float64)
    assert np.abs(got - want).max() < 1e-6


def test_training_reduces_loss(ctx):
    import torch
    rng = np.random.default_rng(9)
    X = rng.uniform(-1, 1, size=(2048, 5)).astype(np.float32)
    y = (np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2] - 0.5 * X[:, 3] ** 2).astype(np.float32)
    Xd, yd = torch.tensor(X, device="cuda"), torch.tensor(y, device="cuda")
    net = gbd.Mlp(ctx, 5, 128, 3, 256, gbd.GBD_MLP_BF16)
    net.set_params(ref.init_params(ref.layer_shapes(5, 128, 3), seed=0).astype(np.float32))
    loss = torch.zeros(1, device="cuda")
    first = None
    for epoch in range(30):
        perm = torch.tensor(rng.permutation(2048).astype(np.int32), device="cuda")
        for s in range(0, 2048, 256):
            net.backward(Xd, yd, rows=perm[s:s + 256], loss_out=loss)
            net.adamw(2e-3)
            if first is None:
                torch.cuda.synchronize()
                first = float(loss.cpu())
    pred = np.concatenate([net.forward(Xd[s:s + 256]).cpu().numpy() for s in range(0, 2048, 256)])
    final = float(np.mean((pred - y) ** 2))
    print("training", first, final, flush=True)
    assert final < 0.05 * first


def test_train_call_equals_step_by_step(ctx):
    """gbd_mlp_train runs exactly backward then AdamW per step: parameters,
    optimiser state (through a further step) and the running loss sum equal
    the step-by-step calls bit for bit."""
    import torch
    rng = np.random.default_rng(4)
    X = rng.uniform(-1, 1, size=(1000, 5)).astype(np.float32)
    y = (np.cos(3 * X[:, 0]) * X[:, 4] + X[:, 1]).astype(np.float32)
    Xd, yd = torch.tensor(X, device="cuda"), torch.tensor(y, device="cuda")
    init = ref.init_params(ref.layer_shapes(5, 128, 3), seed=1).astype(np.float32)
    steps, batch = 7, 96
    rows = torch.tensor(rng.integers(0, 1000, size=(steps, batch)).astype(np.int32), device="cuda")
    lrs = [1e-3 * (1.0 + 0.1 * s) for s in range(steps)]
    a = gbd.Mlp(ctx, 5, 128, 3, 128, gbd.GBD_MLP_BF16)
    a.set_params(init)
    acc_a = torch.zeros(1, device="cuda")
    loss = torch.zeros(1, device="cuda")
    for s in range(steps):
        a.backward(Xd, yd, rows=rows[s], loss_out=loss)
        a.adamw(lrs[s], weight_decay=1e-4)
        acc_a += loss
    b = gbd.Mlp(ctx, 5, 128, 3, 128, gbd.GBD_MLP_BF16)
    b.set_params(init)
    acc_b = torch.zeros(1, device="cuda")
    b.train(Xd, yd, rows, lrs, weight_decay=1e-4, loss_sum=acc_b)
    assert np.array_equal(a.get_params(), b.get_params())
    assert np.array_equal(acc_a.cpu().numpy(), acc_b.cpu().numpy())
    # the moments and the step count carried on: one more identical step agrees
    for net in (a, b):
        net.backward(Xd, yd, rows=rows[0])
        net.adamw(5e-4)
    assert np.array_equal(a.get_params(), b.get_params())
    # refusals before any work: a bad rate, a batch beyond the handle's
    with pytest.raises(gbd.GbdError):
        b.train(Xd, yd, rows, [1e-3] * (steps - 1) + [-1.0])
    assert np.array_equal(a.get_params(), b.get_params())
    with pytest.raises(gbd.GbdError):
        b.train(Xd, yd, torch.zeros((1, 200), dtype=torch.int32, device="cuda"), [1e-3])

