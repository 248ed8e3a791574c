"""GPU MLP (BF16 matrix cores, FP32 accumulation) against the FP64 oracle.

The oracle runs on the BF16-rounded parameters and inputs the GPU uses; the
GPU also rounds hidden activations to BF16, so agreement is at BF16 level:
relative Frobenius error per tensor <= 1e-2.
"""

import numpy as np
import pytest
import torch

from oracle import mlp as om

pytestmark = pytest.mark.gpu


def rel_fro(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def setup(gpu, B=200, seed=0):
    r = np.random.default_rng(seed)
    theta = om.init_params(seed + 1)
    X = r.uniform(0, 1, (B, 64)).astype(np.float32)
    T = r.standard_normal((B, 3)).astype(np.float32)
    net = gpu.Mlp(seed=3, max_batch=256)
    net.set_params(theta)
    th_b = om.bf16_round(theta.astype(np.float32))
    # biases are applied in FP32 on the GPU: keep them unrounded in the oracle
    layers = om.unpack(th_b)
    layers_f = om.unpack(theta.astype(np.float32).astype(np.float64))
    th_mix = om.pack([(W, bf) for (W, _), (_, bf) in zip(layers, layers_f)])
    return net, theta, th_mix, X, T


def test_forward_matches_oracle(gpu):
    print("case: mlp forward", flush=True)
    net, theta, th_mix, X, T = setup(gpu)
    Y = net.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    Yo, _ = om.forward(th_mix, om.bf16_round(X), round_hidden=True)
    e = rel_fro(Y, Yo)
    print("forward rel err %.3e" % e, flush=True)
    assert e < 1e-2


def test_gradients_match_oracle(gpu):
    print("case: mlp gradients", flush=True)
    net, theta, th_mix, X, T = setup(gpu, B=256)
    g, loss = net.gradient(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    go, lo = om.backward(th_mix, om.bf16_round(X), T.astype(np.float64), round_hidden=True)
    assert abs(loss - lo) <= 1e-2 * lo
    gl = om.unpack(g.astype(np.float64))
    ol = om.unpack(go)
    for li, ((Wg, bg), (Wo, bo)) in enumerate(zip(gl, ol)):
        ew, eb = rel_fro(Wg, Wo), rel_fro(bg, bo)
        print("layer %d: dW rel %.3e  db rel %.3e" % (li, ew, eb), flush=True)
        assert ew < 1e-2 and eb < 1e-2


def test_adam_step_and_resume(gpu):
    print("case: mlp adam + resume", flush=True)
    net, theta, th_mix, X, T = setup(gpu, B=128)
    x, t = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    g, _ = net.gradient(x, t)
    net.adam_step(1e-3)
    p1 = net.get_params().astype(np.float64)
    ref, _, _ = om.adam_step(theta.astype(np.float32).astype(np.float64), g.astype(np.float64),
                             np.zeros_like(p1), np.zeros_like(p1), 1, lr=1e-3)
    np.testing.assert_allclose(p1, ref, rtol=1e-5, atol=1e-7)
    # checkpoint, run 3 steps, restore, run the same 3 steps: bit-equal parameters
    st = net.get_state()
    for _ in range(3):
        net.train_step(x, t, 1e-3)
    a = net.get_params()
    net.set_state(st)
    for _ in range(3):
        net.train_step(x, t, 1e-3)
    b = net.get_params()
    assert np.array_equal(a, b)


def test_training_lowers_loss(gpu):
    print("case: mlp training", flush=True)
    r = np.random.default_rng(7)
    X = r.uniform(0, 1, (4096, 64)).astype(np.float32)
    W = r.standard_normal((64, 3)) / 8
    T = np.tanh(X @ W).astype(np.float32)
    net = gpu.Mlp(seed=1, max_batch=1024)
    x, t = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    _, l0 = net.gradient(x[:1024], t[:1024])
    for ep in range(30):
        for i in range(4):
            net.train_step(x[i * 1024:(i + 1) * 1024], t[i * 1024:(i + 1) * 1024], 1e-3)
    _, l1 = net.gradient(x[:1024], t[:1024])
    print("loss %.4e -> %.4e" % (l0, l1), flush=True)
    assert l1 < 0.1 * l0


def test_inference_rows_are_independent(gpu):
    """ddm_mlp_forward (one launch, 64 rows per workgroup): every row's output
    is the same bits whatever the call's row count (1, 63, 64, 65, 1000 and
    70,000 rows: partial and whole tiles, more rows than max_batch), and 1000
    rows agree with the oracle at BF16 level."""
    print("case: mlp inference row counts", flush=True)
    net, theta, th_mix, X, T = setup(gpu, B=1000, seed=4)
    r = np.random.default_rng(9)
    Xl = torch.from_numpy(r.uniform(0, 1, (70_000, 64)).astype(np.float32)).cuda()
    Xl[:1000] = torch.from_numpy(X).cuda()
    Yl = net.forward(Xl)
    for rows in (1, 63, 64, 65, 1000):
        Y = net.forward(Xl[:rows].contiguous())
        torch.cuda.synchronize()
        assert torch.equal(Y, Yl[:rows]), rows
    Yo, _ = om.forward(th_mix, om.bf16_round(X), round_hidden=True)
    e = rel_fro(Yl[:1000].cpu().numpy(), Yo)
    print("forward rel err %.3e" % e, flush=True)
    assert e < 1e-2
