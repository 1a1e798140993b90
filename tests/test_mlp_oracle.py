"""Pins of the numpy MLP oracle: finite differences, torch reference forward,
bf16 rounding against torch's conversion, Adam's first step in closed form."""

import numpy as np
import torch

from oracle import mlp


def _data(n=64, seed=0):
    rng = np.random.default_rng(seed)
    F = rng.normal(0, 1, (n, 5)) * np.array([1e-2, 1e-2, 0.2, 1e-2, 0.3]) + np.array([0, 0, 1, 0, 1])
    t = rng.normal(0, 1e-2, n)
    p = mlp.init(seed=3, in_shift=F.mean(0), in_scale=1 / F.std(0), out_scale=1e-2)
    return p, F, t


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    a = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-3, 5000), [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9, -2.5]])
    a = a.astype(np.float32)
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(mlp.bf16(a), ref)
    assert mlp.bf16(np.float32(1 + 2 ** -8)) == 1.0          # tie to even
    assert mlp.bf16(np.float32(1 + 3 * 2 ** -9)) == 1 + 2 ** -7


def test_forward_matches_torch_fp64():
    p, F, _ = _data()
    d = mlp.unpack(p)
    x = torch.from_numpy(((F.astype(np.float32) - d["in_shift"].astype(np.float32)) *
                          d["in_scale"].astype(np.float32)).astype(np.float64))
    h = torch.relu(torch.nn.functional.linear(x, torch.from_numpy(d["W1"]), torch.from_numpy(d["b1"])))
    h = torch.relu(torch.nn.functional.linear(h, torch.from_numpy(d["W2"]), torch.from_numpy(d["b2"])))
    z = torch.nn.functional.linear(h, torch.from_numpy(d["w3"][None]), torch.from_numpy(d["b3"]))[:, 0]
    y_ref = (z * d["out_scale"][0]).numpy()
    y = mlp.forward(p, F, emulate_bf16=False)
    np.testing.assert_allclose(y, y_ref, rtol=1e-12, atol=1e-15)


def test_backward_matches_finite_differences():
    p, F, t = _data()
    loss, g = mlp.loss_and_grads(p, F, t, emulate_bf16=False)
    p64 = p.astype(np.float64)
    d = mlp.unpack(p64)
    rng = np.random.default_rng(2)
    idx_all = np.arange(mlp.N_PARAMS)
    trainable = np.concatenate([np.full(int(np.prod(s)), n in mlp.TRAINABLE) for n, s in mlp.SIZES])
    for i in rng.choice(idx_all[trainable], 60, replace=False):
        h = 1e-6 * max(1.0, abs(p64[i]))

        def L(q):
            dd = mlp.unpack(q)
            z = mlp.forward(q, F, emulate_bf16=False) / dd["out_scale"][0]
            return np.mean((z - t / dd["out_scale"][0]) ** 2)
        qp, qm = p64.copy(), p64.copy()
        qp[i] += h
        qm[i] -= h
        fd = (L(qp) - L(qm)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g).max(), 1e-12), (i, fd, g[i])
    del d, loss


def test_adam_first_step_closed_form():
    p, F, t = _data()
    _, g = mlp.loss_and_grads(p, F, t)
    m = np.zeros_like(g)
    v = np.zeros_like(g)
    lr = 1e-3
    p1, m1, v1 = mlp.adam(p, g, m, v, 1, lr)
    trainable = np.concatenate([np.full(int(np.prod(s)), n in mlp.TRAINABLE) for n, s in mlp.SIZES])
    expect = p.astype(np.float64) - np.where(trainable, lr * g / (np.abs(g) + 1e-8), 0.0)
    np.testing.assert_allclose(p1, expect, rtol=0, atol=1e-15)
    np.testing.assert_allclose(m1, 0.1 * g)
    np.testing.assert_allclose(v1, 0.001 * g * g)


def test_training_reduces_loss():
    rng = np.random.default_rng(4)
    F = rng.normal(0, 1, (2048, 5))
    t = 1e-2 * np.tanh(F[:, 0] - 0.5 * F[:, 3])
    p = mlp.init(seed=5, in_shift=np.zeros(5), in_scale=np.ones(5), out_scale=1e-2)
    m = np.zeros(mlp.N_PARAMS)
    v = np.zeros(mlp.N_PARAMS)
    l0, _ = mlp.loss_and_grads(p, F, t)
    for s in range(1, 201):
        b = rng.choice(2048, 256, replace=False)
        _, g = mlp.loss_and_grads(p, F[b], t[b])
        p, m, v = mlp.adam(p, g, m, v, s, 3e-3)
        p = p.astype(np.float32)
    l1, _ = mlp.loss_and_grads(p, F, t)
    assert l1 < 0.2 * l0, (l0, l1)
