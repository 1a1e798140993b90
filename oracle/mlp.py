"""numpy oracle of the learned warm-start MLP (test infrastructure only).

Network (per particle): five dimensionless features -> 64 -> 64 -> 1, ReLU.
Packed FP32 parameter vector (the layout the C ABI uses):

    W1[64][5], b1[64], W2[64][64], b2[64], w3[64], b3[1],
    in_shift[5], in_scale[5], out_scale[1]          (4620 floats)

Forward as the device computes it: x = bf16((f - in_shift) * in_scale);
z1 = x W1^T + b1 with bf16 operands and wide accumulation, h1 = bf16(relu(z1));
z2 = h1 W2^T + b2, h2 = bf16(relu(z2)); z = h2 . bf16(w3) + b3;
y = out_scale * z.  Biases stay FP32.  bf16 rounding is round-to-nearest-even
of the FP32 value.  Training minimises mean((z - t / out_scale)^2) with Adam
(Kingma and Ba 2015) on FP32 master parameters.
"""

from __future__ import annotations

import numpy as np

H = 64
NF = 5
SIZES = [("W1", (H, NF)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,)),
         ("in_shift", (NF,)), ("in_scale", (NF,)), ("out_scale", (1,))]
TRAINABLE = ("W1", "b1", "W2", "b2", "w3", "b3")
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)
N_TRAIN = sum(int(np.prod(s)) for n, s in SIZES if n in TRAINABLE)


def unpack(p: np.ndarray) -> dict:
    p = np.asarray(p, np.float64).reshape(-1)
    assert p.size == N_PARAMS, p.size
    out, o = {}, 0
    for n, s in SIZES:
        k = int(np.prod(s))
        out[n] = p[o:o + k].reshape(s)
        o += k
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[n], np.float64).reshape(-1) for n, _ in SIZES]).astype(np.float32)


def init(seed: int = 0, in_shift=None, in_scale=None, out_scale=1.0) -> np.ndarray:
    """He-uniform initial weights (seeded)."""
    rng = np.random.default_rng(seed)
    d = {
        "W1": rng.uniform(-1, 1, (H, NF)) * np.sqrt(6.0 / NF),
        "b1": np.zeros(H),
        "W2": rng.uniform(-1, 1, (H, H)) * np.sqrt(6.0 / H),
        "b2": np.zeros(H),
        "w3": rng.uniform(-1, 1, H) * np.sqrt(6.0 / H) * 0.1,
        "b3": np.zeros(1),
        "in_shift": np.zeros(NF) if in_shift is None else np.asarray(in_shift),
        "in_scale": np.ones(NF) if in_scale is None else np.asarray(in_scale),
        "out_scale": np.array([out_scale]),
    }
    return pack(d)


def bf16(a) -> np.ndarray:
    """Round FP32 values to bfloat16 (nearest, ties to even), returned as FP32."""
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    out = (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)
    return np.where(np.isnan(a), a, out)


def _f32(a):
    return np.asarray(a, np.float32)


def forward(p: np.ndarray, F: np.ndarray, emulate_bf16: bool = True, keep: bool = False):
    """y for features F[n, 5]; with emulate_bf16 the device's roundings are
    applied, sums are FP64 (wider than the device's FP32 accumulation)."""
    d = unpack(p)
    q = bf16 if emulate_bf16 else (lambda a: np.asarray(a, np.float64))
    F = np.asarray(F, np.float64)
    x = q(_f32((_f32(F) - _f32(d["in_shift"])) * _f32(d["in_scale"]))).astype(np.float64)
    if emulate_bf16:
        W1, W2, w3 = (bf16(_f32(d[k])).astype(np.float64) for k in ("W1", "W2", "w3"))
    else:
        W1, W2, w3 = (np.asarray(d[k], np.float64) for k in ("W1", "W2", "w3"))
    z1 = x @ W1.T + d["b1"]
    h1 = q(_f32(np.maximum(z1, 0.0)) if emulate_bf16 else np.maximum(z1, 0.0)).astype(np.float64)
    z2 = h1 @ W2.T + d["b2"]
    h2 = q(_f32(np.maximum(z2, 0.0)) if emulate_bf16 else np.maximum(z2, 0.0)).astype(np.float64)
    z = h2 @ w3 + d["b3"][0]
    y = z * d["out_scale"][0]
    if keep:
        return y, dict(x=x, z1=z1, h1=h1, z2=z2, h2=h2, z=z, W1=W1, W2=W2, w3=w3)
    return y


def error_scale(p: np.ndarray, F: np.ndarray) -> np.ndarray:
    """Per-sample bound scale of |y_device - y_oracle|: every bf16-rounded
    activation may land one bf16 step (2^-8 relative) away when its FP32
    pre-image sits within accumulation-order rounding of a rounding tie; the
    scale propagates such one-ulp changes to the output with absolute values."""
    d = unpack(p)
    y, c = forward(p, F, keep=True)
    aw1, aw2, aw3 = np.abs(c["W1"]), np.abs(c["W2"]), np.abs(c["w3"])
    s_x = 2.0 ** -8 * np.abs(c["x"])
    s_h1 = 2.0 ** -8 * np.abs(c["h1"]) + s_x @ aw1.T
    s_h2 = 2.0 ** -8 * np.abs(c["h2"]) + s_h1 @ aw2.T
    return np.abs(d["out_scale"][0]) * (s_h2 @ aw3 + 1e-6 * (np.abs(c["h2"]) @ aw3 + np.abs(d["b3"][0])))


def grad_scale(p: np.ndarray, F: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Scale of the device-vs-oracle gradient difference: the gradient
    formulas with every operand replaced by its absolute value, so that one
    bf16 step (2^-8 relative) in any rounded operand, or FP32 accumulation,
    moves an entry by a small multiple of this scale."""
    d = unpack(p)
    _, c = forward(p, F, keep=True)
    n = F.shape[0]
    r = c["z"] - np.asarray(t, np.float64) / d["out_scale"][0]
    adz = np.abs(2.0 * r / n)
    a2 = np.abs(np.outer(adz, c["w3"]))
    a1 = a2 @ np.abs(c["W2"])
    g = {k: np.zeros(s) for k, s in SIZES}
    g["b3"] = np.array([adz.sum()])
    g["w3"] = np.abs(c["h2"]).T @ adz
    g["b2"] = a2.sum(axis=0)
    g["W2"] = a2.T @ np.abs(c["h1"])
    g["b1"] = a1.sum(axis=0)
    g["W1"] = a1.T @ np.abs(c["x"])
    return np.concatenate([np.asarray(g[k], np.float64).reshape(-1) for k, _ in SIZES])


def loss_and_grads(p: np.ndarray, F: np.ndarray, t: np.ndarray, emulate_bf16: bool = True):
    """mean((z - t/out_scale)^2) and its gradient with respect to the
    trainable parameters (packed like the parameter vector, zeros for the
    fixed normalisation entries).  With emulate_bf16 the backward pass
    rounds the operands of its products to bf16 as the device does."""
    d = unpack(p)
    q = bf16 if emulate_bf16 else (lambda a: np.asarray(a, np.float64))
    _, c = forward(p, F, emulate_bf16=emulate_bf16, keep=True)
    n = F.shape[0]
    tt = np.asarray(t, np.float64) / d["out_scale"][0]
    r = c["z"] - tt
    loss = float(np.mean(r * r))
    dz = 2.0 * r / n                                           # [n]
    g = {}
    g["b3"] = np.array([dz.sum()])
    g["w3"] = c["h2"].T @ dz
    dz2 = q(_f32(np.outer(dz, c["w3"]) * (c["z2"] > 0))).astype(np.float64)    # [n, 64]
    g["b2"] = dz2.sum(axis=0)
    g["W2"] = dz2.T @ c["h1"]
    dz1 = q(_f32((dz2 @ c["W2"]) * (c["z1"] > 0))).astype(np.float64)          # [n, 64]
    g["b1"] = dz1.sum(axis=0)
    g["W1"] = dz1.T @ c["x"]
    full = {k: np.zeros(s) for k, s in SIZES}
    full.update(g)
    grad = np.concatenate([np.asarray(full[k], np.float64).reshape(-1) for k, _ in SIZES])
    return loss, grad


def adam(p: np.ndarray, grad: np.ndarray, m: np.ndarray, v: np.ndarray, step: int, lr: float,
         beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of the trainable entries (step counts from 1)."""
    d = unpack(p)
    p = np.asarray(p, np.float64).copy()
    mask = np.concatenate([np.full(int(np.prod(s)), n in TRAINABLE) for n, s in SIZES])
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    upd = lr * mh / (np.sqrt(vh) + eps)
    p[mask] -= upd[mask]
    del d
    return p, m, v


def input_jacobian(p: np.ndarray, F: np.ndarray) -> np.ndarray:
    """dy/dF [n, 5] of the un-rounded network (ReLU masks of the emulated
    forward), for propagating feature error scales to the prediction."""
    d = unpack(p)
    _, c = forward(p, F, keep=True)
    m1 = (c["z1"] > 0).astype(np.float64)
    m2 = (c["z2"] > 0).astype(np.float64)
    g2 = m2 * d["w3"]                          # [n, 64]
    g1 = (g2 @ d["W2"]) * m1                   # [n, 64]
    gx = g1 @ d["W1"]                          # [n, 5]
    return d["out_scale"][0] * gx * d["in_scale"]


def step_callback(p: np.ndarray, rel: float = 1e-5):
    """MLP callback for the oracle step: the emulated prediction and its
    error scale in the units of the step's S fields (tolerance rel x S):
    the bf16 bound divided by rel plus the feature scales pushed through the
    input Jacobian."""
    def cb(F, SF):
        y = forward(p, F)
        s = error_scale(p, F) / rel + np.abs(input_jacobian(p, F) * SF).sum(axis=1)
        return y, s
    return cb
