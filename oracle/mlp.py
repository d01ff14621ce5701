"""FP64 reference of the loss-predictor network (test infrastructure only).

Network 16 -> 128 (ReLU) -> 128 (ReLU) -> 1 (logit), trained with the
positively weighted binary cross-entropy on logits and Adam (Kingma & Ba,
"Adam: a method for stochastic optimization", 2015).  Neither the paper nor
the build's workload description fixes more than the shape, BF16 operands
and FP32 accumulation; the rounding points below are this project's
reading and both the GPU kernels and this reference follow them:

* every GEMM operand (inputs X, activations H1 and H2, weights W1, W2, W3,
  back-propagated dZ1, dZ2, dz3) is rounded FP32 -> BF16 with round to
  nearest even on the bit pattern;
* products are accumulated exactly here (FP64) where the kernels accumulate
  in FP32;
* bias, ReLU, the sigmoid and the loss are evaluated in FP64 here and in FP32
  on the GPU.

Parameter vector layout (18,817 FP32): W1[16][128], b1[128], W2[128][128],
b2[128], w3[128], b3[1]; W[i][j] maps input i to output j.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 16, 128
SIZES = [("W1", (N_IN, N_H)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
         ("w3", (N_H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)
assert N_PARAMS == 18817


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SIZES])


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest even on the FP32 bit pattern) and return the
    value as FP64.  The value is first rounded to FP32 (the kernels hold it in
    FP32); NaN stays NaN."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    r = r.astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def standardise(x, norm) -> np.ndarray:
    """Network input from raw features: (x - mean) * inv_std with
    norm = [mean[16], inv_std[16]], evaluated in FP32 (two correctly rounded
    operations) as the kernels do, so that the BF16 rounding that follows
    sees the same value."""
    x = np.asarray(x, dtype=np.float32)
    nm = np.asarray(norm, dtype=np.float32)
    return ((x - nm[:N_IN]) * nm[N_IN:]).astype(np.float64)


def forward(theta, x, rounding: bool = True) -> dict:
    """Returns a dict of the intermediate values and the logits z3 [B]."""
    p = unpack(theta)
    r = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    X = r(x)
    z1 = X @ r(p["W1"]) + p["b1"]
    h1 = np.maximum(z1, 0.0)
    H1 = r(h1)
    z2 = H1 @ r(p["W2"]) + p["b2"]
    h2 = np.maximum(z2, 0.0)
    H2 = r(h2)
    z3 = H2 @ r(p["w3"]) + p["b3"][0]
    return {"X": X, "z1": z1, "H1": H1, "z2": z2, "H2": H2, "z3": z3}


def loss(z3, y, pos_weight: float) -> float:
    """Mean of -[w y log s(z) + (1 - y) log(1 - s(z))] with s the sigmoid,
    written with log1p(exp(-|z|)) so large |z| stays finite."""
    z3 = np.asarray(z3, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    sp_neg = np.maximum(-z3, 0) + np.log1p(np.exp(-np.abs(z3)))   # -log s(z)
    sp_pos = np.maximum(z3, 0) + np.log1p(np.exp(-np.abs(z3)))    # -log(1 - s(z))
    return float(np.mean(pos_weight * y * sp_neg + (1 - y) * sp_pos))


def backward(theta, x, y, pos_weight: float, rounding: bool = True) -> tuple[float, np.ndarray]:
    """Loss and its gradient with respect to the parameters.  The
    back-propagated signals dz3, dZ2, dZ1 are rounded to BF16 where they enter
    a GEMM (with ``rounding``)."""
    p = unpack(theta)
    r = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    f = forward(theta, x, rounding)
    y = np.asarray(y, dtype=np.float64)
    B = len(y)
    s = 1.0 / (1.0 + np.exp(-f["z3"]))
    dz3 = (s * (pos_weight * y + (1 - y)) - pos_weight * y) / B       # dL/dz3
    g = {}
    g["b3"] = np.array([dz3.sum()])
    g["w3"] = f["H2"].T @ r(dz3)
    dh2 = np.outer(r(dz3), r(p["w3"]))
    dZ2 = dh2 * (f["z2"] > 0)
    g["b2"] = dZ2.sum(axis=0)
    g["W2"] = f["H1"].T @ r(dZ2)
    dh1 = r(dZ2) @ r(p["W2"]).T
    dZ1 = dh1 * (f["z1"] > 0)
    g["b1"] = dZ1.sum(axis=0)
    g["W1"] = f["X"].T @ r(dZ1)
    return loss(f["z3"], y, pos_weight), pack(g)


def adam_step(theta, m, v, grad, step: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (step counts from 1): m <- b1 m + (1-b1) g,
    v <- b2 v + (1-b2) g^2, theta <- theta - lr mhat / (sqrt(vhat) + eps)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mhat = m / (1 - b1 ** step)
    vhat = v / (1 - b2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def he_init(seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)) from Philox-derived Gaussians,
    zero biases; weight j of the packed vector uses the oracle's deviate of
    (seed, particle id = j, turn 0, element 0)."""
    import oracle
    theta = np.zeros(N_PARAMS)
    o = 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        if name.startswith(("W", "w")):
            fan_in = shape[0]
            std = np.sqrt(2.0 / fan_in)
            theta[o:o + n] = [std * oracle.gauss_at(seed, o + k, 0, 0, 0) for k in range(n)]
        o += n
    return theta
