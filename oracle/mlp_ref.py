"""FP64 reference of the sphericity-correction network -- TEST INFRASTRUCTURE.

Plain numpy forward and backward of the 34 -> 64 -> 64 -> 64 -> 1 SiLU network
used by the learned correction (not a method of the paper; its inputs are the
paper's local-thickness measures).  With ``bf16=True`` the operands of every
matrix product are rounded to bfloat16 (round to nearest even) at the same points
as the device kernels -- standardised inputs, weights, hidden activations and the
back-propagated gradients entering a product -- while all arithmetic stays FP64.
With ``bf16=False`` it is the exact FP64 network, which the tests pin against
central finite differences.

Parameters use the device's packed layout: W1[64][48] b1[64] W2[64][64] b2[64]
W3[64][64] b3[64] W4[16][64] b4[16] (inputs 34..47, rows 1..15 of W4 and entries
1..15 of b4 are unused and zero).
"""
from __future__ import annotations

import numpy as np

IN, INP, H, OUTP = 34, 48, 64, 16
OFF = {}
_o = 0
for _name, _n in (("W1", H * INP), ("b1", H), ("W2", H * H), ("b2", H), ("W3", H * H), ("b3", H),
                  ("W4", OUTP * H), ("b4", OUTP)):
    OFF[_name] = (_o, _n)
    _o += _n
N_PARAM = _o


def unpack(p: np.ndarray) -> dict:
    d = {k: np.asarray(p[o:o + n], dtype=np.float64) for k, (o, n) in OFF.items()}
    d["W1"] = d["W1"].reshape(H, INP)
    d["W2"] = d["W2"].reshape(H, H)
    d["W3"] = d["W3"].reshape(H, H)
    d["W4"] = d["W4"].reshape(OUTP, H)
    return d


def pack(d: dict) -> np.ndarray:
    out = np.zeros(N_PARAM)
    for k, (o, n) in OFF.items():
        out[o:o + n] = np.asarray(d[k]).ravel()
    return out


def bf16(x):
    """Round float32-representable values to bfloat16, nearest even (as FP64)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def _r(x, on):
    return bf16(x) if on else np.asarray(x, dtype=np.float64)


def forward(p: np.ndarray, x: np.ndarray, mean, inv_std, bf16_ops: bool = True):
    """x: (B, 34) raw features.  Returns (prediction (B,), cache)."""
    w = unpack(p)
    B = x.shape[0]
    xs = np.zeros((B, INP))
    xs[:, :IN] = (np.asarray(x, np.float64) - np.asarray(mean, np.float64)) * np.asarray(inv_std, np.float64)
    xs[~np.isfinite(xs)] = 0.0
    a0 = _r(xs, bf16_ops)
    z1 = a0 @ _r(w["W1"], bf16_ops).T + w["b1"]
    a1 = _r(silu(z1), bf16_ops)
    z2 = a1 @ _r(w["W2"], bf16_ops).T + w["b2"]
    a2 = _r(silu(z2), bf16_ops)
    z3 = a2 @ _r(w["W3"], bf16_ops).T + w["b3"]
    a3 = _r(silu(z3), bf16_ops)
    pred = a3 @ _r(w["W4"], bf16_ops)[0] + w["b4"][0]
    return pred, dict(a0=a0, z1=z1, a1=a1, z2=z2, a2=a2, z3=z3, a3=a3, w=w)


def loss(p, x, y, mean, inv_std, bf16_ops=False):
    pred, _ = forward(p, x, mean, inv_std, bf16_ops)
    return float(np.mean((pred - y) ** 2))


def backward(p: np.ndarray, x, y, mean, inv_std, bf16_ops: bool = True) -> np.ndarray:
    """Gradient of the mean squared error, packed like the parameters."""
    pred, c = forward(p, x, mean, inv_std, bf16_ops)
    w = c["w"]
    B = x.shape[0]
    d = 2.0 * (pred - np.asarray(y, np.float64)) / B            # dL/dpred
    g = {k: np.zeros_like(v) for k, v in w.items()}
    g["b4"][0] = d.sum()
    db = _r(d, bf16_ops)
    g["W4"][0] = db @ c["a3"]
    dh3 = np.outer(db, _r(w["W4"], bf16_ops)[0])
    dz3 = dh3 * dsilu(c["z3"])
    g["b3"] = dz3.sum(axis=0)
    dz3r = _r(dz3, bf16_ops)
    g["W3"] = dz3r.T @ c["a2"]
    dh2 = dz3r @ _r(w["W3"], bf16_ops)
    dz2 = dh2 * dsilu(c["z2"])
    g["b2"] = dz2.sum(axis=0)
    dz2r = _r(dz2, bf16_ops)
    g["W2"] = dz2r.T @ c["a1"]
    dh1 = dz2r @ _r(w["W2"], bf16_ops)
    dz1 = dh1 * dsilu(c["z1"])
    g["b1"] = dz1.sum(axis=0)
    g["W1"] = _r(dz1, bf16_ops).T @ c["a0"]
    return pack(g)
