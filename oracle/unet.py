"""FP64 NumPy oracle of the learned preconditioner's network -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  The learned warm start / preconditioner is not part of
the paper: it is this project's extension of the PCG solve of Sec. 3.2.  What
is computed here is the plain definition of each layer:

  conv3   y[o,p] = b[o] + sum_c sum_{d in {-1,0,1}^3} W[o,c,d] x[c,(p+d) mod n]
          (cross-correlation with periodic padding)
  down    y[o,P] = b[o] + sum_c sum_{d in {0,1}^3} W[o,c,d] x[c,2P+d]
          (2x2x2 stride-2 convolution)
  up      y[o,2P+d] = b[o] + sum_c W[c,o,d] x[c,P]
          (2x2x2 stride-2 transposed convolution; W stored [in, out, ...])
  relu    max(0, .)

and their adjoints (backward data / backward weight).  BF16 storage of
weights and activations is emulated by rounding FP64 -> FP32 -> BF16
(round-to-nearest-even at each step); all arithmetic is FP64 on the rounded
operands.  Array layout: [C, z, y, x].

Network (three levels, 16-32-64 channels, 3^3 kernels, periodic padding):
  e1a = relu(conv3(x, 1->c1));  e1b = relu(conv3(e1a, c1->c1))       level 1
  d1  = relu(down(e1b, c1->c2)); e2a = relu(conv3(d1, c2->c2))        level 2
  d2  = relu(down(e2a, c2->c3)); b3a = relu(conv3(d2, c3->c3));
  b3b = relu(conv3(b3a, c3->c3))                                      level 3
  u2  = relu(up(b3b, c3->c2) + e2a); e2c = relu(conv3(u2, c2->c2))    level 2
  u1  = relu(up(e2c, c2->c1) + e1b); e1c = relu(conv3(u1, c1->c1))    level 1
  out = conv3(e1c, c1->1)                      (linear, not rounded to BF16)
"""
from __future__ import annotations

import numpy as np

# (name, kind, cin, cout) with channel symbols resolved by layer_specs()
_ARCH = [
    ("e1a", "conv3", "1", "c1"),
    ("e1b", "conv3", "c1", "c1"),
    ("d1", "down", "c1", "c2"),
    ("e2a", "conv3", "c2", "c2"),
    ("d2", "down", "c2", "c3"),
    ("b3a", "conv3", "c3", "c3"),
    ("b3b", "conv3", "c3", "c3"),
    ("u2", "up", "c3", "c2"),
    ("e2c", "conv3", "c2", "c2"),
    ("u1", "up", "c2", "c1"),
    ("e1c", "conv3", "c1", "c1"),
    ("out", "conv3", "c1", "1"),
]


def layer_specs(c1=16, c2=32, c3=64):
    ch = {"1": 1, "c1": c1, "c2": c2, "c3": c3}
    return [(n, k, ch[a], ch[b]) for (n, k, a, b) in _ARCH]


def weight_shape(kind, cin, cout):
    if kind == "conv3":
        return (cout, cin, 3, 3, 3)
    if kind == "down":
        return (cout, cin, 2, 2, 2)
    return (cin, cout, 2, 2, 2)  # up


def init_params(seed=0, c1=16, c2=32, c3=64):
    """He-normal weights, zero biases (FP64)."""
    rng = np.random.default_rng(seed)
    params = {}
    for name, kind, cin, cout in layer_specs(c1, c2, c3):
        shp = weight_shape(kind, cin, cout)
        fan_in = cin * (27 if kind == "conv3" else 8 if kind == "down" else 1)
        params[name + ".W"] = rng.standard_normal(shp) * np.sqrt(2.0 / fan_in)
        params[name + ".b"] = np.zeros(cout)
    return params


def flatten(params, specs):
    """Canonical flat order: for each layer, W (shape of weight_shape) then b."""
    return np.concatenate([np.concatenate([params[n + ".W"].ravel(), params[n + ".b"].ravel()])
                           for (n, _, _, _) in specs])


def unflatten(flat, specs):
    params, o = {}, 0
    for name, kind, cin, cout in specs:
        shp = weight_shape(kind, cin, cout)
        n = int(np.prod(shp))
        params[name + ".W"] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shp)
        o += n
        params[name + ".b"] = np.asarray(flat[o:o + cout], dtype=np.float64)
        o += cout
    return params


# ------------------------------------------------------------ rounding ---

def bf16(a):
    """Round to the nearest BF16 value (FP64 -> FP32 -> BF16, RNE)."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# -------------------------------------------------------------- layers ---

def _shift(x, d):
    """s[c, p] = x[c, (p + d) mod n] for d = (dz, dy, dx)."""
    return np.roll(x, shift=(-d[0], -d[1], -d[2]), axis=(1, 2, 3))


def _offsets3():
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                yield dz, dy, dx


def conv3_fwd(x, W, b):
    y = np.zeros((W.shape[0],) + x.shape[1:])
    for d in _offsets3():
        y += np.tensordot(W[:, :, d[0] + 1, d[1] + 1, d[2] + 1], _shift(x, d), axes=(1, 0))
    return y + b[:, None, None, None]


def conv3_bwd_data(dy, W):
    dx = np.zeros((W.shape[1],) + dy.shape[1:])
    for d in _offsets3():
        dx += np.tensordot(W[:, :, d[0] + 1, d[1] + 1, d[2] + 1], _shift(dy, (-d[0], -d[1], -d[2])),
                           axes=(0, 0))
    return dx


def conv3_bwd_weight(x, dy):
    dW = np.zeros((dy.shape[0], x.shape[0], 3, 3, 3))
    for d in _offsets3():
        dW[:, :, d[0] + 1, d[1] + 1, d[2] + 1] = np.tensordot(dy, _shift(x, d),
                                                              axes=([1, 2, 3], [1, 2, 3]))
    return dW, dy.sum(axis=(1, 2, 3))


def _blocks(x):
    """x[c, 2Z+a, 2Y+b, 2X+e] -> B[c, a, b, e, Z, Y, X]."""
    C, n = x.shape[0], x.shape[1]
    m = n // 2
    return x.reshape(C, m, 2, m, 2, m, 2).transpose(0, 2, 4, 6, 1, 3, 5)


def _unblocks(B):
    C, m = B.shape[0], B.shape[4]
    return B.transpose(0, 4, 1, 5, 2, 6, 3).reshape(C, 2 * m, 2 * m, 2 * m)


def down_fwd(x, W, b):
    return np.tensordot(W, _blocks(x), axes=([1, 2, 3, 4], [0, 1, 2, 3])) + b[:, None, None, None]


def down_bwd_data(dy, W):
    return _unblocks(np.tensordot(W, dy, axes=(0, 0)))


def down_bwd_weight(x, dy):
    dW = np.tensordot(dy, _blocks(x), axes=([1, 2, 3], [4, 5, 6]))
    return dW, dy.sum(axis=(1, 2, 3))


def up_fwd(x, W, b):
    # W[c, o, a, b, e]: Y[o, a, b, e, P] = sum_c W[c,o,a,b,e] x[c,P]
    return _unblocks(np.tensordot(W, x, axes=(0, 0))) + b[:, None, None, None]


def up_bwd_data(dy, W):
    return np.tensordot(W, _blocks(dy), axes=([1, 2, 3, 4], [0, 1, 2, 3]))


def up_bwd_weight(x, dy):
    dW = np.tensordot(x, _blocks(dy), axes=([1, 2, 3], [4, 5, 6]))
    return dW, dy.sum(axis=(1, 2, 3))


_FWD = {"conv3": conv3_fwd, "down": down_fwd, "up": up_fwd}
_BWD_DATA = {"conv3": conv3_bwd_data, "down": down_bwd_data, "up": up_bwd_data}
_BWD_W = {"conv3": conv3_bwd_weight, "down": down_bwd_weight, "up": up_bwd_weight}

_SKIP = {"u2": "e2a", "u1": "e1b"}


# ------------------------------------------------------------- network ---

def forward(params, x, specs, round_bf16=True):
    """x: [n, n, n] input.  Returns (out [n,n,n], cache of layer inputs/outputs)."""
    rnd = bf16 if round_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    a = rnd(np.asarray(x, dtype=np.float64)[None])
    acts = {"in": a}
    cur = a
    for name, kind, cin, cout in specs:
        W = rnd(params[name + ".W"])
        y = _FWD[kind](cur, W, params[name + ".b"])
        if name in _SKIP:
            y = y + acts[_SKIP[name]]
        if name == "out":
            acts[name] = y
            cur = y
            break
        y = rnd(np.maximum(y, 0.0))
        acts[name] = y
        cur = y
    return cur[0], acts


def backward(params, acts, dout, specs, round_bf16=True):
    """Gradients of sum(out * dout) w.r.t. every parameter (and the input).
    Gradients flowing between layers are rounded to BF16 like activations."""
    rnd = bf16 if round_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    names = [s[0] for s in specs]
    inputs = {}
    prev = "in"
    for name in names:
        inputs[name] = prev
        prev = name
    grads = {}
    g_act = {n: None for n in names}
    g_act["in"] = None
    g = rnd(np.asarray(dout, dtype=np.float64)[None])
    for idx in range(len(specs) - 1, -1, -1):
        name, kind, cin, cout = specs[idx]
        if name != "out":
            g = g if g_act[name] is None else g_act[name]
            g = rnd(g * (acts[name] > 0.0))
        if name in _SKIP:
            s = _SKIP[name]
            g_act[s] = g if g_act[s] is None else g_act[s] + g
        W = rnd(params[name + ".W"])
        x_in = acts[inputs[name]]
        dW, db = _BWD_W[kind](x_in, g)
        grads[name + ".W"], grads[name + ".b"] = dW, db
        gx = _BWD_DATA[kind](g, W)
        src = inputs[name]
        g_act[src] = gx if g_act[src] is None else g_act[src] + gx
        g = g_act[src]
    return grads, g_act["in"][0]


# --------------------------------------------------------- loss, Adam ---

def apply_A1(u):
    """Unit-spacing periodic 7-point operator -Lap_1 on [n,n,n]."""
    return (6.0 * u - sum(np.roll(u, s, axis=a) for a in (0, 1, 2) for s in (1, -1)))


def loss(out, target, rhs, lam=1.0):
    """L = ||o - t||^2/||t||^2 + lam ||A1 o - r||^2/||r||^2 and dL/do."""
    d1 = out - target
    d2 = apply_A1(out) - rhs
    nt, nr = np.sum(target * target), np.sum(rhs * rhs)
    L = np.sum(d1 * d1) / nt + lam * np.sum(d2 * d2) / nr
    g = 2.0 * d1 / nt + 2.0 * lam * apply_A1(d2) / nr
    return L, g


def adam(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma & Ba, 2015), bias-corrected; returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def precondition(params, r, h, specs, round_bf16=True):
    """z = s * NN(h^2 r / s) with s = rms(h^2 r), mean removed (FP64)."""
    n = round(len(r) ** (1 / 3))
    rh = (h * h) * np.asarray(r, dtype=np.float64)
    s = np.sqrt(np.mean(rh * rh))
    if s == 0.0:
        return np.zeros_like(rh)
    o, _ = forward(params, (rh / s).reshape(n, n, n), specs, round_bf16)
    z = s * o.ravel()
    return z - z.mean()
