"""FP64 NumPy oracle of the learned preconditioner's network -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  The learned warm start / preconditioner is not part of
the paper: it is this project's extension of the PCG solve of Sec. 3.2.  What
is computed here is the plain definition of each piece:

  conv3   y[o,p] = b[o] + sum_c sum_{d in {-1,0,1}^3} W[o,c,d] x[c,(p+d) mod n]
          (cross-correlation with periodic padding)
  pool    y[c,P] = (1/8) sum_{d in {0,1}^3} x[c,2P+d]     (2x2x2 average)
  up      y[c,2P+d] = x[c,P]                             (nearest, x2 per axis)
  relu    max(0, .)

and their adjoints.  BF16 storage of weights, activations and of the
gradients at each convolution's output is emulated by rounding FP64 -> FP32
-> BF16 (round-to-nearest-even at each step); all arithmetic is FP64 on the
rounded operands.  Array layout: [C, z, y, x].

Network: three levels with 16-32-64 channels, 3^3 periodic convolutions,
average pooling down and nearest up-sampling, additive skips:
  e1a = relu(conv3(x, 1->c1));       e1b = relu(conv3(e1a, c1->c1))   level 1
  p1  = pool(e1b)
  e2a = relu(conv3(p1, c1->c2));     e2b = relu(conv3(e2a, c2->c2))   level 2
  p2  = pool(e2b)
  b3a = relu(conv3(p2, c2->c3));     b3b = relu(conv3(b3a, c3->c2))   level 3
  u2  = up(b3b)
  d2a = relu(conv3(u2, c2->c2) + e2b); d2b = relu(conv3(d2a, c2->c1)) level 2
  u1  = up(d2b)
  d1a = relu(conv3(u1, c1->c1) + e1b)                                  level 1
  out = conv3(d1a, c1->1)                      (linear, not rounded to BF16)
"""
from __future__ import annotations

import numpy as np

# (name, cin, cout); every weighted layer is a 3^3 periodic convolution
_ARCH = [
    ("e1a", "1", "c1"),
    ("e1b", "c1", "c1"),
    ("e2a", "c1", "c2"),
    ("e2b", "c2", "c2"),
    ("b3a", "c2", "c3"),
    ("b3b", "c3", "c2"),
    ("d2a", "c2", "c2"),
    ("d2b", "c2", "c1"),
    ("d1a", "c1", "c1"),
    ("out", "c1", "1"),
]


def layer_specs(c1=16, c2=32, c3=64):
    ch = {"1": 1, "c1": c1, "c2": c2, "c3": c3}
    return [(n, ch[a], ch[b]) for (n, a, b) in _ARCH]


def weight_shape(cin, cout):
    return (cout, cin, 3, 3, 3)


def init_params(seed=0, c1=16, c2=32, c3=64):
    """He-normal weights, zero biases (FP64)."""
    rng = np.random.default_rng(seed)
    params = {}
    for name, cin, cout in layer_specs(c1, c2, c3):
        params[name + ".W"] = rng.standard_normal(weight_shape(cin, cout)) * np.sqrt(2.0 / (27 * cin))
        params[name + ".b"] = np.zeros(cout)
    return params


def flatten(params, specs):
    """Canonical flat order: for each layer, W [cout][cin][3][3][3] then b [cout]."""
    return np.concatenate([np.concatenate([params[n + ".W"].ravel(), params[n + ".b"].ravel()])
                           for (n, _, _) in specs])


def unflatten(flat, specs):
    params, o = {}, 0
    for name, cin, cout in specs:
        shp = weight_shape(cin, cout)
        k = int(np.prod(shp))
        params[name + ".W"] = np.asarray(flat[o:o + k], dtype=np.float64).reshape(shp)
        o += k
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


def pool_fwd(x):
    return _blocks(x).mean(axis=(1, 2, 3))


def pool_bwd(g):
    return up_fwd(g) / 8.0


def up_fwd(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def up_bwd(g):
    return _blocks(g).sum(axis=(1, 2, 3))


# ------------------------------------------------------------- network ---

def _ident(a):
    return np.asarray(a, dtype=np.float64)


def forward(params, x, specs, round_bf16=True):
    """x: [n, n, n] input.  Returns (out [n,n,n], activations)."""
    R = bf16 if round_bf16 else _ident
    A = {"in": R(np.asarray(x, dtype=np.float64)[None])}

    def conv(name, inp, skip=None, relu=True):
        y = conv3_fwd(inp, R(params[name + ".W"]), params[name + ".b"])
        if skip is not None:
            y = y + skip
        return R(np.maximum(y, 0.0)) if relu else y

    A["e1a"] = conv("e1a", A["in"])
    A["e1b"] = conv("e1b", A["e1a"])
    A["p1"] = R(pool_fwd(A["e1b"]))
    A["e2a"] = conv("e2a", A["p1"])
    A["e2b"] = conv("e2b", A["e2a"])
    A["p2"] = R(pool_fwd(A["e2b"]))
    A["b3a"] = conv("b3a", A["p2"])
    A["b3b"] = conv("b3b", A["b3a"])
    A["u2"] = up_fwd(A["b3b"])
    A["d2a"] = conv("d2a", A["u2"], skip=A["e2b"])
    A["d2b"] = conv("d2b", A["d2a"])
    A["u1"] = up_fwd(A["d2b"])
    A["d1a"] = conv("d1a", A["u1"], skip=A["e1b"])
    A["out"] = conv("out", A["d1a"], relu=False)
    return A["out"][0], A


def backward(params, A, dout, specs, round_bf16=True):
    """Gradients of sum(out * dout) w.r.t. every parameter and the input.
    Each convolution's output gradient (after the ReLU mask) is rounded to
    BF16, as the GPU stores it; all other gradients stay unrounded."""
    R = bf16 if round_bf16 else _ident
    grads = {}

    def back(name, g_pre, x_in):
        g_pre = R(g_pre)
        dW, db = conv3_bwd_weight(x_in, g_pre)
        grads[name + ".W"], grads[name + ".b"] = dW, db
        return conv3_bwd_data(g_pre, R(params[name + ".W"])), g_pre

    def mask(name):
        return A[name] > 0.0

    g, _ = back("out", np.asarray(dout, dtype=np.float64)[None], A["d1a"])
    g_u1, skip1 = back("d1a", g * mask("d1a"), A["u1"])
    g, _ = back("d2b", up_bwd(g_u1) * mask("d2b"), A["d2a"])
    g_u2, skip2 = back("d2a", g * mask("d2a"), A["u2"])
    g, _ = back("b3b", up_bwd(g_u2) * mask("b3b"), A["b3a"])
    g_p2, _ = back("b3a", g * mask("b3a"), A["p2"])
    g, _ = back("e2b", (pool_bwd(g_p2) + skip2) * mask("e2b"), A["e2a"])
    g_p1, _ = back("e2a", g * mask("e2a"), A["p1"])
    g, _ = back("e1b", (pool_bwd(g_p1) + skip1) * mask("e1b"), A["e1a"])
    g_in, _ = back("e1a", g * mask("e1a"), A["in"])
    return grads, g_in[0]


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
