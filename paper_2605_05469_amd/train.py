"""Training of the learned warm start / preconditioner on the GPU.

The training set is made by the method itself: Landau-damping runs on a
128^3 grid with 8 particles per cell (perturbation amplitude alpha in
[0.01, 0.1], k in {0.5, 1.0}) advanced by this library's plain FP64 PIC step;
every step contributes its right-hand side b and solved potential phi.  In the
scale-free form the network maps r_hat = h^2 b / s (s = rms(h^2 b)) to the
correction e_hat = phi / s, so one network serves any grid spacing.  The
pairs are scaled (pic_net_make_pair), and every forward, backward, loss and
Adam update runs (pic_net_train_step, pic_net_loss), in the library's
kernels; torch only holds the device buffers.

    python -m paper_2605_05469_amd.train --out weights.npy
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def generate_pairs(net, N=128, ppc=8, alphas=None, ks=(0.5, 1.0), steps=100, seed=5000,
                   dt=0.05, rtol=1e-10, device="cuda", stride=1, diffs=True):
    """Run the plain solver and keep (r_hat, e_hat) FP32 pairs on the device,
    scaled by the library (pic_net_make_pair on the training network `net`).
    With `diffs`, the step-to-step changes (b_t - b_{t-1}, phi_t - phi_{t-1})
    are kept too: by linearity they are exact pairs as well, and they look like
    the residual corrections the preconditioner sees inside the solve."""
    import torch

    import paper_2605_05469_amd as P
    from paper_2605_05469_amd import synth

    if alphas is None:
        alphas = np.linspace(0.01, 0.1, 10)
    rhs, tgt = [], []
    run = 0
    for k in ks:
        for a in alphas:
            p = P.landau_params(N, ppc, k=k, dt=dt, rtol=rtol, check_every=32)
            ctx = P.Context(p)
            parts = synth.landau_particles_torch(N, ppc, k=k, alpha=float(a), seed=seed + run,
                                                 device=device)
            sim = P.Simulation(ctx, *parts)
            del parts
            sim.init()
            h = p.length / N
            prev = None
            for s in range(steps):
                info = sim.step()
                if s % stride:
                    continue
                r_t = torch.empty(N ** 3, dtype=torch.float32, device=device)
                t_t = torch.empty_like(r_t)
                net.make_pair(sim.rho, sim.phi, h, r_t, t_t)
                rhs.append(r_t)
                tgt.append(t_t)
                if diffs and prev is not None:
                    r_d = torch.empty_like(r_t)
                    t_d = torch.empty_like(r_t)
                    if net.make_pair(sim.rho, sim.phi, h, r_d, t_d, prev[0], prev[1]) > 0:
                        rhs.append(r_d)
                        tgt.append(t_d)
                prev = (sim.rho.clone(), sim.phi.clone()) if diffs else None
            log("run %d (k=%.2f alpha=%.3f): %d pairs, last solve %d iterations"
                % (run, k, a, len(rhs), info["iterations"]))
            run += 1
            del sim, ctx
    return rhs, tgt


def train(net, rhs, tgt, epochs=10, lr=1e-3, lam=1.0, seed=0, holdout=0.1, log_every=200,
          max_seconds=None, on_epoch=None):
    """Adam over shuffled pairs; returns (train losses, held-out losses).
    Stops early (after the current pair) once `max_seconds` have passed."""
    rng = np.random.default_rng(seed)
    n = len(rhs)
    idx = rng.permutation(n)
    nh = max(1, int(holdout * n))
    hold, tr = idx[:nh], idx[nh:]
    hist, hout = [], []
    step = 0
    total = epochs * len(tr)
    t0 = time.time()
    for ep in range(epochs):
        order = rng.permutation(tr)
        for i in order:
            frac = step / max(1, total)
            if max_seconds is not None:
                frac = min(1.0, max(frac, (time.time() - t0) / max_seconds))
            cur_lr = lr * (0.5 * (1 + math.cos(math.pi * frac)) * 0.9 + 0.1)
            want = (step % log_every) == 0
            L = net.train_step(rhs[i], tgt[i], lam=lam, lr=cur_lr, want_loss=want)
            if want:
                hist.append((step, L))
                log("step %d/%d  loss %.4e  lr %.2e  %.1f s" % (step, total, L, cur_lr,
                                                                 time.time() - t0))
            step += 1
            if max_seconds is not None and time.time() - t0 > max_seconds:
                break
        hout.append(evaluate(net, rhs, tgt, hold, lam))
        log("epoch %d: held-out loss %.4e  (%d steps, %.1f s)" % (ep, hout[-1], step,
                                                                 time.time() - t0))
        if on_epoch is not None:
            on_epoch(ep)
        if max_seconds is not None and time.time() - t0 > max_seconds:
            break
    return hist, hout


def evaluate(net, rhs, tgt, which, lam=1.0):
    """Mean loss over the given pairs without an update (pic_net_loss)."""
    tot = 0.0
    for i in which:
        tot += net.loss(rhs[i], tgt[i], lam=lam)
    return tot / max(1, len(which))


# (name, in channels, out channels) in the library's parameter order: for each
# layer the weights [cout][cin][3][3][3], then the biases [cout]
LAYERS = [("e1a", 1, 16), ("e1b", 16, 16), ("e2a", 16, 32), ("e2b", 32, 32),
          ("b3a", 32, 64), ("b3b", 64, 32), ("d2a", 32, 32), ("d2b", 32, 16),
          ("d1a", 16, 16), ("out", 16, 1)]


def init_params(seed=0):
    """He-normal weights, zero biases, canonical order (FP32 numpy).  The
    output layer starts at zero: the network's first output is 0 (loss 2), and
    its gradient reaches the hidden layers only after the first steps.  With a
    random output layer the first losses are O(10) (the A-term amplifies a
    random output by up to 12x) and Adam at batch size 1 drives every ReLU of a
    layer dead within a few hundred steps (the loss then stays at exactly 2)."""
    rng = np.random.default_rng(seed)
    chunks = []
    for name, ci, co in LAYERS:
        w = (rng.standard_normal(27 * ci * co) * math.sqrt(2.0 / (27 * ci))).astype(np.float32)
        if name == "out":
            w[:] = 0.0
        chunks.append(w)
        chunks.append(np.zeros(co, dtype=np.float32))
    return np.concatenate(chunks)


def main():
    ap = argparse.ArgumentParser(description="train the learned preconditioner")
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--ppc", type=int, default=8)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lam", type=float, default=1.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default="unet_landau.npy")
    ap.add_argument("--max-seconds", type=float, default=None,
                    help="stop training after this many seconds (weights saved every epoch)")
    ap.add_argument("--no-diffs", action="store_true",
                    help="do not add the step-to-step difference pairs")
    args = ap.parse_args()

    import torch

    import paper_2605_05469_amd as P

    torch.cuda.set_device(0)
    net = P.Net(args.grid, training=True)
    net.set_params(torch.from_numpy(init_params(args.seed)).cuda())
    t0 = time.time()
    rhs, tgt = generate_pairs(net, N=args.grid, ppc=args.ppc, steps=args.steps,
                              diffs=not args.no_diffs)
    log("generated %d pairs in %.1f s" % (len(rhs), time.time() - t0))
    params = torch.empty(P.unet_param_count(), dtype=torch.float32, device="cuda")

    def save(ep):
        net.get_params(params)
        np.save(args.out, params.cpu().numpy())
        log("saved %s after epoch %d" % (args.out, ep))

    t0 = time.time()
    hist, hout = train(net, rhs, tgt, epochs=args.epochs, lr=args.lr, lam=args.lam, seed=args.seed,
                       max_seconds=args.max_seconds, on_epoch=save)
    log("trained in %.1f s; held-out losses %s" % (time.time() - t0,
                                                   " ".join("%.3e" % v for v in hout)))


if __name__ == "__main__":
    main()
