"""Seeded synthetic inputs: the Landau-damping initial state.

This module holds the input generator only -- none of the method's arithmetic
(no deposit, solve, gather or push).  Both the HIP path's callers and the
oracle's callers draw their inputs from here, so both start from the same
bits.

Initial state (Sec. 2.1, "Landau Damping"): on the periodic cube [0, L)^3 with
L = 2*pi/k, the electron distribution is a Maxwellian in v times
prod_d (1 + alpha*cos(k x_d)).  The density factorises over the axes, so each
coordinate is drawn independently by inverting its CDF
    F(x) = (x + (alpha/k) sin(k x)) / L
with Newton's method (F' > 0 for alpha < 1), and each velocity component is
N(0, 1).  Units: eps0 = 1, q/m = -1, mean electron density 1, so the total
electron charge is Q_e = -L^3, each macro-particle carries q = Q_e/Np and the
neutralising background is rho_bg = -Q_e/L^3 = +1 (Sec. 2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def box_length(k: float = 0.5) -> float:
    return 2.0 * math.pi / k


def normal_field(n: int, seed: int) -> np.ndarray:
    """n independent N(0, 1) values (FP64) from PCG64(seed): a generic
    right-hand side for solves on boxes without particles."""
    return np.random.Generator(np.random.PCG64(seed)).standard_normal(n)


@dataclass
class LandauParams:
    N: int = 32
    ppc: int = 8
    k: float = 0.5
    alpha: float = 0.05
    dt: float = 0.05
    qm: float = -1.0
    seed: int = 20260

    @property
    def L(self) -> float:
        return box_length(self.k)

    @property
    def np_total(self) -> int:
        return self.ppc * self.N ** 3

    @property
    def q(self) -> float:
        return -(self.L ** 3) / self.np_total

    @property
    def rho_bg(self) -> float:
        return -(self.q * self.np_total) / self.L ** 3


def _invert_cdf_np(u: np.ndarray, k: float, alpha: float, L: float) -> np.ndarray:
    """Solve (x + (alpha/k) sin(kx)) = u*L for x in [0, L) by Newton."""
    target = u * L
    x = target.copy()
    a_k = alpha / k
    for _ in range(50):
        f = x + a_k * np.sin(k * x) - target
        dx = f / (1.0 + alpha * np.cos(k * x))
        x -= dx
        if np.max(np.abs(dx), initial=0.0) <= 1e-14 * L:
            break
    x = np.where(x >= L, x - L, x)
    x = np.where(x < 0.0, x + L, x)
    return np.where(x >= L, 0.0, x)


def landau_particles_np(N: int, ppc: int, k: float = 0.5, alpha: float = 0.05,
                        seed: int = 20260, np_total: int | None = None):
    """(x, y, z, vx, vy, vz) FP64 NumPy arrays, PCG64-seeded (host)."""
    L = box_length(k)
    n = ppc * N ** 3 if np_total is None else int(np_total)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    pos = [_invert_cdf_np(rng.random(n), k, alpha, L) for _ in range(3)]
    vel = [rng.standard_normal(n) for _ in range(3)]
    return (*pos, *vel)


def landau_particles_torch(N: int, ppc: int, k: float = 0.5, alpha: float = 0.05,
                           seed: int = 20262, device="cuda", np_total: int | None = None,
                           chunk: int = 1 << 26, out=None):
    """Same recipe drawn by torch's seeded generator on ``device``.

    For the 2^30-particle workloads a host draw would take minutes, so these
    inputs are drawn on the device in chunks (torch's Philox stream; the bits
    differ from the NumPy variant, the distribution is the same).  ``out`` may
    hold six preallocated FP64 device tensors.
    """
    import torch

    L = box_length(k)
    n = ppc * N ** 3 if np_total is None else int(np_total)
    if out is None:
        out = [torch.empty(n, dtype=torch.float64, device=device) for _ in range(6)]
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    a_k = alpha / k
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        for d in range(3):
            u = torch.rand(e - s, dtype=torch.float64, device=device, generator=g)
            t = u * L
            x = t.clone()
            for _ in range(50):
                dx = (x + a_k * torch.sin(k * x) - t) / (1.0 + alpha * torch.cos(k * x))
                x -= dx
                if float(dx.abs().max()) <= 1e-14 * L:
                    break
            x = torch.where(x >= L, x - L, x)
            x = torch.where(x < 0.0, x + L, x)
            x = torch.where(x >= L, torch.zeros_like(x), x)
            out[d][s:e].copy_(x)
        for d in range(3):
            out[3 + d][s:e].normal_(generator=g)
    return out
