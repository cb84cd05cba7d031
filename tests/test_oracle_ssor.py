"""Pins of the oracle's SSOR preconditioner and SSOR-PCG (Sec. 4.1 names SSOR
with four inner and two outer iterations and damping pi/2; the reading is
stated in the oracle).  Every operator here is circulant, so each Fourier
mode is an eigenvector with a multiplier in closed form; and with many inner
iterations the approximate solves converge to the textbook SSOR, which an FFT
applies exactly."""
import math

import numpy as np
import pytest

from paper_2605_05469_amd import synth

W = math.pi / 2


def _theta(N, m):
    return 2 * np.pi * np.asarray(m, dtype=float) / N


def _multiplier(N, L, m, omega, inner, outer):
    """Closed form of the SSOR multiplier on the mode exp(i theta.x)."""
    h = L / N
    th = _theta(N, m)
    s = np.sum(np.exp(-1j * th))          # backward shifts
    c = omega / 6.0
    dinv = h * h / 6.0
    P = sum((c * s) ** j for j in range(inner + 1))
    mu = omega * (2 - omega) * dinv * abs(P) ** 2
    lam = np.sum(2 - 2 * np.cos(th)) / h ** 2
    z = 0.0
    for _ in range(outer):
        z = z + mu * (1.0 - lam * z)      # z <- z + M(r - A z) on the mode, r = 1
    return z


def _mode(N, m):
    i = np.arange(N)
    Z, Y, X = np.meshgrid(i, i, i, indexing="ij")
    th = _theta(N, m)
    return np.cos(th[0] * X + th[1] * Y + th[2] * Z).ravel()


@pytest.mark.parametrize("m,inner,outer", [((1, 0, 0), 4, 2), ((3, 5, 2), 4, 2),
                                           ((7, 1, 4), 1, 1), ((8, 8, 8), 6, 3),
                                           ((2, 0, 5), 0, 2)])
def test_ssor_fourier_multiplier(orc, m, inner, outer):
    N, L = 16, 4 * math.pi
    u = _mode(N, m)
    z = orc.ssor_apply(N, L, u, W, inner, outer)
    mu = _multiplier(N, L, m, W, inner, outer)
    assert np.max(np.abs(z - mu * u)) <= 1e-12 * max(abs(mu), 1e-300)


def test_ssor_symmetric_positive(orc):
    N, L = 12, 4 * math.pi
    rng = np.random.default_rng(1)
    u, v = rng.standard_normal(N ** 3), rng.standard_normal(N ** 3)
    Mu, Mv = orc.ssor_apply(N, L, u), orc.ssor_apply(N, L, v)
    assert abs(Mu @ v - u @ Mv) <= 1e-12 * np.linalg.norm(Mu) * np.linalg.norm(v)
    assert Mu @ u > 0 and Mv @ v > 0


def test_ssor_many_inner_is_textbook_ssor(orc):
    """inner -> infinity: w (2 - w) (D + w U)^-1 D (D + w L)^-1, applied by FFT."""
    N, L = 16, 4 * math.pi
    h = L / N
    rng = np.random.default_rng(2)
    r = rng.standard_normal(N ** 3)
    z = orc.ssor_apply(N, L, r, W, 150, 1)
    th = 2 * np.pi * np.fft.fftfreq(N)
    TZ, TY, TX = np.meshgrid(th, th, th, indexing="ij")
    d = 6 / h ** 2
    lo = d - (W / h ** 2) * (np.exp(-1j * TX) + np.exp(-1j * TY) + np.exp(-1j * TZ))
    up = np.conj(lo)
    zh = W * (2 - W) * d * np.fft.fftn(r.reshape(N, N, N)) / (lo * up)
    ref = np.real(np.fft.ifftn(zh)).ravel()
    assert np.max(np.abs(z - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_pcg_ssor_converges_in_fewer_iterations(orc):
    N = 32
    P = synth.LandauParams(N=N, ppc=8)
    parts = synth.landau_particles_np(N, 8, seed=18)
    b, _ = orc.deposit(N, P.L, P.q, P.rho_bg, *parts[:3])
    x, info = orc.pcg_ssor(N, P.L, b, np.zeros(N ** 3), 1e-10, 5000)
    assert info["converged"]
    # true residual with an operator applied independently of the oracle (FFT)
    h = P.L / N
    m = np.arange(N)
    s = (2 - 2 * np.cos(2 * np.pi * m / N)) / h ** 2
    lam = s[:, None, None] + s[None, :, None] + s[None, None, :]
    Ax = np.real(np.fft.ifftn(np.fft.fftn(x.reshape(N, N, N)) * lam)).ravel()
    assert np.linalg.norm(b - Ax) <= 1.0001e-10 * np.linalg.norm(b)
    _, pj = orc.pcg(N, P.L, b, np.zeros(N ** 3), 1e-10, 5000)
    assert info["iters"] < pj["iters"]
