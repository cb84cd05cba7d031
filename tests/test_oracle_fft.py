"""Pins of the oracle's FFT Poisson solves (the paper's FFT solver, Sec. 3.1,
and the discrete-symbol variant that solves the PCG's own system)."""
import math

import numpy as np
import pytest

from oracle import spectral
from paper_2605_05469_amd import synth


def _grid(N, L):
    x = np.arange(N) * (L / N)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return X, Y, Z


@pytest.mark.parametrize("m", [(1, 0, 0), (2, 3, 1), (0, 0, 5)])
def test_single_mode_closed_forms(m):
    N, L = 16, 4 * math.pi
    X, Y, Z = _grid(N, L)
    k = [2 * math.pi * mi / L for mi in m]
    b = np.cos(k[0] * X + k[1] * Y + k[2] * Z).ravel()
    h = L / N
    lam_d = sum((2 - 2 * math.cos(ki * h)) / h ** 2 for ki in k)
    lam_s = sum(ki ** 2 for ki in k)
    assert np.max(np.abs(spectral.fft_poisson(N, L, b, "discrete") - b / lam_d)) <= 1e-13 / lam_d
    phi = spectral.fft_poisson(N, L, b, "spectral")
    assert np.max(np.abs(phi - b / lam_s)) <= 1e-13 / lam_s
    # E = -grad phi = sin(k.x) k / lam_s exactly for the spectral field
    s = np.sin(k[0] * X + k[1] * Y + k[2] * Z).ravel()
    for E, kd in zip(spectral.spectral_field(N, L, phi), k):
        assert np.max(np.abs(E - kd * s / lam_s)) <= 1e-13 * (1 + abs(kd) / lam_s)


def test_discrete_symbol_solves_the_pcg_system(orc):
    N = 32
    P = synth.LandauParams(N=N, ppc=8)
    parts = synth.landau_particles_np(N, 8, seed=19)
    b, _ = orc.deposit(N, P.L, P.q, P.rho_bg, *parts[:3])
    phi = spectral.fft_poisson(N, P.L, b, "discrete")
    # the oracle's own 7-point operator (not an FFT) reproduces b
    assert orc.residual_norm(N, P.L, b, phi) <= 1e-12 * np.linalg.norm(b)
    assert abs(phi.mean()) <= 1e-14 * np.abs(phi).max()


def test_discrete_symbol_dense_direct_solve():
    """4^3: the dense (A + 11^T / N^3) solve with A assembled entry by entry."""
    N, L = 4, 3.0
    h = L / N
    n3 = N ** 3
    A = np.zeros((n3, n3))
    idx = lambda x, y, z: ((z % N) * N + (y % N)) * N + (x % N)
    for z in range(N):
        for y in range(N):
            for x in range(N):
                i = idx(x, y, z)
                A[i, i] += 6 / h ** 2
                for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    A[i, idx(x + dx, y + dy, z + dz)] -= 1 / h ** 2
    rng = np.random.default_rng(4)
    b = rng.standard_normal(n3)
    b -= b.mean()
    ref = np.linalg.solve(A + np.ones((n3, n3)) / n3, b)
    assert np.max(np.abs(spectral.fft_poisson(N, L, b, "discrete") - ref)) <= 1e-12 * np.abs(ref).max()
