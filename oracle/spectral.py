"""FFT Poisson solves of the oracle (test infrastructure; only tests/, the
smoke check and the benchmark's CPU baseline use this package).

The paper's FFT solver (Sec. 3.1) is pseudo-spectral: phi_hat = rho_hat / |k|^2
on the periodic box, E = -grad phi by multiplying with -i k.  The discrete
variant divides by the eigenvalues of the 7-point operator instead,
lambda(m) = sum_d (2 - 2 cos(2 pi m_d / N)) / h^2, which gives the exact
zero-mean solution of the same linear system the PCG solves (the system is
circulant).  numpy's FFT is the library primitive; the mean (m = 0) mode is
set to zero in both."""
from __future__ import annotations

import numpy as np


def _modes(N):
    return np.fft.fftfreq(N, d=1.0 / N)  # signed integers 0, 1, ..., -1


def symbol(N: int, L: float, kind: str = "discrete") -> np.ndarray:
    """Multiplier of -Laplacian per Fourier mode, [z][y][x] order, full grid."""
    m = _modes(N)
    if kind == "discrete":
        h = L / N
        s = (2.0 - 2.0 * np.cos(2.0 * np.pi * m / N)) / h ** 2
    elif kind == "spectral":
        s = (2.0 * np.pi * m / L) ** 2
    else:
        raise ValueError(kind)
    return s[:, None, None] + s[None, :, None] + s[None, None, :]


def fft_poisson(N: int, L: float, b, kind: str = "discrete") -> np.ndarray:
    """phi with -Lap phi = b (zero-mean part), by the chosen symbol."""
    bh = np.fft.fftn(np.asarray(b, dtype=np.float64).reshape(N, N, N))
    lam = symbol(N, L, kind)
    lam[0, 0, 0] = 1.0
    ph = bh / lam
    ph[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(ph)).ravel()


def spectral_field(N: int, L: float, phi):
    """E = -grad phi by -i k multiplication (the Nyquist derivative set to 0)."""
    m = _modes(N).copy()
    if N % 2 == 0:
        m[N // 2] = 0.0
    k = 2.0 * np.pi * m / L
    ph = np.fft.fftn(np.asarray(phi, dtype=np.float64).reshape(N, N, N))
    ex = np.real(np.fft.ifftn(-1j * k[None, None, :] * ph)).ravel()
    ey = np.real(np.fft.ifftn(-1j * k[None, :, None] * ph)).ravel()
    ez = np.real(np.fft.ifftn(-1j * k[:, None, None] * ph)).ravel()
    return ex, ey, ez
