"""Particle-in-Fourier (PIF) oracle -- TEST INFRASTRUCTURE (NumPy, FP64).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module; it shares no code with the HIP path.

What it follows:
  * PIF (Sec. 3.4): the charge density's Fourier coefficients come straight
    from the particles by a type-1 non-uniform transform,
        rho_hat(k) = sum_j q_j exp(-i k . x_j),   k in K_N,
    Poisson's equation is solved mode by mode, |k|^2 phi_hat = rho_hat
    (eps0 = 1; the k = 0 mode, which the neutralising background cancels,
    is dropped), E_hat = -i k phi_hat, and the field at the particles comes
    back by a type-2 transform,
        E(x_j) = (1/L^3) sum_k E_hat(k) exp(i k . x_j)
    (the 1/L^3 of the Fourier series of a periodic function on [0, L)^3).
  * K_N = (2 pi / L) {-N/2, ..., N/2 - 1}^3 (appendix, NUFFT), N even.
  * NUFFT (appendix, Eqs. type1nufft and type2nufft): spread with a compact
    window onto an oversampled grid of M = sigma N points per axis (sigma = 2),
    uniform FFT, keep the modes of K_N, divide by the window's Fourier
    transform; type 2 reverses the steps.

Readings (the paper names neither the window nor its width):
  * window: the "exponential of semicircle" kernel of Barnett, Magland and
    af Klinteberg (SIAM J. Sci. Comput. 41, 2019),
        phi(z) = exp(beta (sqrt(1 - z^2) - 1)) for |z| <= 1, 0 otherwise,
    over w grid points with w = ceil(log10(1/eps)) + 1 and beta = 2.30 w
    (their choice for sigma = 2); the paper's NUFFT tolerance is 1e-4
    (Sec. 4), i.e. w = 5.
  * a point at s = x / h (h = L / M) touches the w grid points
    i0, ..., i0 + w - 1 with i0 = ceil(s - w/2), at offsets
    z = (i - s) / (w/2) in [-1, 1), indices taken modulo M.
  * the field is the real part of the type-2 sum (the modes with a
    component -N/2 have no partner in K_N).
The window's Fourier transform is formed by Gauss-Legendre quadrature (in
the angle of t = sin(theta), where the integrand is smooth).
"""
from __future__ import annotations

import math

import numpy as np


def modes(N: int) -> np.ndarray:
    """Integer mode numbers -N/2 .. N/2-1 (index m + N/2)."""
    if N % 2:
        raise ValueError("N must be even")
    return np.arange(-N // 2, N // 2)


def wavenumbers(L: float, N: int) -> np.ndarray:
    return 2.0 * math.pi / L * modes(N)


# -------------------------------------------------------------- NUDFT ----

def nudft1(L: float, N: int, pos, q) -> np.ndarray:
    """rho_hat[kz, ky, kx] = sum_j q_j exp(-i k . x_j) by the direct sum
    (exp of a sum is the product of the three axis factors)."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    k = wavenumbers(L, N)
    ex = np.exp(-1j * np.outer(pos[:, 0], k))
    ey = np.exp(-1j * np.outer(pos[:, 1], k))
    ez = np.exp(-1j * np.outer(pos[:, 2], k))
    return np.einsum("j,jc,jb,ja->cba", q, ez, ey, ex, optimize=True)


def nudft2(L: float, N: int, fhat, pos) -> np.ndarray:
    """f(x_j) = sum_k fhat[kz, ky, kx] exp(i k . x_j) by the direct sum."""
    pos = np.asarray(pos, dtype=np.float64)
    k = wavenumbers(L, N)
    ex = np.exp(1j * np.outer(pos[:, 0], k))
    ey = np.exp(1j * np.outer(pos[:, 1], k))
    ez = np.exp(1j * np.outer(pos[:, 2], k))
    return np.einsum("cba,jc,jb,ja->j", fhat, ez, ey, ex, optimize=True)


# ------------------------------------------------------------- window ----

def es_params(eps: float):
    """(w, beta) of the exponential-of-semicircle window for tolerance eps."""
    w = int(math.ceil(math.log10(1.0 / eps))) + 1
    w = min(max(w, 2), 16)
    return w, 2.30 * w


def es_kernel(z, beta):
    z = np.asarray(z, dtype=np.float64)
    inside = np.abs(z) <= 1.0
    return np.where(inside, np.exp(beta * (np.sqrt(np.where(inside, 1.0 - z * z, 0.0)) - 1.0)),
                    0.0)


def window_ft(k, h: float, w: int, beta: float, nq: int = 100) -> np.ndarray:
    """psi_hat(k) = int psi(x) exp(-i k x) dx for psi(x) = phi(x / (w h / 2)):
    (w h / 2) int_{-1}^{1} phi(t) cos(k t w h / 2) dt (phi is even), with
    t = sin(theta) so that the integrand is smooth:
    (w h / 2) int_{-pi/2}^{pi/2} exp(beta (cos theta - 1)) cos(k (w h / 2) sin theta)
    cos theta dtheta, by Gauss-Legendre quadrature in theta."""
    g, wt = np.polynomial.legendre.leggauss(nq)
    th = 0.5 * np.pi * g
    a = 0.5 * w * h
    f = np.exp(beta * (np.cos(th) - 1.0)) * np.cos(th) * (0.5 * np.pi * wt)
    k = np.asarray(k, dtype=np.float64)
    return a * np.cos(np.multiply.outer(k, np.sin(th)) * a) @ f


def _stencil(s, w, M):
    """Grid indices (mod M) and offsets z of the w points a coordinate s = x/h
    touches: i0 = ceil(s - w/2), z = (i - s)/(w/2)."""
    i0 = np.ceil(s - 0.5 * w).astype(np.int64)
    idx = i0[:, None] + np.arange(w)[None, :]
    z = (idx - s[:, None]) / (0.5 * w)
    return np.mod(idx, M), z


# ------------------------------------------------------------- NUFFT ----

def nufft1(L: float, N: int, pos, q, eps: float, sigma: int = 2) -> np.ndarray:
    """Type 1 by spread -> FFT -> select K_N -> divide by the window's
    transform (appendix, Eq. type1nufft)."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    w, beta = es_params(eps)
    M = sigma * N
    h = L / M
    grid = np.zeros((M, M, M))
    ix, zx = _stencil(pos[:, 0] / h, w, M)
    iy, zy = _stencil(pos[:, 1] / h, w, M)
    iz, zz = _stencil(pos[:, 2] / h, w, M)
    wx, wy, wz = es_kernel(zx, beta), es_kernel(zy, beta), es_kernel(zz, beta)
    for c in range(w):
        for b in range(w):
            for a in range(w):
                np.add.at(grid, (iz[:, c], iy[:, b], ix[:, a]), q * ((wz[:, c] * wy[:, b]) * wx[:, a]))
    G = np.fft.fftn(grid)                  # sum_m g[m] exp(-2 pi i k m / M)
    m = modes(N)
    sel = np.mod(m, M)
    Gk = G[np.ix_(sel, sel, sel)]
    c1 = h / window_ft(wavenumbers(L, N), h, w, beta)
    return Gk * (c1[:, None, None] * c1[None, :, None] * c1[None, None, :])


def nufft2(L: float, N: int, fhat, pos, eps: float, sigma: int = 2) -> np.ndarray:
    """Type 2 by the reversed steps (appendix, Eq. type2nufft)."""
    pos = np.asarray(pos, dtype=np.float64)
    w, beta = es_params(eps)
    M = sigma * N
    h = L / M
    c1 = h / window_ft(wavenumbers(L, N), h, w, beta)
    F = np.zeros((M, M, M), dtype=np.complex128)
    sel = np.mod(modes(N), M)
    F[np.ix_(sel, sel, sel)] = fhat * (c1[:, None, None] * c1[None, :, None] * c1[None, None, :])
    u = np.fft.ifftn(F) * (M ** 3)         # sum_k F(k) exp(+2 pi i k m / M)
    ix, zx = _stencil(pos[:, 0] / h, w, M)
    iy, zy = _stencil(pos[:, 1] / h, w, M)
    iz, zz = _stencil(pos[:, 2] / h, w, M)
    wx, wy, wz = es_kernel(zx, beta), es_kernel(zy, beta), es_kernel(zz, beta)
    out = np.zeros(pos.shape[0], dtype=np.complex128)
    for c in range(w):
        for b in range(w):
            for a in range(w):
                out += u[iz[:, c], iy[:, b], ix[:, a]] * ((wz[:, c] * wy[:, b]) * wx[:, a])
    return out


# --------------------------------------------------------- PIF field ----

def field_spectrum(L: float, N: int, rho_hat) -> list:
    """E_hat_d = -i k_d rho_hat / |k|^2 (zero at k = 0), d = x, y, z."""
    k = wavenumbers(L, N)
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    k2 = KX * KX + KY * KY + KZ * KZ
    k2[N // 2, N // 2, N // 2] = 1.0
    phi = rho_hat / k2
    phi[N // 2, N // 2, N // 2] = 0.0
    return [-1j * KX * phi, -1j * KY * phi, -1j * KZ * phi]


def pif_efield(L: float, N: int, pos, q, eps: float | None = None) -> np.ndarray:
    """E at the particles, (Np, 3): exact non-uniform DFTs when eps is None,
    NUFFTs of tolerance eps otherwise."""
    if eps is None:
        rho_hat = nudft1(L, N, pos, q)
        back = lambda f: nudft2(L, N, f, pos)
    else:
        rho_hat = nufft1(L, N, pos, q, eps)
        back = lambda f: nufft2(L, N, f, pos, eps)
    Ek = field_spectrum(L, N, rho_hat)
    return np.stack([back(e).real / L ** 3 for e in Ek], axis=1)


def hermitian_part(L: float, N: int, fhat) -> np.ndarray:
    """The spectrum of Re(sum_k fhat(k) exp(i k.x)) on the mode set
    K_N u -K_N, as an array over -N/2 .. N/2 per axis (index m + N/2):
    (fhat(k) + conj(fhat(-k))) / 2, each term where its mode is in K_N."""
    F = np.zeros((N + 1, N + 1, N + 1), dtype=np.complex128)
    F[:N, :N, :N] += 0.5 * fhat
    F[1:, 1:, 1:] += 0.5 * np.conj(fhat[::-1, ::-1, ::-1])
    return F


def pif_wx(L: float, N: int, rho_hat) -> float:
    """W_x = (1/2) int E_x^2 dx of the real field, by Parseval:
    (1 / (2 L^3)) sum |E_hat_x|^2 over the Hermitian part of its spectrum."""
    ex = field_spectrum(L, N, rho_hat)[0]
    H = hermitian_part(L, N, ex)
    return float(np.sum(np.abs(H) ** 2) / (2.0 * L ** 3))
