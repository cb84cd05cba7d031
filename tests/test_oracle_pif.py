"""Pins of the PIF oracle (Sec. 3.4 and the NUFFT appendix): the non-uniform
DFTs against closed forms, a uniform lattice (where they reduce to NumPy's
FFT) and their adjointness; the NUFFTs against the direct sums within the
requested tolerance (the paper's NUFFT tolerance is 1e-4); the PIF field of a
single-mode charge density against its closed form; and W_x against a
quadrature that is exact for the field's trigonometric polynomial."""
import math

import numpy as np
import pytest

from oracle import pif
from paper_2605_05469_amd import synth

L = 4 * math.pi


def _particles(n, seed, L=L):
    u = synth.normal_field(4 * n, seed)
    pos = (0.5 + np.arctan(u[: 3 * n]) / math.pi).reshape(n, 3) * L   # in (0, L)
    q = u[3 * n:]
    return pos, q


def test_nudft_single_particle_closed_forms():
    N = 8
    k = pif.wavenumbers(L, N)
    # a particle at the origin: every coefficient is q
    assert np.allclose(pif.nudft1(L, N, [[0.0, 0.0, 0.0]], [2.5]), 2.5, atol=1e-15)
    # at x = (L/2, 0, L/4): exp(-i pi mx) exp(-i pi mz / 2)
    got = pif.nudft1(L, N, [[L / 2, 0.0, L / 4]], [1.0])
    m = pif.modes(N)
    ref = np.exp(-1j * np.pi * m)[None, None, :] * np.exp(-0.5j * np.pi * m)[:, None, None]
    assert np.allclose(got, np.broadcast_to(ref, got.shape), atol=1e-13)
    # type 2 of one mode is that plane wave
    f = np.zeros((N, N, N), dtype=complex)
    f[N // 2 + 1, N // 2 - 2, N // 2 + 3] = 1.0          # (kz, ky, kx) = (1, -2, 3)
    pos, _ = _particles(7, 1)
    kk = 2 * np.pi / L * np.array([3, -2, 1])
    assert np.allclose(pif.nudft2(L, N, f, pos), np.exp(1j * pos @ kk), atol=1e-13)
    assert k[0] == -np.pi * N / L


def test_nudft_on_a_lattice_is_the_fft():
    """Particles on the N^3 lattice x = i L/N: the type-1 sum is NumPy's FFT
    with the modes reordered to -N/2 .. N/2-1."""
    N = 8
    i = np.arange(N)
    Z, Y, X = np.meshgrid(i, i, i, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1) * (L / N)
    g = synth.normal_field(N ** 3, 3)
    ref = np.fft.fftshift(np.fft.fftn(g.reshape(N, N, N)))
    assert np.allclose(pif.nudft1(L, N, pos, g), ref, atol=1e-11)


def test_nudft_types_are_adjoint():
    N = 6
    pos, q = _particles(40, 5)
    f = (synth.normal_field(N ** 3, 6) + 1j * synth.normal_field(N ** 3, 7)).reshape(N, N, N)
    lhs = np.vdot(f, pif.nudft1(L, N, pos, q))            # <f, A q>
    rhs = np.vdot(pif.nudft2(L, N, f, pos), q)            # <A^H f, q>
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_window_transform_quadrature():
    """psi_hat(0) is the window's integral; a finer quadrature agrees."""
    w, beta = pif.es_params(1e-4)
    assert (w, beta) == (5, 11.5)
    h = 0.3
    t = np.linspace(-1, 1, 200001)
    integral = 0.5 * w * h * np.trapezoid(pif.es_kernel(t, beta), t)
    assert abs(pif.window_ft(0.0, h, w, beta) - integral) <= 1e-7 * integral
    k = np.linspace(0, np.pi / h, 7)
    assert np.allclose(pif.window_ft(k, h, w, beta), pif.window_ft(k, h, w, beta, nq=300),
                       rtol=1e-13, atol=0)


@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-9])
def test_nufft_type1_within_tolerance(eps):
    N = 12
    pos, q = _particles(300, 11)
    ref = pif.nudft1(L, N, pos, q)
    got = pif.nufft1(L, N, pos, q, eps)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    # the width rule w = ceil(log10(1/eps)) + 1 gives about eps (within a
    # small factor) for the exponential-of-semicircle window at sigma = 2
    assert err <= 10 * eps, err


@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-9])
def test_nufft_type2_within_tolerance(eps):
    N = 12
    pos, _ = _particles(300, 12)
    f = (synth.normal_field(N ** 3, 13) + 1j * synth.normal_field(N ** 3, 14)).reshape(N, N, N)
    ref = pif.nudft2(L, N, f, pos)
    got = pif.nufft2(L, N, f, pos, eps)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    # the width rule w = ceil(log10(1/eps)) + 1 gives about eps (within a
    # small factor) for the exponential-of-semicircle window at sigma = 2
    assert err <= 10 * eps, err


def test_pif_field_of_a_single_mode():
    """Charges q_j = A cos(k0.x_j) (L/n)^3 on an n^3 lattice (n >= N): the
    lattice sums are exact (discrete orthogonality), so rho_hat is
    (A L^3 / 2) at +-k0, phi = A cos(k0.x) / |k0|^2 and
    E = A k0 sin(k0.x) / |k0|^2."""
    N, n = 8, 10
    i = np.arange(n)
    Z, Y, X = np.meshgrid(i, i, i, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1) * (L / n)
    k0 = 2 * np.pi / L * np.array([1.0, -2.0, 3.0])
    A = 0.7
    q = A * np.cos(pos @ k0) * (L / n) ** 3
    E = pif.pif_efield(L, N, pos, q)
    ref = A * np.outer(np.sin(pos @ k0), k0) / np.dot(k0, k0)
    assert np.max(np.abs(E - ref)) <= 1e-12 * np.abs(ref).max()
    # the same field through NUFFTs, within their tolerance
    En = pif.pif_efield(L, N, pos, q, eps=1e-9)
    assert np.max(np.abs(En - ref)) <= 1e-8 * np.abs(ref).max()


def test_pif_field_matches_minus_gradient_of_phi():
    """E at the particles equals -grad of the mode-sum potential, by central
    differences of a tiny step (independent of the -i k factor)."""
    N = 6
    pos, q = _particles(30, 21)
    rho = pif.nudft1(L, N, pos, q)
    k = pif.wavenumbers(L, N)
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    k2[N // 2, N // 2, N // 2] = np.inf
    phi_hat = rho / k2
    probe = pos[:5]
    d = 1e-5
    E = pif.pif_efield(L, N, pos, q)[:5]
    for ax in range(3):
        e = np.zeros(3)
        e[ax] = d
        fp = pif.nudft2(L, N, phi_hat, probe + e).real / L ** 3
        fm = pif.nudft2(L, N, phi_hat, probe - e).real / L ** 3
        assert np.allclose(E[:, ax], -(fp - fm) / (2 * d), rtol=1e-6, atol=1e-9)


def test_pif_wx_is_the_field_energy():
    """(1/2) int E_x^2: the real field is a trigonometric polynomial of
    degree <= N/2, so a uniform grid of more than N points per axis
    integrates its square exactly."""
    N = 6
    pos, q = _particles(25, 31)
    rho = pif.nudft1(L, N, pos, q)
    n = N + 2
    i = np.arange(n)
    Z, Y, X = np.meshgrid(i, i, i, indexing="ij")
    grid = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1) * (L / n)
    ex = pif.field_spectrum(L, N, rho)[0]
    Ex = pif.nudft2(L, N, ex, grid).real / L ** 3
    ref = 0.5 * np.sum(Ex ** 2) * (L / n) ** 3
    assert abs(pif.pif_wx(L, N, rho) - ref) <= 1e-12 * ref
