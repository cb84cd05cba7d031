"""Pins of the oracle's bounded boxes: the PCG solver's Dirichlet and Neumann
boundaries (Sec. 3.2 and the solver table of Sec. 3 list both for PCG; the
discretisation is the oracle's reading).  The operator is checked against a
dense matrix assembled independently from 1-D second-difference matrices,
against the sine (Dirichlet) and cosine (Neumann) eigenvectors with their
closed-form eigenvalues, and the solves against the discrete sine and cosine
transforms that diagonalise it; the SSOR factors of the bounded box are true
triangular matrices, so with enough inner steps the preconditioner is the
textbook SSOR applied by dense triangular solves."""
import math

import numpy as np
import pytest
import scipy.fft
import scipy.linalg

from paper_2605_05469_amd import synth

DIR, NEU = 1, 2
L = 4 * math.pi
W = math.pi / 2


def _h(N, bc):
    return L / (N + 1) if bc == DIR else L / N


def _t1(N, bc):
    """1-D second difference (times h^2): Dirichlet ends drop the outside
    neighbour, Neumann ends mirror it (the end's own value cancels once)."""
    T = 2 * np.eye(N) - np.eye(N, k=1) - np.eye(N, k=-1)
    if bc == NEU:
        T[0, 0] -= 1.0
        T[-1, -1] -= 1.0
    return T


def _dense(N, bc):
    """A = (Tz x I x I + I x Ty x I + I x I x Tx) / h^2 for the [iz][iy][ix]
    layout (ix fastest)."""
    T, I = _t1(N, bc), np.eye(N)
    A = np.kron(np.kron(T, I), I) + np.kron(np.kron(I, T), I) + np.kron(np.kron(I, I), T)
    return A / _h(N, bc) ** 2


def _rand(N, seed):
    return synth.normal_field(N ** 3, seed)


@pytest.mark.parametrize("bc", [DIR, NEU])
@pytest.mark.parametrize("N", [1, 2, 5])
def test_operator_equals_assembled_matrix(orc, bc, N):
    u = _rand(N, 10 + N + bc)
    got = orc.apply_A(N, L, u, bc=bc)
    ref = _dense(N, bc) @ u
    assert np.allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max() + 1e-300)


def _modes(N, bc, m):
    i = np.arange(N)
    if bc == DIR:
        th = [np.pi * mm / (N + 1) for mm in m]
        f = [np.sin(t * (i + 1)) for t in th]
        lam = sum(4 * np.sin(t / 2) ** 2 for t in th) / _h(N, bc) ** 2
    else:
        th = [np.pi * mm / N for mm in m]
        f = [np.cos(t * (i + 0.5)) for t in th]
        lam = sum(4 * np.sin(t / 2) ** 2 for t in th) / _h(N, bc) ** 2
    u = np.einsum("k,j,i->kji", f[2], f[1], f[0]).reshape(-1)
    return u, lam, th


@pytest.mark.parametrize("bc,m", [(DIR, (1, 1, 1)), (DIR, (3, 1, 7)), (DIR, (12, 2, 5)),
                                  (NEU, (1, 0, 0)), (NEU, (2, 3, 5)), (NEU, (11, 11, 1))])
def test_eigenvectors(orc, bc, m):
    """Sine modes vanish on the Dirichlet boundary; cosine modes at the cell
    centres have zero normal difference at the faces: A u = lambda u."""
    N = 12
    u, lam, _ = _modes(N, bc, m)
    got = orc.apply_A(N, L, u, bc=bc)
    assert np.max(np.abs(got - lam * u)) <= 1e-12 * lam


def test_constants(orc):
    """Neumann: constants are the kernel (A 1 = 0 exactly).  Dirichlet:
    A 1 = m / h^2 where m counts the faces a point touches."""
    N = 6
    one = np.ones(N ** 3)
    assert np.array_equal(orc.apply_A(N, L, one, bc=NEU), np.zeros(N ** 3))
    i = np.arange(N)
    e = ((i == 0).astype(int) + (i == N - 1).astype(int))
    m = (e[:, None, None] + e[None, :, None] + e[None, None, :]).reshape(-1)
    assert np.allclose(orc.apply_A(N, L, one, bc=DIR), m / _h(N, DIR) ** 2, rtol=1e-14, atol=0)


@pytest.mark.parametrize("bc", [DIR, NEU])
def test_operator_is_symmetric(orc, bc):
    N = 9
    u, v = _rand(N, 21), _rand(N, 22)
    a = np.dot(orc.apply_A(N, L, u, bc=bc), v)
    b = np.dot(u, orc.apply_A(N, L, v, bc=bc))
    assert abs(a - b) <= 1e-13 * abs(a)


def _transform_solve(N, bc, b):
    """The discrete sine (DST-I) / cosine (DCT-II) transform diagonalises the
    Dirichlet / Neumann operator; the Neumann solution has zero mean."""
    h = _h(N, bc)
    B = b.reshape(N, N, N)
    m = np.arange(N)
    if bc == DIR:
        s = 4 * np.sin(np.pi * (m + 1) / (2 * (N + 1))) ** 2 / h ** 2
        lam = s[:, None, None] + s[None, :, None] + s[None, None, :]
        return scipy.fft.idstn(scipy.fft.dstn(B, type=1) / lam, type=1).reshape(-1)
    s = 4 * np.sin(np.pi * m / (2 * N)) ** 2 / h ** 2
    lam = s[:, None, None] + s[None, :, None] + s[None, None, :]
    bh = scipy.fft.dctn(B, type=2)
    lam[0, 0, 0] = 1.0
    bh = bh / lam
    bh[0, 0, 0] = 0.0
    return scipy.fft.idctn(bh, type=2).reshape(-1)


@pytest.mark.parametrize("bc", [DIR, NEU])
def test_pcg_matches_transform_solve(orc, bc):
    N = 16
    b = _rand(N, 30 + bc)
    if bc == NEU:
        b -= b.mean()       # solvability of the Neumann problem
    ref = _transform_solve(N, bc, b)
    x, info = orc.pcg(N, L, b, np.zeros(N ** 3), 1e-12, 5000, bc=bc)
    assert info["converged"]
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)
    assert orc.residual_norm(N, L, b, x, bc=bc) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("bc", [DIR, NEU])
def test_pcg_matches_dense_solve(orc, bc):
    N = 4
    b = _rand(N, 40 + bc)
    A = _dense(N, bc)
    if bc == NEU:
        b -= b.mean()
        ref = np.linalg.lstsq(A, b, rcond=None)[0]   # minimum norm = zero mean
    else:
        ref = np.linalg.solve(A, b)
    x, info = orc.pcg(N, L, b, np.zeros(N ** 3), 1e-13, 1000, bc=bc)
    assert info["converged"]
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("bc,m", [(DIR, (1, 2, 3)), (DIR, (7, 1, 1)), (NEU, (1, 2, 3)),
                                  (NEU, (0, 5, 1))])
def test_field_of_modes(orc, bc, m):
    """Central differences through the boundary rule, in closed form:
    Dirichlet sin(t(i+1)) -> -cos(t(i+1)) sin(t) / h; Neumann cos(t(i+1/2))
    -> sin(t(i+1/2)) sin(t) / h (the mirrored value is the mode's own value
    across the face).  A Dirichlet potential keeps its mean."""
    N = 10
    h = _h(N, bc)
    u, _, th = _modes(N, bc, m)
    i = np.arange(N)
    if bc == DIR:
        f = [np.sin(t * (i + 1)) for t in th]
        d = [-np.cos(t * (i + 1)) * np.sin(t) / h for t in th]
    else:
        f = [np.cos(t * (i + 0.5)) for t in th]
        d = [np.sin(t * (i + 0.5)) * np.sin(t) / h for t in th]
    phi, ex, ey, ez, wx = orc.efield(N, L, u, bc=bc)
    if bc == DIR:
        assert np.array_equal(phi, u)
    else:
        assert np.allclose(phi, u - u.mean(), rtol=0, atol=1e-15)
    rex = np.einsum("k,j,i->kji", f[2], f[1], d[0]).reshape(-1)
    rey = np.einsum("k,j,i->kji", f[2], d[1], f[0]).reshape(-1)
    rez = np.einsum("k,j,i->kji", d[2], f[1], f[0]).reshape(-1)
    for a, r in ((ex, rex), (ey, rey), (ez, rez)):
        assert np.max(np.abs(a - r)) <= 1e-13 * (np.abs(r).max() + 1.0 / h)
    assert abs(wx - 0.5 * h ** 3 * np.sum(rex ** 2)) <= 1e-12 * max(wx, 1e-300)


def _textbook_ssor(N, bc, r, omega):
    """omega (2 - omega) (D + omega U)^-1 D (D + omega L)^-1 r with D the
    interior diagonal 6/h^2 and L, U the strictly lower / upper parts of the
    bounded operator (its couplings between unknowns)."""
    A = _dense(N, bc)
    D = 6.0 / _h(N, bc) ** 2
    Lo, Up = np.tril(A, -1), np.triu(A, 1)
    y = scipy.linalg.solve_triangular(D * np.eye(N ** 3) + omega * Lo, r, lower=True)
    z = scipy.linalg.solve_triangular(D * np.eye(N ** 3) + omega * Up, D * y, lower=False)
    return omega * (2 - omega) * z


@pytest.mark.parametrize("bc", [DIR, NEU])
def test_ssor_is_textbook_in_the_exact_limit(orc, bc):
    """On the bounded grid the longest chain of backward neighbours has 3N-3
    links, so (D^-1 L)^(3N-2) = 0 and 3N-3 inner Jacobi steps (the Neumann
    series through that power) solve each triangular system exactly."""
    N = 4
    r = _rand(N, 50 + bc)
    got = orc.ssor_apply(N, L, r, W, inner=3 * N - 3, outer=1, bc=bc)
    ref = _textbook_ssor(N, bc, r, W)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)
    # one inner step short of exact differs
    short = orc.ssor_apply(N, L, r, W, inner=3 * N - 4, outer=1, bc=bc)
    assert np.linalg.norm(short - ref) > 1e-8 * np.linalg.norm(ref)


@pytest.mark.parametrize("bc", [DIR, NEU])
def test_ssor_outer_steps_are_stationary_iteration(orc, bc):
    """outer = 2: z = M r + M (r - A M r), the second stationary step."""
    N = 4
    r = _rand(N, 60 + bc)
    A = _dense(N, bc)
    m1 = _textbook_ssor(N, bc, r, W)
    ref = m1 + _textbook_ssor(N, bc, r - A @ m1, W)
    got = orc.ssor_apply(N, L, r, W, inner=3 * N - 3, outer=2, bc=bc)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("bc", [DIR, NEU])
def test_ssor_paper_setting_is_symmetric(orc, bc):
    N = 8
    r, s = _rand(N, 70), _rand(N, 71)
    a = np.dot(orc.ssor_apply(N, L, r, W, 4, 2, bc=bc), s)
    b = np.dot(r, orc.ssor_apply(N, L, s, W, 4, 2, bc=bc))
    assert abs(a - b) <= 1e-12 * abs(a)


@pytest.mark.parametrize("bc", [DIR, NEU])
def test_pcg_ssor_matches_transform_solve(orc, bc):
    N = 16
    b = _rand(N, 80 + bc)
    if bc == NEU:
        b -= b.mean()
    ref = _transform_solve(N, bc, b)
    x, info = orc.pcg_ssor(N, L, b, np.zeros(N ** 3), 1e-12, 2000, bc=bc)
    assert info["converged"]
    if bc == NEU:
        x = x - x.mean()     # the SSOR directions are not mean-free
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)
    _, jinfo = orc.pcg(N, L, b, np.zeros(N ** 3), 1e-12, 5000, bc=bc)
    assert info["iters"] < jinfo["iters"]
