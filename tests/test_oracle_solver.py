"""Pins of the oracle's field pieces (operator, PCG, field, mixed precision,
flexible CG) against closed forms, dense and FFT solves.  CPU only."""
import math

import numpy as np
import pytest

from paper_2605_05469_amd import synth


def _grid(N, L):
    c = np.arange(N) * (L / N)
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    return X, Y, Z


def _lam(N, L, m):
    h = L / N
    return sum(2.0 - 2.0 * math.cos(2 * math.pi * md / N) for md in m) / h ** 2


def _dense_A(N, L):
    """A = (T(x)I(x)I + I(x)T(x)I + I(x)I(x)T)/h^2 with T = circ(-1, 2, -1):
    an assembly independent of the stencil code."""
    T = 2 * np.eye(N) - np.roll(np.eye(N), 1, axis=1) - np.roll(np.eye(N), -1, axis=1)
    I = np.eye(N)
    h = L / N
    return (np.kron(np.kron(T, I), I) + np.kron(np.kron(I, T), I) + np.kron(np.kron(I, I), T)) / h ** 2


def _fft_solve(N, L, b):
    """Exact discrete zero-mean solution: phi_hat(m) = b_hat(m)/lambda(m)."""
    h = L / N
    m = np.arange(N)
    s = (2 - 2 * np.cos(2 * np.pi * m / N)) / h ** 2
    lam = s[:, None, None] + s[None, :, None] + s[None, None, :]
    bh = np.fft.fftn(b.reshape(N, N, N))
    lam[0, 0, 0] = 1.0
    ph = bh / lam
    ph[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(ph)).ravel()


# ------------------------------------------------------------- operator ---

@pytest.mark.parametrize("m", [(1, 0, 0), (0, 2, 0), (1, 1, 3), (4, 4, 4)])
def test_laplacian_single_mode_eigenvalue(orc, m):
    N, L = 8, 4 * math.pi
    X, Y, Z = _grid(N, L)
    k = 2 * np.pi / L
    u = np.cos(k * (m[0] * X + m[1] * Y + m[2] * Z)).ravel()
    Au = orc.apply_A(N, L, u)
    lam = _lam(N, L, m)
    assert np.allclose(Au, lam * u, rtol=0, atol=1e-12 * lam)


def test_laplacian_matches_kron_assembly_symmetric_and_kills_constants(orc):
    N, L = 6, 2.5
    A = _dense_A(N, L)
    rng = np.random.default_rng(11)
    u, v = rng.standard_normal((2, N ** 3))
    assert np.allclose(orc.apply_A(N, L, u), A @ u, rtol=1e-13, atol=1e-11)
    assert abs(orc.apply_A(N, L, u) @ v - u @ orc.apply_A(N, L, v)) < 1e-11 * np.abs(A).sum()
    assert np.all(orc.apply_A(N, L, np.full(N ** 3, 3.7)) == 0.0)


# ------------------------------------------------------------------ PCG ---

@pytest.mark.parametrize("N", [4, 6, 8])
def test_pcg_matches_dense_direct_solve(orc, N):
    L = 4 * math.pi
    rng = np.random.default_rng(N)
    b = rng.standard_normal(N ** 3)
    b -= b.mean()
    A1 = _dense_A(N, L) + np.ones((N ** 3, N ** 3)) / N ** 3
    ref = np.linalg.solve(A1, b)
    x, info = orc.pcg(N, L, b, np.zeros(N ** 3), 1e-14, 10000)
    assert info["converged"] and info["true_rel_res"] <= 1e-14
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("N", [16, 32])
def test_pcg_matches_fft_exact_solution(orc, N):
    P = synth.LandauParams(N=N, ppc=8)
    parts = synth.landau_particles_np(N, 8, seed=100 + N)
    b, nb = orc.deposit(N, P.L, P.q, P.rho_bg, *parts[:3])
    ref = _fft_solve(N, P.L, b)
    x, info = orc.pcg(N, P.L, b, np.zeros(N ** 3), 1e-12, 20000)
    assert info["converged"] and info["true_rel_res"] <= 1e-12
    kappa = 3.0 / math.sin(math.pi / N) ** 2
    assert np.linalg.norm(x - ref) <= kappa * 1e-12 * np.linalg.norm(ref)


def test_pcg_single_mode_converges_in_one_iteration(orc):
    N, L = 16, 4 * math.pi
    X, Y, Z = _grid(N, L)
    k = 2 * np.pi / L
    b = np.cos(k * (X + 2 * Y)).ravel()
    x, info = orc.pcg(N, L, b, np.zeros(N ** 3), 1e-10, 100)
    assert info["iters"] == 1 and info["converged"]
    assert np.allclose(x, b / _lam(N, L, (1, 2, 0)), rtol=0, atol=1e-13)


def test_pcg_terminates_within_number_of_distinct_eigenvalues(orc):
    N, L = 16, 4 * math.pi
    X, Y, Z = _grid(N, L)
    k = 2 * np.pi / L
    b = (np.cos(k * X) + 0.5 * np.sin(k * 3 * Y) - 2.0 * np.cos(k * (2 * Z + X))).ravel()
    x, info = orc.pcg(N, L, b, np.zeros(N ** 3), 1e-10, 100)
    assert info["converged"] and info["iters"] <= 3


def test_pcg_zero_rhs_and_exact_warm_start(orc):
    N, L = 8, 1.0
    x, info = orc.pcg(N, L, np.zeros(N ** 3), np.ones(N ** 3), 1e-10, 100)
    assert info["iters"] == 0 and info["converged"] and np.all(x == 0)
    rng = np.random.default_rng(12)
    b = rng.standard_normal(N ** 3)
    b -= b.mean()
    sol = _fft_solve(N, L, b)
    x, info = orc.pcg(N, L, b, sol, 1e-10, 100)
    assert info["iters"] == 0 and info["converged"]


def test_pcg_warm_start_is_used(orc):
    """Sec. 4.1: the previous solution is the starting guess; a nearby guess
    needs fewer iterations than zero."""
    N = 16
    P = synth.LandauParams(N=N, ppc=8)
    parts = synth.landau_particles_np(N, 8, seed=13)
    b, _ = orc.deposit(N, P.L, P.q, P.rho_bg, *parts[:3])
    sol = _fft_solve(N, P.L, b)
    _, cold = orc.pcg(N, P.L, b, np.zeros(N ** 3), 1e-10, 1000)
    _, warm = orc.pcg(N, P.L, b, sol * (1 + 1e-4), 1e-10, 1000)
    assert warm["iters"] < cold["iters"]


def test_pcg_not_converged_reports(orc):
    N = 16
    rng = np.random.default_rng(14)
    b = rng.standard_normal(N ** 3)
    b -= b.mean()
    _, info = orc.pcg(N, 1.0, b, np.zeros(N ** 3), 1e-10, 3)
    assert not info["converged"] and info["iters"] == 3 and info["true_rel_res"] > 1e-10


# ---------------------------------------------------------------- field ---

def test_efield_single_mode_closed_form(orc):
    N, L = 16, 4 * math.pi
    h = L / N
    X, Y, Z = _grid(N, L)
    k = 2 * np.pi / L * 2
    phi = np.cos(k * Y).ravel() + 3.0  # a constant offset is removed by the gauge
    p2, ex, ey, ez, wx = orc.efield(N, L, phi)
    assert abs(p2.mean()) < 1e-15
    assert np.allclose(ey, (math.sin(k * h) / h) * np.sin(k * Y).ravel(), rtol=0, atol=1e-14)
    assert np.all(np.abs(ex) < 1e-15) and np.all(np.abs(ez) < 1e-15)
    assert wx < 1e-28
    for e in (ex, ey, ez):
        assert abs(e.sum()) < 1e-12


def test_field_energy_closed_form(orc):
    """phi = cos(kx): W_x = (1/2) h^3 sum E_x^2 = (1/4) L^3 (sin(kh)/h)^2."""
    N, L = 16, 4 * math.pi
    h = L / N
    X, Y, Z = _grid(N, L)
    k = 2 * np.pi / L
    _, ex, _, _, wx = orc.efield(N, L, np.cos(k * X).ravel())
    assert math.isclose(wx, 0.25 * L ** 3 * (math.sin(k * h) / h) ** 2, rel_tol=1e-12)


def test_momentum_invariant(orc):
    """Symmetric A and the antisymmetric central gradient commute, so
    sum_i b_i E_i = sum_i r_i E_i ~ 0 for the solved phi."""
    N = 16
    P = synth.LandauParams(N=N, ppc=8)
    parts = synth.landau_particles_np(N, 8, seed=15)
    b, _ = orc.deposit(N, P.L, P.q, P.rho_bg, *parts[:3])
    phi, _ = orc.pcg(N, P.L, b, np.zeros(N ** 3), 1e-12, 5000)
    _, ex, ey, ez, _ = orc.efield(N, P.L, phi)
    for e in (ex, ey, ez):
        assert abs(b @ e) <= 1e-10 * np.linalg.norm(b) * np.linalg.norm(e)


# -------------------------------------------------------- mixed precision --

def test_mixed_precision_reaches_fp64_tolerance(orc):
    N = 32
    P = synth.LandauParams(N=N, ppc=8)
    parts = synth.landau_particles_np(N, 8, seed=16)
    b, _ = orc.deposit(N, P.L, P.q, P.rho_bg, *parts[:3])
    ref = _fft_solve(N, P.L, b)
    x, info = orc.mixed_pcg(N, P.L, b, np.zeros(N ** 3), 1e-10)
    assert info["converged"] and info["true_rel_res"] <= 1e-10
    # true residual measured independently of the oracle's operator
    r = b - _fft_apply(N, P.L, x)
    assert np.linalg.norm(r) <= 1.0001e-10 * np.linalg.norm(b)
    kappa = 3.0 / math.sin(math.pi / N) ** 2
    assert np.linalg.norm(x - ref) <= kappa * 1e-10 * np.linalg.norm(ref)
    # each refinement step contracts by about the inner tolerance (1e-3)
    assert info["outer"] <= 5


@pytest.mark.parametrize("inner_rtol", [1e-1, 1e-2])
def test_mixed_reliable_updates_keep_cg_convergence(orc, inner_rtol):
    """Reliable form: CG's recurrence continues across refinements with the
    residual replaced, so the total inner count stays near plain CG's (a wrong
    continuation coefficient costs 2-7x here), while the restarted form pays a
    fresh Krylov start per refinement; both reach the FP64 tolerance under an
    operator applied independently of the oracle (FFT)."""
    N = 32
    P = synth.LandauParams(N=N, ppc=8)
    parts = synth.landau_particles_np(N, 8, seed=17)
    b, _ = orc.deposit(N, P.L, P.q, P.rho_bg, *parts[:3])
    _, pinfo = orc.pcg(N, P.L, b, np.zeros(N ** 3), 1e-10, 20000)
    x, rel = orc.mixed_pcg(N, P.L, b, np.zeros(N ** 3), 1e-10, inner_rtol=inner_rtol,
                           reliable=True)
    _, rst = orc.mixed_pcg(N, P.L, b, np.zeros(N ** 3), 1e-10, inner_rtol=inner_rtol)
    assert rel["converged"] and rst["converged"]
    r = b - _fft_apply(N, P.L, x)
    assert np.linalg.norm(r) <= 1.0001e-10 * np.linalg.norm(b)
    assert rel["inner"] <= 1.3 * pinfo["iters"]
    assert rst["inner"] >= 1.3 * rel["inner"]
    # the refinement count is set by the inner tolerance, not by the form
    assert abs(rel["outer"] - rst["outer"]) <= 1


def test_mixed_gap_test_fires_when_fp32_drift_exceeds_inner_tolerance(orc):
    """The reliable form carries the inner direction across a refinement only
    while the refinement's true reduction is within 4x the inner solve's
    recursive one.  FP32 inner solves drift from their true residual by about
    eps32 * kappa(A) (1.9e-5 at 32^3): an inner tolerance of 1e-6 lies below
    that drift, so the test must refuse a carry; at 1e-1 (above it) it must
    never fire.  Either way the solve reaches the FP64 tolerance under an
    operator applied independently of the oracle (FFT)."""
    N = 32
    P = synth.LandauParams(N=N, ppc=8)
    parts = synth.landau_particles_np(N, 8, seed=17)
    b, _ = orc.deposit(N, P.L, P.q, P.rho_bg, *parts[:3])
    kappa = 3.0 / math.sin(math.pi / N) ** 2
    drift = float(np.finfo(np.float32).eps) * kappa
    assert 1e-6 < drift < 1e-1
    for inner_rtol, fires in ((1e-6, True), (1e-7, True), (1e-1, False), (1e-2, False)):
        x, info = orc.mixed_pcg(N, P.L, b, np.zeros(N ** 3), 1e-10, inner_rtol=inner_rtol,
                                reliable=True)
        assert info["converged"] and not info["switched"], info
        assert (info["refused"] > 0) == fires, (inner_rtol, info)
        r = b - _fft_apply(N, P.L, x)
        assert np.linalg.norm(r) <= 1.0001e-10 * np.linalg.norm(b)
    # the restarted form never carries a direction, so nothing is refused
    _, rst = orc.mixed_pcg(N, P.L, b, np.zeros(N ** 3), 1e-10, inner_rtol=1e-6)
    assert rst["converged"] and rst["refused"] == 0


def test_mixed_progress_stop_hands_over_to_fp64_pcg(orc):
    """Three refinements in a row that do not bring the FP64 true residual
    below 0.9x the best so far end the refinement loop; FP64 Jacobi-PCG then
    finishes from the current iterate.  With one inner iteration per
    refinement the loop stalls (CG's residual norm is not monotone); with an
    unattainable tolerance (1e-17, below FP64 rounding of the residual) the
    loop stops long before max_outer and the FP64 solve reports failure."""
    N = 32
    P = synth.LandauParams(N=N, ppc=8)
    parts = synth.landau_particles_np(N, 8, seed=17)
    b, _ = orc.deposit(N, P.L, P.q, P.rho_bg, *parts[:3])
    _, pinfo = orc.pcg(N, P.L, b, np.zeros(N ** 3), 1e-10, 20000)
    for reliable in (False, True):
        x, info = orc.mixed_pcg(N, P.L, b, np.zeros(N ** 3), 1e-10, inner_rtol=1e-3,
                                max_inner=1, reliable=reliable)
        assert info["switched"] and info["converged"], info
        assert info["inner"] == info["outer"] <= 10
        assert 0 < info["fp64_iters"] <= pinfo["iters"] + 10
        r = b - _fft_apply(N, P.L, x)
        assert np.linalg.norm(r) <= 1.0001e-10 * np.linalg.norm(b)
    _, info = orc.mixed_pcg(N, P.L, b, np.zeros(N ** 3), 1e-17, inner_rtol=0.1, reliable=True,
                            max_iter=300)
    assert info["switched"] and not info["converged"] and info["fp64_iters"] == 300
    assert info["outer"] < 50
    # an ordinary solve never takes the stop
    _, info = orc.mixed_pcg(N, P.L, b, np.zeros(N ** 3), 1e-10, inner_rtol=0.1, reliable=True)
    assert info["converged"] and not info["switched"] and info["fp64_iters"] == 0


def _fft_apply(N, L, u):
    h = L / N
    m = np.arange(N)
    s = (2 - 2 * np.cos(2 * np.pi * m / N)) / h ** 2
    lam = s[:, None, None] + s[None, :, None] + s[None, None, :]
    return np.real(np.fft.ifftn(np.fft.fftn(u.reshape(N, N, N)) * lam)).ravel()


# ---------------------------------------------------------- flexible CG ---

def _landau_rhs(orc, N, seed):
    P = synth.LandauParams(N=N, ppc=8)
    parts = synth.landau_particles_np(N, 8, seed=seed)
    b, _ = orc.deposit(N, P.L, P.q, P.rho_bg, *parts[:3])
    return P, b


def test_fcg_with_jacobi_matches_pcg_iterations(orc):
    N = 16
    P, b = _landau_rhs(orc, N, 17)
    c = (P.L / N) ** 2 / 6
    _, pinfo = orc.pcg(N, P.L, b, np.zeros(N ** 3), 1e-10, 5000)
    x, finfo = orc.fcg(N, P.L, b, np.zeros(N ** 3), 1e-10, 5000, lambda r: c * r)
    assert finfo["converged"] and not finfo["fell_back"]
    assert abs(finfo["iters"] - pinfo["iters"]) <= 1


def test_fcg_exact_preconditioner_one_iteration(orc):
    N = 16
    P, b = _landau_rhs(orc, N, 18)
    x, info = orc.fcg(N, P.L, b, np.zeros(N ** 3), 1e-10, 100, lambda r: _fft_solve(N, P.L, r))
    assert info["converged"] and info["iters"] == 1


@pytest.mark.parametrize("bad", ["neg", "nan", "zero", "noise"])
def test_fcg_fallback_on_bad_preconditioner(orc, bad):
    N = 16
    P, b = _landau_rhs(orc, N, 19)
    rng = np.random.default_rng(0)
    nets = {"neg": lambda r: -r, "nan": lambda r: np.full_like(r, np.nan),
            "zero": lambda r: np.zeros_like(r),
            "noise": lambda r: np.abs(rng.standard_normal(r.size)) * np.abs(r).max()}
    x, info = orc.fcg(N, P.L, b, np.zeros(N ** 3), 1e-10, 5000, nets[bad])
    assert info["converged"] and info["true_rel_res"] <= 1e-10
    if bad != "noise":
        assert info["fell_back"]


def test_single_reduction_arrangement_reproduces_textbook_pcg(orc):
    """The GPU's single-reduction arrangement of Jacobi-PCG (one set of dot
    products per iteration: r.r, gamma = r.u, delta = u.A u, sigma = u.A p,
    pi = p.A p with u = M^{-1} r; alpha = gamma / (delta + 2 beta sigma +
    beta^2 pi)), written out here with the oracle's operator, takes the same
    iterations as the oracle's textbook recurrences and reaches the same
    solution to rounding (host check of the recurrence the sweep uses)."""
    N = 16
    P = synth.LandauParams(N=N, ppc=8)
    parts = synth.landau_particles_np(N, 8, seed=77)
    b, nb = orc.deposit(N, P.L, P.q, P.rho_bg, *parts[:3])
    h = P.L / N
    minv = h * h / 6.0
    x = np.zeros(N ** 3)
    r = b.copy()
    u = minv * r
    gamma, delta = r @ u, u @ orc.apply_A(N, P.L, u)
    alpha, beta = gamma / delta, 0.0
    p = np.zeros(N ** 3)
    it = 0
    while True:
        p = minv * r + beta * p
        q = orc.apply_A(N, P.L, p)
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        if np.linalg.norm(r) <= 1e-10 * nb or it >= 5000:
            break
        u = minv * r
        g1 = r @ u
        d1, s1, p1 = u @ orc.apply_A(N, P.L, u), u @ q, p @ q
        beta = g1 / gamma
        alpha = g1 / (d1 + 2 * beta * s1 + beta * beta * p1)
        gamma = g1
    ref, info = orc.pcg(N, P.L, b, np.zeros(N ** 3), 1e-10, 5000)
    assert info["converged"] and info["replacements"] == 0
    assert it == info["iters"]
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


def test_sstep_arrangement_reproduces_textbook_pcg(orc):
    """The GPU's s-step arrangement of Jacobi-PCG (S = 3 iterations per outer
    step), written out here with the oracle's operator: the basis T_0..T_S of
    p and T_0..T_{S-1} of r, T_j Chebyshev polynomials of Ahat - I with Ahat =
    M^{-1} A; the Gram matrix from the 6S inner products the Gram sweep
    reduces (T_i T_j = (T_{i+j} + T_{|i-j|}) / 2); S CG iterations on
    coordinates, stopping on ||r|| = sqrt(z'G z') / c after each one; the new
    p, r and the x increment as combinations of the basis.  It takes the same
    iterations as the oracle's textbook recurrences and reaches the same
    solution to rounding (host check of the recurrence the two sweeps use)."""
    S = 3
    N = 16
    P = synth.LandauParams(N=N, ppc=8)
    parts = synth.landau_particles_np(N, 8, seed=78)
    b, nb = orc.deposit(N, P.L, P.q, P.rho_bg, *parts[:3])
    h = P.L / N
    c = h * h / 6.0

    def T(v, m):  # Chebyshev basis of Ahat - I applied to v, levels 0..m
        out = [v, c * orc.apply_A(N, P.L, v) - v]
        for _ in range(1, m):
            out.append(2.0 * (c * orc.apply_A(N, P.L, out[-1]) - out[-1]) - out[-2])
        return out[:m + 1]

    nv = 2 * S + 1
    B = np.zeros((nv, nv))  # Ahat on coordinates
    for b0, top in ((0, S), (S + 1, S - 1)):
        B[b0, b0] = B[b0 + 1, b0] = 1.0
        for j in range(1, top + 1):
            B[b0 + j, b0 + j] = 1.0
            B[b0 + j - 1, b0 + j] = 0.5
            if j + 1 <= top:
                B[b0 + j + 1, b0 + j] = 0.5
    x, r, p = np.zeros(N ** 3), b.copy(), c * b
    it, done = 0, False
    while not done and it < 5000:
        Y = T(p, S) + T(r, S - 1)
        # the 6S products, then the moments and the whole Gram matrix
        mp = [Y[0] @ Y[k] for k in range(S + 1)]
        mp += [2.0 * (Y[S] @ Y[j]) - mp[S - j] for j in range(1, S + 1)]
        mr = [Y[S + 1] @ Y[S + 1 + k] for k in range(S)]
        mr += [2.0 * (Y[2 * S] @ Y[S + 1 + j]) - mr[S - 1 - j] for j in range(1, S)]
        mx = [Y[0] @ Y[S + 1 + k] for k in range(S)]
        for i in range(1, S + 1):
            mx.append(2.0 * (Y[i] @ Y[2 * S]) - mx[abs(i - (S - 1))])
        G = np.empty((nv, nv))
        for i in range(nv):
            for j in range(nv):
                a, bb = min(i, j), max(i, j)
                if bb <= S:
                    G[i, j] = 0.5 * (mp[a + bb] + mp[bb - a])
                elif a > S:
                    G[i, j] = 0.5 * (mr[a + bb - 2 * S - 2] + mr[bb - a])
                else:
                    G[i, j] = 0.5 * (mx[a + bb - S - 1] + mx[abs(a - (bb - S - 1))])
        assert np.allclose(G, np.array([[u @ v for v in Y] for u in Y]), rtol=1e-12, atol=0)
        D = np.array([1.0] * (S + 1) + [c] * S)  # z-world basis: r-chain times c
        Gz = G * np.outer(D, D)
        pp, zz, xx = np.eye(nv)[0], np.eye(nv)[S + 1], np.zeros(nv)
        mu = zz @ Gz @ zz
        for _ in range(S):
            w = B @ pp
            alpha = mu / (pp @ Gz @ w)
            xx, zz = xx + alpha * pp, zz - alpha * w
            mu2 = zz @ Gz @ zz
            it += 1
            if np.sqrt(mu2) / c <= 1e-10 * nb:
                done = True
                break
            pp, mu = zz + (mu2 / mu) * pp, mu2
        x = x + sum(a * v for a, v in zip(xx * D, Y))
        r = sum(a * v for a, v in zip(zz / np.where(D == 1.0, c, 1.0), Y))
        p = sum(a * v for a, v in zip(pp * D, Y))
    ref, info = orc.pcg(N, P.L, b, np.zeros(N ** 3), 1e-10, 5000)
    assert info["converged"] and info["replacements"] == 0
    assert it == info["iters"]
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)
    assert orc.residual_norm(N, P.L, b, x) <= 1e-10 * nb * 1.0001
