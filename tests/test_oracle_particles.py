"""Pins of the oracle's particle pieces (keys, stable sort, CIC deposit, gather,
push) against facts fixed by the paper and by arithmetic -- not against the
oracle itself.  CPU only."""
import json
import math
import os

import numpy as np
import pytest

from paper_2605_05469_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_golden_setup_particle_counts():
    """Table setup_sizes / weak_scaling_setup: particles = 8 * grid points."""
    g = json.load(open(os.path.join(GOLDEN, "landau_setup.json")))
    cs = g["strong_scaling_cases"]
    for case in ("A", "B"):
        assert cs[case]["particles"] == cs["ppc"] * cs[case]["grid"] ** 3
    for row in g["weak_scaling_setup"]["rows"]:
        assert row["particles"] == 8 * int(np.prod(row["grid"]))
    assert synth.LandauParams(N=512, ppc=8).np_total == cs["A"]["particles"]
    assert abs(synth.box_length(g["landau"]["k"]) - 4 * math.pi) < 1e-15


def _tent(d, h, L):
    """Periodic CIC (tent) shape, written as max(0, 1 - |dist|/h)."""
    d = np.abs(d)
    d = np.minimum(d, L - d)
    return np.maximum(0.0, 1.0 - d / h)


# ----------------------------------------------------------------- keys ---

def test_keys_dyadic_integer_positions(orc):
    """With h = 1 (L = N), x = i + f/256 is exact, so the cell is i."""
    N = 8
    rng = np.random.default_rng(1)
    i = rng.integers(0, N, size=(3, 1000))
    f = rng.integers(0, 256, size=(3, 1000)) / 256.0
    pos = i + f
    key = orc.cell_keys(N, float(N), *pos)
    assert np.array_equal(key, ((i[2] * N + i[1]) * N + i[0]).astype(np.uint32))


def test_keys_vertex_and_edge(orc):
    N, L = 32, 4 * math.pi
    h = L / N
    x = np.array([0.0, 3 * h, np.nextafter(L, 0.0), h / 2])
    # 3*h may round to just below a vertex; the key is floor(x*N/L), clamped.
    key = orc.cell_keys(N, L, x, np.zeros(4), np.zeros(4))
    assert key[0] == 0
    assert key[2] == N - 1
    assert key[3] == 0
    assert key[1] in (2, 3)
    assert key.max() < N ** 3


# ----------------------------------------------------------------- sort ---

def test_sort_is_stable_counting_sort(orc):
    rng = np.random.default_rng(2)
    ncell = 64
    key = rng.integers(0, ncell, size=5000).astype(np.uint32)
    perm, cs = orc.sort_by_key(key, ncell)
    # a library stable sort is the same permutation (ties keep input order)
    assert np.array_equal(perm, np.argsort(key, kind="stable"))
    assert cs[0] == 0 and cs[-1] == key.size
    assert np.array_equal(cs[:-1], np.searchsorted(key[perm], np.arange(ncell)))
    # idempotent; un-permuting restores the input
    perm2, cs2 = orc.sort_by_key(key[perm], ncell)
    assert np.array_equal(perm2, np.arange(key.size)) and np.array_equal(cs2, cs)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    assert np.array_equal(key[perm][inv], key)


def test_sort_empty_and_out_of_range(orc):
    perm, cs = orc.sort_by_key(np.zeros(0, np.uint32), 8)
    assert perm.size == 0 and np.all(cs == 0)
    with pytest.raises(ValueError):
        orc.sort_by_key(np.array([9], np.uint32), 8)


# -------------------------------------------------------------- deposit ---

def test_deposit_matches_tent_function_definition(orc):
    """rho_e[v] = q/h^3 sum_p prod_d tent(x_pd - v_d h): brute force."""
    N, L = 4, 3.0
    h = L / N
    rng = np.random.default_rng(3)
    n = 37
    pos = rng.random((3, n)) * L
    q = -0.7
    b, nb, rho_e = orc.deposit(N, L, q, 0.0, *pos, want_rho_e=True)
    ref = np.zeros((N, N, N))
    for iz in range(N):
        for iy in range(N):
            for ix in range(N):
                w = (_tent(pos[0] - ix * h, h, L) * _tent(pos[1] - iy * h, h, L)
                     * _tent(pos[2] - iz * h, h, L))
                ref[iz, iy, ix] = q / h ** 3 * w.sum()
    assert np.allclose(rho_e.reshape(N, N, N), ref, rtol=1e-13, atol=1e-13 * abs(q) / h ** 3)
    # zero-mean projection and its norm
    assert abs(b.mean()) < 1e-14 * np.abs(ref).max()
    assert np.isclose(nb, np.linalg.norm(b), rtol=1e-14)


def test_deposit_single_particle_vertex_and_centre(orc):
    N, L = 8, 8.0  # h = 1
    q = 2.0
    _, _, r = orc.deposit(N, L, q, 0.0, [3.0], [5.0], [1.0], want_rho_e=True)
    r = r.reshape(N, N, N)
    assert r[1, 5, 3] == q and np.count_nonzero(r) == 1
    _, _, r = orc.deposit(N, L, q, 0.0, [7.5], [0.5], [3.5], want_rho_e=True)
    r = r.reshape(N, N, N)
    nz = np.argwhere(r)
    assert len(nz) == 8 and np.all(r[r != 0] == q / 8)
    assert {tuple(v) for v in nz} == {(z, y, x) for z in (3, 4) for y in (0, 1) for x in (7, 0)}


def test_deposit_charge_conservation(orc):
    # random positions: h^3 sum rho_e = q Np to rounding
    N = 16
    P = synth.LandauParams(N=N, ppc=8)
    parts = synth.landau_particles_np(N, 8, seed=5)
    _, _, re = orc.deposit(N, P.L, P.q, P.rho_bg, *parts[:3], want_rho_e=True)
    h = P.L / N
    total = re.sum() * h ** 3
    assert abs(total - P.q * P.np_total) <= 1e-13 * abs(P.q * P.np_total)
    # dyadic positions (h = 1/4, offsets multiples of h/256): exact conservation
    N, L = 8, 2.0
    rng = np.random.default_rng(6)
    pos = rng.integers(0, N * 256, size=(3, 4096)) / (256.0 * N / L)
    _, _, re = orc.deposit(N, L, 1.0, 0.0, *pos, want_rho_e=True)
    assert re.sum() * (L / N) ** 3 == 4096.0


def test_deposit_lattice_loading_is_uniform(orc):
    N = 8
    P = synth.LandauParams(N=N, ppc=1)
    h = P.L / N
    c = (np.arange(N) + 0.5) * h
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    b, nb, re = orc.deposit(N, P.L, P.q, P.rho_bg, x.ravel(), y.ravel(), z.ravel(), want_rho_e=True)
    assert np.allclose(re, -1.0, rtol=1e-13)
    assert nb < 1e-12


def test_deposit_gather_adjoint(orc):
    """sum_v rho_e[v] F[v] h^3 == sum_p q * gather(F)(x_p): same CIC shape."""
    N = 8
    P = synth.LandauParams(N=N, ppc=4)
    parts = synth.landau_particles_np(N, 4, seed=7)
    _, _, re = orc.deposit(N, P.L, P.q, 0.0, *parts[:3], want_rho_e=True)
    F = np.random.default_rng(8).standard_normal(N ** 3)
    lhs = (re * F).sum() * (P.L / N) ** 3
    rhs = P.q * orc.gather_scalar(N, P.L, *parts[:3], F).sum()
    assert abs(lhs - rhs) <= 1e-12 * np.abs(re * F).sum() * (P.L / N) ** 3


# -------------------------------------------------------- gather + push ---

def test_gather_matches_tent_definition(orc):
    N, L = 4, 5.0
    h = L / N
    rng = np.random.default_rng(9)
    pos = rng.random((3, 50)) * L
    F = rng.standard_normal((N, N, N))
    got = orc.gather_scalar(N, L, *pos, F.ravel())
    ref = np.zeros(50)
    for iz in range(N):
        for iy in range(N):
            for ix in range(N):
                ref += F[iz, iy, ix] * (_tent(pos[0] - ix * h, h, L) * _tent(pos[1] - iy * h, h, L)
                                        * _tent(pos[2] - iz * h, h, L))
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)


def test_push_free_streaming(orc):
    N, L, dt = 8, 10.0, 0.05
    rng = np.random.default_rng(10)
    x = rng.random((3, 200)) * L
    v = rng.standard_normal((3, 200)) * 3
    zero = np.zeros(N ** 3)
    out = orc.gather_push(N, L, dt, -1.0, *x, *v, zero, zero, zero)
    for d in range(3):
        assert np.array_equal(out[3 + d], v[d])
        assert np.allclose(out[d], np.mod(x[d] + dt * v[d], L), rtol=0, atol=1e-12)
        assert np.all((out[d] >= 0) & (out[d] < L))
    assert np.array_equal(out[6], orc.cell_keys(N, L, *out[:3]))


def test_push_uniform_field_parabola(orc):
    """Uniform E: v_n = v0 + n dt qm E, x_n = x0 + n dt v0 + dt^2 qm E n(n+1)/2."""
    N, L, dt, qm = 8, 1000.0, 0.1, -1.0
    E = 0.3
    x0 = np.array([400.0, 500.0]); v0 = np.array([0.25, -1.0])
    ex = np.full(N ** 3, E); zero = np.zeros(N ** 3)
    st = [x0.copy(), np.full(2, 100.0), np.full(2, 100.0), v0.copy(), np.zeros(2), np.zeros(2)]
    n = 40
    for _ in range(n):
        st = list(orc.gather_push(N, L, dt, qm, *st, ex, zero, zero)[:6])
    assert np.allclose(st[3], v0 + n * dt * qm * E, rtol=1e-12)
    assert np.allclose(st[0], x0 + n * dt * v0 + dt * dt * qm * E * n * (n + 1) / 2, rtol=1e-11)


def test_wrap_edge_cases(orc):
    """A tiny negative coordinate wraps to 0, never to L; x = L - tiny stays in the box."""
    N, L = 4, 2.0
    zero = np.zeros(N ** 3)
    x = np.array([1e-30, np.nextafter(L, 0.0)])
    v = np.array([-1e-10, 0.0])
    out = orc.gather_push(N, L, 1e-20, -1.0, x, x.copy(), x.copy(), v, v.copy(), v.copy(),
                          zero, zero, zero)
    for d in range(3):
        assert np.all((out[d] >= 0.0) & (out[d] < L))
    assert out[6][1] == (N - 1) * (N * N + N + 1)


def test_cold_plasma_oscillation_frequency(orc):
    """Cold plasma, small displacement delta*sin(kx): the leapfrog frequency obeys
    sin(w dt/2) = (dt/2) w_g with w_g -> w_p = 1 as kh -> 0 (kh ~ 0.2; 1%)."""
    N, k, dt = 32, 0.5, 0.05
    L = 2 * math.pi / k
    g = (np.arange(2 * N) + 0.5) * (L / (2 * N))
    Xg, Yg, Zg = np.meshgrid(g, g, g, indexing="ij")
    X, Y, Z = Xg.ravel(), Yg.ravel(), Zg.ravel()
    X = np.mod(X + 1e-3 * np.sin(k * X), L)
    npart = X.size
    st = orc.State(N, L, -(L ** 3) / npart, -1.0, dt, X, Y, Z,
                   np.zeros(npart), np.zeros(npart), np.zeros(npart))
    st.init(1e-12, 5000)

    def amp():
        return np.fft.fftn(st.ex.reshape(N, N, N))[0, 0, 1].imag

    # E at integer steps; the half-kick start keeps the phase at t = 0
    s = [amp()]
    for _ in range(280):
        st.step(1e-12, 5000)
        s.append(amp())
    s = np.array(s)
    t = np.arange(len(s)) * dt
    zc = [t[i] - s[i] * dt / (s[i + 1] - s[i]) for i in range(len(s) - 1)
          if s[i] != 0 and np.sign(s[i]) != np.sign(s[i + 1])]
    half = (zc[-1] - zc[0]) / (len(zc) - 1)
    w = math.pi / half
    w_theory = 2.0 / dt * math.asin(dt / 2 * 1.0)
    assert len(zc) >= 4
    assert abs(w - w_theory) / w_theory < 0.01


def test_deposit_vertices_matches_full_deposit(orc):
    N = 8
    P = synth.LandauParams(N=N, ppc=4)
    parts = synth.landau_particles_np(N, 4, seed=21)
    _, _, re = orc.deposit(N, P.L, P.q, 0.0, *parts[:3], want_rho_e=True)
    vid = np.array([0, 7, 63, 64, 200, N ** 3 - 1])
    got = orc.deposit_vertices(N, P.L, P.q, *parts[:3], vid)
    assert np.allclose(got, re[vid], rtol=1e-13, atol=1e-13 * np.abs(re).max())


def test_deposit_order_bound_holds_and_is_tight(orc):
    """The association bound used to compare two deposits that add the same
    terms in different orders: an unsorted and a sorted oracle deposit of the
    same particles stay within it, and dropping one particle (a deposit that
    is wrong by a single weight) breaks it."""
    from deposit_bound import check_deposit
    N, ppc = 32, 8
    P = synth.LandauParams(N=N, ppc=ppc)
    parts = synth.landau_particles_np(N, ppc, seed=41)
    keys = orc.cell_keys(N, P.L, *parts[:3])
    perm, cs = orc.sort_by_key(keys, N ** 3)
    xs = [a[perm] for a in parts[:3]]
    b_sorted, _, rho_e = orc.deposit(N, P.L, P.q, P.rho_bg, *xs, want_rho_e=True)
    rng = np.random.default_rng(2)
    shuf = rng.permutation(xs[0].size)
    b_shuf, _ = orc.deposit(N, P.L, P.q, P.rho_bg, *[a[shuf] for a in xs])
    assert not np.array_equal(b_shuf, b_sorted)  # the order does change bits
    check_deposit(N, b_shuf, b_sorted, rho_e, P.rho_bg, np.diff(cs))
    b_drop, _ = orc.deposit(N, P.L, P.q, P.rho_bg, *[a[1:] for a in xs])
    with pytest.raises(AssertionError):
        check_deposit(N, b_drop, b_sorted, rho_e, P.rho_bg, np.diff(cs))
