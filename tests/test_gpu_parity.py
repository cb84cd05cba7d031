"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle, on
identical seeded inputs.  Integer and per-particle results bit-exact; field
results within the tolerances stated at each test."""
import math

import numpy as np
import pytest

from paper_2605_05469_amd import synth
from deposit_bound import check_deposit

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def pic():
    import paper_2605_05469_amd as P
    P.lib()
    return P


def _ctx(pic, N, ppc=8, np_max=None, **kw):
    p = pic.landau_params(N, ppc, np_max=np_max, **kw)
    return pic.Context(p), p


def _landau(N, ppc, seed, n=None):
    return synth.landau_particles_np(N, ppc, seed=seed, np_total=n)


# ---------------------------------------------------------------- keys ----

@pytest.mark.parametrize("N,ppc", [(32, 8), (64, 1), (96, 2)])
def test_keys_bit_exact(pic, orc, N, ppc):
    ctx, p = _ctx(pic, N, ppc)
    parts = _landau(N, ppc, 1000 + N)
    # add exact vertex positions and the last representable value below L
    h = p.length / N
    parts[0][:4] = [0.0, 3 * h, np.nextafter(p.length, 0.0), h]
    xs = [_dev(a) for a in parts[:3]]
    key = torch.empty(xs[0].numel(), dtype=torch.int32, device="cuda")
    ctx.cell_keys(*xs, key)
    ref = orc.cell_keys(N, p.length, *parts[:3])
    assert np.array_equal(_host(key).view(np.uint32), ref)


# ------------------------------------------------------------ gather/push --

def _random_field(N, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(N ** 3) for _ in range(3)]


@pytest.mark.parametrize("N,ppc,ragged", [(32, 8, 0), (64, 2, 777)])
def test_gather_push_bit_exact(pic, orc, N, ppc, ragged):
    n = ppc * N ** 3 - ragged
    ctx, p = _ctx(pic, N, ppc)
    parts = list(_landau(N, ppc, 2000 + N, n=n))
    parts[3][:3] = [1e3, -1e3, 0.0]  # particles that cross the box edge in one step
    parts[0][:3] = [0.0, p.length - 1e-13, 1e-300]
    E = _random_field(N, 5)
    d = [_dev(a) for a in parts]
    dE = [_dev(a) for a in E]
    key = torch.empty(n, dtype=torch.int32, device="cuda")
    ctx.gather_push(*d, *dE, key)
    ref = orc.gather_push(N, p.length, p.dt, p.qm, *parts, *E)
    for k in range(6):
        assert np.array_equal(_host(d[k]), ref[k]), k
    assert np.array_equal(_host(key).view(np.uint32), ref[6])


def test_half_kick_bit_exact(pic, orc):
    N, ppc = 32, 4
    ctx, p = _ctx(pic, N, ppc)
    parts = _landau(N, ppc, 3000)
    E = _random_field(N, 6)
    d = [_dev(a) for a in parts]
    ctx.half_kick(*d, *[_dev(a) for a in E])
    ref = orc.half_kick(N, p.length, p.dt, p.qm, *parts, *E)
    for k in range(3):
        assert np.array_equal(_host(d[3 + k]), ref[k])
        assert np.array_equal(_host(d[k]), parts[k])


def test_empty_particle_set(pic):
    ctx, p = _ctx(pic, 32, 1)
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    f = torch.zeros(32 ** 3, dtype=torch.float64, device="cuda")
    ctx.gather_push(e, e, e, e, e, e, f, f, f, None)
    rho = torch.empty(32 ** 3, dtype=torch.float64, device="cuda")
    cs = torch.empty(32 ** 3 + 1, dtype=torch.int32, device="cuda")
    ctx.sort_cells(torch.empty(0, dtype=torch.int32, device="cuda"), [e] * 6,
                   [torch.empty(0, dtype=torch.float64, device="cuda") for _ in range(6)], cs)
    assert np.all(_host(cs) == 0)
    nb = ctx.deposit(None, None, None, None, rho, want_norm=True)
    assert nb == 0.0 and np.all(_host(rho) == 0.0)


# ---------------------------------------------------------------- sort ----

def _sort_case(pic, orc, N, keys_np):
    n = keys_np.size
    ctx, p = _ctx(pic, N, 1, np_max=max(n, 1))
    rng = np.random.default_rng(n)
    src = [rng.standard_normal(n) for _ in range(6)]
    key = _dev(keys_np.astype(np.uint32).view(np.int32))
    ds = [_dev(a) for a in src]
    dd = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(6)]
    cs = torch.empty(N ** 3 + 1, dtype=torch.int32, device="cuda")
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    ctx.sort_cells(key, ds, dd, cs, perm)
    rperm, rcs = orc.sort_by_key(keys_np.astype(np.uint32), N ** 3)
    assert np.array_equal(_host(perm).view(np.uint32).astype(np.int64), rperm)
    assert np.array_equal(_host(cs).view(np.uint32).astype(np.int64), rcs)
    for k in range(6):
        assert np.array_equal(_host(dd[k]), src[k][rperm])


def test_sort_landau_keys_bit_exact(pic, orc):
    N, ppc = 32, 8
    parts = _landau(N, ppc, 4000)
    keys = orc.cell_keys(N, synth.box_length(), *parts[:3])
    _sort_case(pic, orc, N, keys)


@pytest.mark.parametrize("case", ["ragged", "ties", "reverse", "one", "sorted"])
def test_sort_edge_cases(pic, orc, case):
    N = 32
    rng = np.random.default_rng(7)
    n = {"ragged": 4096 * 3 + 1234, "ties": 20000, "reverse": 9000, "one": 1, "sorted": 5000}[case]
    if case == "ragged":
        keys = rng.integers(0, N ** 3, n)
    elif case == "ties":
        keys = rng.integers(0, 3, n) * 1000 + N ** 3 - 3001
    elif case == "reverse":
        keys = np.arange(n)[::-1] % N ** 3
    elif case == "one":
        keys = np.array([N ** 3 - 1])
    else:
        keys = np.sort(rng.integers(0, N ** 3, n))
    _sort_case(pic, orc, N, np.asarray(keys))


@pytest.mark.parametrize("N,kind", [(64, "near"), (64, "random"), (128, "near"), (128, "random")])
def test_sort_multi_tile(pic, orc, N, kind):
    """Several 12288-key tiles and a ragged last one; 18-bit keys (two 9-bit
    passes) at 64^3, 21-bit keys (three 7-bit passes) at 128^3; keys either
    uniform or the near-sorted keys of a cell-sorted state whose particles
    moved a few cells (the PIC step's case), so runs of equal digits are long
    and ties are many."""
    rng = np.random.default_rng(N + len(kind))
    n = 5 * 12288 + 777
    if kind == "random":
        keys = rng.integers(0, N ** 3, n)
    else:
        c = np.sort(rng.integers(0, N ** 3, n))
        iz, iy, ix = c // (N * N), (c // N) % N, c % N
        d = np.rint(rng.standard_normal((3, n)) * 2).astype(np.int64)
        keys = (((iz + d[0]) % N) * N + (iy + d[1]) % N) * N + (ix + d[2]) % N
    _sort_case(pic, orc, N, np.asarray(keys))


# ------------------------------------------------------------- deposit ----

@pytest.mark.parametrize("N,ppc", [(32, 8), (64, 3)])
def test_deposit_sorted_and_atomic(pic, orc, N, ppc):
    ctx, p = _ctx(pic, N, ppc)
    parts = _landau(N, ppc, 5000 + N)
    keys = orc.cell_keys(N, p.length, *parts[:3])
    perm, cs = orc.sort_by_key(keys, N ** 3)
    xs = [a[perm] for a in parts[:3]]
    ref_b, ref_nb, rho_e = orc.deposit(N, p.length, p.charge, p.rho_bg, *xs, want_rho_e=True)
    d = [_dev(a) for a in xs]
    rho = torch.empty(N ** 3, dtype=torch.float64, device="cuda")
    nb = ctx.deposit(*d, _dev(cs.astype(np.uint32).view(np.int32)), rho, want_norm=True)
    got = _host(rho)
    scale = np.abs(ref_b).max()
    # same terms, summed per cell, per cell row and per vertex (GPU) instead
    # of sequentially over the sorted particles (oracle): within the
    # association bound of every vertex
    check_deposit(N, got, ref_b, rho_e, p.rho_bg, np.diff(cs))
    assert np.max(np.abs(got - ref_b)) <= 1e-13 * scale
    assert abs(nb - ref_nb) <= 1e-12 * ref_nb
    # unsorted path (atomics): same values up to summation order
    rng = np.random.default_rng(1)
    shuf = rng.permutation(xs[0].size)
    d2 = [_dev(a[shuf]) for a in xs]
    ctx.deposit(*d2, None, rho)
    assert np.max(np.abs(_host(rho) - ref_b)) <= 1e-12 * scale


def test_deposit_charge_conservation_dyadic(pic, orc):
    """Positions on multiples of h/256 with h a power of two: the weight sums
    are exact, so total charge is conserved bit for bit."""
    N = 32
    L = 8.0  # h = 1/4
    p = pic.landau_params(N, 4)
    p.length = L
    p.charge = 1.0
    p.rho_bg = 0.0
    ctx = pic.Context(p)
    rng = np.random.default_rng(3)
    n = 4 * N ** 3
    pos = [rng.integers(0, N * 256, n) / (256.0 * N / L) for _ in range(3)]
    keys = orc.cell_keys(N, L, *pos)
    perm, cs = orc.sort_by_key(keys, N ** 3)
    rho = torch.empty(N ** 3, dtype=torch.float64, device="cuda")
    ctx.deposit(*[_dev(a[perm]) for a in pos], _dev(cs.astype(np.uint32).view(np.int32)), rho)
    got = _host(rho)
    h = L / N
    ref_b, _, re = orc.deposit(N, L, 1.0, 0.0, *[a[perm] for a in pos], want_rho_e=True)
    assert re.sum() * h ** 3 == n
    # every sum is exact here, in any order, so the projected field is bit-exact
    assert np.array_equal(got, ref_b)


# --------------------------------------------------------------- solve ----

def _rhs(orc, N, ppc, seed):
    L = synth.box_length()
    P = synth.LandauParams(N=N, ppc=ppc)
    parts = _landau(N, ppc, seed)
    b, nb = orc.deposit(N, L, P.q, P.rho_bg, *parts[:3])
    return b


def _pcg_flags(pic, form):
    return {"single": pic.FLAG_PCG_SINGLE_SWEEP, "two_sweep": pic.FLAG_PCG_TWO_SWEEP,
            "sstep": 0}[form]


@pytest.mark.parametrize("form", ["sstep", "single", "two_sweep"])
@pytest.mark.parametrize("N", [32, 64, 96, 128])
def test_pcg_fp64_parity(pic, orc, N, form):
    """Every arrangement of Jacobi-PCG on the GPU (the s-step form's Gram and
    update sweeps on 32 x 32 tiles, the default; the single-reduction sweep,
    64- and 32-wide tiles; the direction + update pair) against the oracle's
    textbook recurrences.  At 128^3 the 64 x 32 tiles of the single-reduction sweep
    (the 512^3 launch shape) sit two to a row, so halos cross tiles in x and
    y; the s-step tiles sit four to a row.  When the two sides stop one
    iteration apart (dot products summed in another order), the side that
    ran longer is run again with the other's count, so the iterates are
    always compared after the same number of iterations."""
    flags = _pcg_flags(pic, form)
    ctx, p = _ctx(pic, N, 8, np_max=0, check_every=8, flags=flags)
    b = _rhs(orc, N, 8, 6000 + N)
    x0 = np.zeros(N ** 3)
    db, dx = _dev(b), _dev(x0)
    info = ctx.poisson(db, dx)
    ref, rinfo = orc.pcg(N, p.length, b, x0, p.rtol, p.max_iter)
    assert info["converged"] and rinfo["converged"]
    assert abs(info["iterations"] - rinfo["iters"]) <= 1
    got = _host(dx)
    # true residual under the oracle's operator
    assert orc.residual_norm(N, p.length, b, got) <= p.rtol * np.linalg.norm(b)
    m = min(info["iterations"], rinfo["iters"])
    if rinfo["iters"] > m:
        ref, rinfo = orc.pcg(N, p.length, b, x0, p.rtol, m)
        assert rinfo["iters"] == m
    elif info["iterations"] > m:
        ctx_m, _ = _ctx(pic, N, 8, np_max=0, check_every=8, flags=flags, max_iter=m)
        dx = _dev(x0)
        info_m = ctx_m.poisson(db, dx)
        assert info_m["iterations"] == m
        got = _host(dx)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("form", ["sstep", "single"])
def test_pcg_warm_start_and_zero_rhs(pic, orc, form):
    N = 32
    ctx, p = _ctx(pic, N, 8, np_max=0, flags=_pcg_flags(pic, form))
    b = _rhs(orc, N, 8, 6100)
    ref, _ = orc.pcg(N, p.length, b, np.zeros(N ** 3), 1e-12, 20000)
    dx = _dev(ref)
    info = ctx.poisson(_dev(b), dx)
    assert info["iterations"] == 0 and info["converged"]
    z = torch.zeros(N ** 3, dtype=torch.float64, device="cuda")
    dx = _dev(np.ones(N ** 3))
    info = ctx.poisson(z, dx)
    assert info["converged"] and info["iterations"] == 0 and np.all(_host(dx) == 0)


@pytest.mark.parametrize("form", ["sstep", "single"])
def test_pcg_not_converged_status(pic, orc, form):
    """The iteration cap ends the solve at exactly max_iter iterations (five:
    inside the s-step form's second outer step)."""
    N = 32
    ctx, p = _ctx(pic, N, 8, np_max=0, max_iter=5, check_every=4, flags=_pcg_flags(pic, form))
    b = _rhs(orc, N, 8, 6200)
    dx = torch.zeros(N ** 3, dtype=torch.float64, device="cuda")
    info = ctx.poisson(_dev(b), dx)
    assert info["status"] == 1 and not info["converged"] and info["iterations"] == 5
    ref, rinfo = orc.pcg(N, p.length, b, np.zeros(N ** 3), p.rtol, 5)
    assert np.linalg.norm(_host(dx) - ref) <= 1e-13 * np.linalg.norm(ref)
    assert abs(info["rel_res"] - rinfo["true_rel_res"]) <= 1e-10 * rinfo["true_rel_res"]
    # an unattainable tolerance: the iterations go on at the rounding floor
    # (directions whose curvature is lost to cancellation restart) until the
    # cap, which ends the solve with PIC_NOT_CONVERGED; the iterate stays a
    # solution to the usual tolerance (up to a constant, A's null space,
    # which the field's gauge fix removes)
    ctx2, p2 = _ctx(pic, N, 8, np_max=0, max_iter=400, rtol=1e-17, flags=_pcg_flags(pic, form))
    dx = torch.zeros(N ** 3, dtype=torch.float64, device="cuda")
    info = ctx2.poisson(_dev(b), dx)
    assert info["status"] == 1 and not info["converged"] and info["iterations"] == 400, info
    assert orc.residual_norm(N, p.length, b, _host(dx)) <= 1e-10 * np.linalg.norm(b)


def test_efield_parity(pic, orc):
    N = 64
    ctx, p = _ctx(pic, N, 8, np_max=0)
    rng = np.random.default_rng(8)
    phi = rng.standard_normal(N ** 3) + 0.3
    dphi = _dev(phi)
    E = [torch.empty(N ** 3, dtype=torch.float64, device="cuda") for _ in range(3)]
    wx = ctx.efield(dphi, *E)
    rphi, rex, rey, rez, rwx = orc.efield(N, p.length, phi)
    # the mean is summed in a different order: phi agrees to its rounding
    assert np.max(np.abs(_host(dphi) - rphi)) <= 1e-13 * np.abs(rphi).max()
    for g, r in zip(E, (rex, rey, rez)):
        assert np.max(np.abs(_host(g) - r)) <= 1e-13 * np.abs(r).max()
    assert abs(wx - rwx) <= 1e-12 * rwx


def test_mixed_precision_reaches_tolerance(pic, orc):
    N = 64
    ctx, p = _ctx(pic, N, 8, np_max=0, solver="pcg_mixed")
    b = _rhs(orc, N, 8, 6300)
    dx = torch.zeros(N ** 3, dtype=torch.float64, device="cuda")
    info = ctx.poisson(_dev(b), dx)
    assert info["converged"] and info["outer_iterations"] >= 2, info
    got = _host(dx)
    assert orc.residual_norm(N, p.length, b, got) <= p.rtol * np.linalg.norm(b)
    ref, rinfo = orc.pcg(N, p.length, b, np.zeros(N ** 3), 1e-13, 20000)
    kappa = 3.0 / math.sin(math.pi / N) ** 2
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err <= kappa * p.rtol
    # the same refinement in the oracle takes the same number of outer steps
    mref, minfo = orc.mixed_pcg(N, p.length, b, np.zeros(N ** 3), p.rtol,
                                inner_rtol=p.inner_rtol, max_inner=p.max_inner)
    assert minfo["outer"] == info["outer_iterations"]
    assert abs(minfo["inner"] - info["iterations"]) <= 2 * info["outer_iterations"]


@pytest.mark.parametrize("N,inner_rtol", [(64, 1e-1), (96, 1e-2), (128, 1e-1)])
def test_mixed_reliable_matches_oracle(pic, orc, N, inner_rtol):
    """Reliable updates: the inner direction carries over between refinements;
    same refinement count as the oracle, inner count within a few per step."""
    ctx, p = _ctx(pic, N, 8, np_max=0, solver="pcg_mixed", inner_rtol=inner_rtol)
    ctx.set_flags(pic.FLAG_MIXED_RELIABLE)
    b = _rhs(orc, N, 8, 6400 + N)
    dx = torch.zeros(N ** 3, dtype=torch.float64, device="cuda")
    info = ctx.poisson(_dev(b), dx)
    assert info["converged"], info
    assert orc.residual_norm(N, p.length, b, _host(dx)) <= p.rtol * np.linalg.norm(b)
    _, minfo = orc.mixed_pcg(N, p.length, b, np.zeros(N ** 3), p.rtol, inner_rtol=inner_rtol,
                             max_inner=p.max_inner, reliable=True)
    assert minfo["converged"]
    assert abs(minfo["outer"] - info["outer_iterations"]) <= 1
    assert abs(minfo["inner"] - info["iterations"]) <= 3 * info["outer_iterations"] + 2
    _, pinfo = orc.pcg(N, p.length, b, np.zeros(N ** 3), p.rtol, p.max_iter)
    assert info["iterations"] <= 1.3 * pinfo["iters"]


@pytest.mark.parametrize("N,inner_rtol,fires", [(32, 1e-6, True), (64, 1e-6, True),
                                                (32, 1e-1, False), (64, 1e-1, False)])
def test_mixed_gap_restarts_match_oracle(pic, orc, N, inner_rtol, fires):
    """The residual-gap test of the reliable form: it refuses to carry the
    inner direction when the FP32 drift (eps32 kappa) exceeds the inner
    tolerance, on the GPU as in the oracle, and never at a loose tolerance."""
    ctx, p = _ctx(pic, N, 8, np_max=0, solver="pcg_mixed", inner_rtol=inner_rtol,
                  flags=pic.FLAG_MIXED_RELIABLE)
    b = _rhs(orc, N, 8, 6700 + N)
    dx = torch.zeros(N ** 3, dtype=torch.float64, device="cuda")
    info = ctx.poisson(_dev(b), dx)
    assert info["converged"] and not info["fell_back"], info
    assert orc.residual_norm(N, p.length, b, _host(dx)) <= p.rtol * np.linalg.norm(b)
    _, minfo = orc.mixed_pcg(N, p.length, b, np.zeros(N ** 3), p.rtol, inner_rtol=inner_rtol,
                             max_inner=p.max_inner, reliable=True)
    assert minfo["converged"] and not minfo["switched"]
    assert (info["gap_restarts"] > 0) == fires == (minfo["refused"] > 0), (info, minfo)
    assert abs(info["gap_restarts"] - minfo["refused"]) <= 1
    assert abs(minfo["outer"] - info["outer_iterations"]) <= 1


@pytest.mark.parametrize("reliable", [False, True])
def test_mixed_progress_stop_matches_oracle(pic, orc, reliable):
    """One inner iteration per refinement stalls the refinement loop; after
    three refinements without progress FP64 Jacobi-PCG finishes the solve, on
    the GPU as in the oracle.  An unattainable tolerance ends in
    PIC_NOT_CONVERGED after max_iter FP64 iterations, not after max_outer
    refinements of max_inner inner iterations."""
    N = 32
    flags = pic.FLAG_MIXED_RELIABLE if reliable else 0
    ctx, p = _ctx(pic, N, 8, np_max=0, solver="pcg_mixed", inner_rtol=1e-3, max_inner=1,
                  flags=flags)
    b = _rhs(orc, N, 8, 6800)
    dx = torch.zeros(N ** 3, dtype=torch.float64, device="cuda")
    info = ctx.poisson(_dev(b), dx)
    assert info["converged"] and info["fell_back"], info
    assert orc.residual_norm(N, p.length, b, _host(dx)) <= p.rtol * np.linalg.norm(b)
    _, minfo = orc.mixed_pcg(N, p.length, b, np.zeros(N ** 3), p.rtol, inner_rtol=1e-3,
                             max_inner=1, reliable=reliable)
    assert minfo["switched"] and minfo["converged"]
    assert info["outer_iterations"] == minfo["outer"]
    assert abs(info["fp64_iterations"] - minfo["fp64_iters"]) <= 1
    assert info["iterations"] == info["outer_iterations"] + info["fp64_iterations"]
    ctx2, p2 = _ctx(pic, N, 8, np_max=0, solver="pcg_mixed", inner_rtol=0.1, rtol=1e-17,
                    max_iter=300, flags=pic.FLAG_MIXED_RELIABLE)
    dx = torch.zeros(N ** 3, dtype=torch.float64, device="cuda")
    info = ctx2.poisson(_dev(b), dx)
    assert info["status"] == 1 and not info["converged"] and info["fell_back"], info
    assert info["fp64_iterations"] == 300 and info["outer_iterations"] < 50


@pytest.mark.parametrize("unfused", [False, True])
@pytest.mark.parametrize("N,inner,outer", [(32, 4, 2), (64, 4, 2), (64, 2, 1), (96, 3, 2),
                                           (64, 1, 3)])
def test_pcg_ssor_matches_oracle(pic, orc, N, inner, outer, unfused):
    """The paper's SSOR preconditioner (Sec. 4.1) inside FP64 PCG: same
    iteration count as the oracle (dot-product order only), true residual;
    triangular solves fused into one z-march each, or one sweep per step."""
    ctx, p = _ctx(pic, N, 8, np_max=0, solver="pcg_ssor", ssor_inner=inner, ssor_outer=outer,
                  flags=pic.FLAG_SSOR_UNFUSED if unfused else 0)
    b = _rhs(orc, N, 8, 6500 + N)
    dx = torch.zeros(N ** 3, dtype=torch.float64, device="cuda")
    info = ctx.poisson(_dev(b), dx)
    ref, rinfo = orc.pcg_ssor(N, p.length, b, np.zeros(N ** 3), p.rtol, p.max_iter,
                              math.pi / 2, inner, outer)
    assert info["converged"] and rinfo["converged"]
    assert abs(info["iterations"] - rinfo["iters"]) <= 1
    got = _host(dx)
    assert orc.residual_norm(N, p.length, b, got) <= p.rtol * np.linalg.norm(b)
    if info["iterations"] == rinfo["iters"]:
        assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("N", [64, 128])
def test_ssor_fused_equals_unfused(pic, orc, N):
    """The fused triangular solves compute the same z as the per-step sweeps
    (same operations in the same order); only r . z is reduced in another
    block order, so the two solves agree to rounding of the dot products."""
    b = _dev(_rhs(orc, N, 8, 6600 + N))
    res = []
    for flags in (0, pic.FLAG_SSOR_UNFUSED):
        ctx, p = _ctx(pic, N, 8, np_max=0, solver="pcg_ssor", flags=flags)
        dx = torch.zeros(N ** 3, dtype=torch.float64, device="cuda")
        info = ctx.poisson(b, dx)
        assert info["converged"]
        res.append((info["iterations"], _host(dx)))
    assert abs(res[0][0] - res[1][0]) <= 1
    if res[0][0] == res[1][0]:
        assert np.linalg.norm(res[0][1] - res[1][1]) <= 1e-11 * np.linalg.norm(res[1][1])


# ------------------------------------------------------------ full step ----

def test_step_parity_config0(pic, orc):
    """32^3, 8 ppc, dt 0.05, 20 steps (the small Landau configuration):
    the GPU run and the oracle run from the same bits stay together."""
    N, ppc, nsteps = 32, 8, 20
    p = pic.landau_params(N, ppc)
    ctx = pic.Context(p)
    parts = _landau(N, ppc, 20260)
    sim = pic.Simulation(ctx, *[_dev(a) for a in parts])
    st = orc.State(N, p.length, p.charge, p.qm, p.dt, *parts)
    gi = sim.init()
    oi = st.init(p.rtol, p.max_iter)
    assert abs(gi["iterations"] - oi["iters"]) <= 1
    key_mismatch = 0
    for s in range(nsteps):
        g = sim.step()
        o = st.step(p.rtol, p.max_iter)
        assert g["converged"] and o["converged"]
        assert abs(g["iterations"] - o["iters"]) <= 1
        assert abs(g["wx"] - st.wx) <= 1e-9 * st.wx
    x = _host(sim.particles[0])
    assert np.max(np.abs(x - st.x)) <= 1e-9 * p.length
    gk = orc.cell_keys(N, p.length, *[_host(a) for a in sim.particles[:3]])
    ok = orc.cell_keys(N, p.length, st.x, st.y, st.z)
    key_mismatch = int(np.count_nonzero(gk != ok))
    assert key_mismatch == 0
    phi = _host(sim.phi)
    assert np.linalg.norm(phi - st.phi) <= 1e-9 * np.linalg.norm(st.phi)


def test_mixed_form_error_vs_fp64_oracle(pic, orc):
    """The mixed form (FP32 inner solves inside FP64 refinement, reliable
    updates) driving the PIC loop beside the FP64 oracle from the same
    particles, 64^3 x 8 ppc, 6 steps.  Both solves stop at relative residual
    1e-10, so their solutions may differ by up to ||A^+|| (||r_m|| + ||r_o||):
    relative to ||phi|| at most 2 kappa rtol, kappa = 3 / sin^2(pi/N).  The
    field differs by at most ||grad_h|| <= sqrt(3)/h times the potential's
    difference, and the leapfrog carries the gathered field's difference
    into positions as dt^2 |q/m| summed twice over the steps (doubled for
    the gather at displaced positions).  The errors are printed and held to
    these bounds; keys stay identical."""
    N, ppc, nsteps = 64, 8, 6
    p = pic.landau_params(N, ppc, solver="pcg_mixed", inner_rtol=0.1,
                          flags=pic.FLAG_MIXED_RELIABLE)
    ctx = pic.Context(p)
    parts = _landau(N, ppc, 20300)
    sim = pic.Simulation(ctx, *[_dev(a) for a in parts])
    st = orc.State(N, p.length, p.charge, p.qm, p.dt, *parts)
    gi = sim.init()
    st.init(p.rtol, p.max_iter)
    assert gi["converged"]
    h = p.length / N
    kappa = 3.0 / math.sin(math.pi / N) ** 2
    bound_phi = 2.0 * kappa * p.rtol
    dx_bound, dv_bound = 0.0, 0.0
    errs = []
    for s in range(nsteps + 1):
        if s > 0:
            g = sim.step()
            st.step(p.rtol, p.max_iter)
            assert g["converged"] and g["outer_iterations"] >= 1
        phi = _host(sim.phi)
        e_phi = np.linalg.norm(phi - st.phi) / np.linalg.norm(st.phi)
        dE = [_host(a) - r for a, r in zip((sim.ex, sim.ey, sim.ez), (st.ex, st.ey, st.ez))]
        nE = math.sqrt(sum(float(np.dot(r, r)) for r in (st.ex, st.ey, st.ez)))
        e_E = math.sqrt(sum(float(np.dot(d, d)) for d in dE)) / nE
        bound_E = bound_phi * (math.sqrt(3.0) / h) * np.linalg.norm(st.phi) / nE
        x = [_host(a) for a in sim.particles[:3]]
        dxs = [np.abs(a - r) for a, r in zip(x, (st.x, st.y, st.z))]
        dxs = [np.minimum(d, p.length - d) for d in dxs]  # periodic distance
        e_x = max(float(d.max()) for d in dxs) / h
        errs.append((s, e_phi, e_E, e_x))
        assert e_phi <= bound_phi, (s, e_phi, bound_phi)
        assert e_E <= bound_E, (s, e_E, bound_E)
        assert e_x <= dx_bound / h + 1e-15, (s, e_x, dx_bound / h)
        # the next step's push: dv += dt |qm| max|dE| (doubled), dx += dt dv
        maxdE = max(float(np.abs(d).max()) for d in dE)
        dv_bound += 2.0 * p.dt * abs(p.qm) * maxdE
        dx_bound += p.dt * dv_bound
    for s, a, b, c in errs:
        print("step %d: phi %.2e  E %.2e  max|dx|/h %.2e" % (s, a, b, c))
    gk = orc.cell_keys(N, p.length, *[_host(a) for a in sim.particles[:3]])
    ok = orc.cell_keys(N, p.length, st.x, st.y, st.z)
    assert np.array_equal(gk, ok)
