"""Bounded boxes on the GPU (Sec. 3.2: the PCG solver takes Dirichlet and
Neumann boundaries besides periodic ones), through the C ABI, against the FP64
oracle's bounded operator, Jacobi-PCG, SSOR-PCG and field on identical seeded
right-hand sides: iteration counts within one (dot-product order only), the
true residual under the oracle's operator, the solution, and the field."""
import math

import numpy as np
import pytest

from paper_2605_05469_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DIR, NEU = 1, 2
L = 4 * math.pi


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def pic():
    import paper_2605_05469_amd as P
    P.lib()
    return P


def _ctx(pic, N, bc, solver="pcg_fp64", **kw):
    p = pic.landau_params(N, 1, np_max=0, solver=solver, bc=bc, **kw)
    p.length = L
    return pic.Context(p), p


def _rhs(N, bc, seed):
    b = synth.normal_field(N ** 3, seed)
    if bc == NEU:
        b -= b.mean()       # the Neumann problem's solvability condition
    return b


@pytest.mark.parametrize("bc", [DIR, NEU])
@pytest.mark.parametrize("N", [32, 64, 96])
def test_pcg_bounded_matches_oracle(pic, orc, bc, N):
    ctx, p = _ctx(pic, N, bc)
    b = _rhs(N, bc, 7000 + N + bc)
    x = torch.zeros(N ** 3, dtype=torch.float64, device="cuda")
    info = ctx.poisson(_dev(b), x)
    ref, rinfo = orc.pcg(N, L, b, np.zeros(N ** 3), p.rtol, p.max_iter, bc=bc)
    assert info["converged"] and rinfo["converged"]
    assert abs(info["iterations"] - rinfo["iters"]) <= 1
    got = _host(x)
    assert orc.residual_norm(N, L, b, got, bc=bc) <= p.rtol * np.linalg.norm(b)
    if info["iterations"] == rinfo["iters"]:
        assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("unfused", [False, True])
@pytest.mark.parametrize("bc", [DIR, NEU])
@pytest.mark.parametrize("N", [32, 64])
def test_pcg_ssor_bounded_matches_oracle(pic, orc, bc, N, unfused):
    ctx, p = _ctx(pic, N, bc, solver="pcg_ssor",
                  flags=pic.FLAG_SSOR_UNFUSED if unfused else 0)
    b = _rhs(N, bc, 7100 + N + bc)
    x = torch.zeros(N ** 3, dtype=torch.float64, device="cuda")
    info = ctx.poisson(_dev(b), x)
    ref, rinfo = orc.pcg_ssor(N, L, b, np.zeros(N ** 3), p.rtol, p.max_iter, bc=bc)
    assert info["converged"] and rinfo["converged"]
    assert abs(info["iterations"] - rinfo["iters"]) <= 1
    got = _host(x)
    assert orc.residual_norm(N, L, b, got, bc=bc) <= p.rtol * np.linalg.norm(b)
    if info["iterations"] == rinfo["iters"]:
        assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("bc", [DIR, NEU])
def test_mixed_bounded_solves(pic, orc, bc):
    """The mixed form has no bounded oracle of its own: its answer is checked
    through the true residual under the oracle's operator, and against the
    oracle's FP64 solution within the conditioning bound (kappa ~ N^2)."""
    N = 64
    ctx, p = _ctx(pic, N, bc, solver="pcg_mixed", inner_rtol=0.1,
                  flags=pic.FLAG_MIXED_RELIABLE)
    b = _rhs(N, bc, 7200 + bc)
    x = torch.zeros(N ** 3, dtype=torch.float64, device="cuda")
    info = ctx.poisson(_dev(b), x)
    assert info["converged"], info
    got = _host(x)
    assert orc.residual_norm(N, L, b, got, bc=bc) <= p.rtol * np.linalg.norm(b)
    ref, _ = orc.pcg(N, L, b, np.zeros(N ** 3), 1e-13, p.max_iter, bc=bc)
    if bc == NEU:
        got = got - got.mean()
        ref = ref - ref.mean()
    assert np.linalg.norm(got - ref) <= 1e-10 * N * N * np.linalg.norm(ref)


@pytest.mark.parametrize("bc", [DIR, NEU])
@pytest.mark.parametrize("N", [32, 96])
def test_field_bounded_matches_oracle(pic, orc, bc, N):
    ctx, p = _ctx(pic, N, bc)
    phi0 = synth.normal_field(N ** 3, 7300 + N + bc) + 0.5
    phi = _dev(phi0)
    ex, ey, ez = (torch.empty_like(phi) for _ in range(3))
    wx = ctx.efield(phi, ex, ey, ez)
    rphi, rex, rey, rez, rwx = orc.efield(N, L, phi0, bc=bc)
    if bc == DIR:
        assert np.array_equal(_host(phi), phi0)   # no gauge shift
    assert np.max(np.abs(_host(phi) - rphi)) <= 1e-14 * np.abs(rphi).max()
    for a, r in ((ex, rex), (ey, rey), (ez, rez)):
        assert np.max(np.abs(_host(a) - r)) <= 1e-13 * np.abs(r).max()
    assert abs(wx - rwx) <= 1e-12 * rwx


def test_bounded_context_refuses_particle_phases(pic):
    ctx, p = _ctx(pic, 32, DIR)
    rho = torch.zeros(32 ** 3, dtype=torch.float64, device="cuda")
    with pytest.raises(pic.PicError):
        ctx.deposit(None, None, None, None, rho)
    with pytest.raises(pic.PicError):
        ctx.set_solver("fft")
    with pytest.raises(pic.PicError):
        ctx.set_solver("fcg_learned")
