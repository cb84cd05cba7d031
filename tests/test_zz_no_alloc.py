"""pic_deposit_cic_noalloc (no context, static scratch) against
pic_deposit_cic (context scratch) through the C ABI: the same kernels, so
the same bits, on two calls in a row with the second on a smaller input, and
the unsorted (atomic) path against the oracle."""
import numpy as np
import pytest

from paper_2605_05469_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _sorted_case(orc, N, ppc, seed):
    parts = synth.landau_particles_np(N, ppc, seed=seed)
    import paper_2605_05469_amd as P
    p = P.landau_params(N, ppc)
    keys = orc.cell_keys(N, p.length, *parts[:3])
    perm, cs = orc.sort_by_key(keys, N ** 3)
    xs = [a[perm] for a in parts[:3]]
    return p, xs, cs


def test_noalloc_deposit_matches_context_deposit(orc):
    import paper_2605_05469_amd as P
    P.lib()
    for N, ppc, seed in ((64, 8, 91), (32, 3, 92)):  # the second call is smaller
        print("no-alloc deposit: N=%d ppc=%d seed=%d" % (N, ppc, seed), flush=True)
        p, xs, cs = _sorted_case(orc, N, ppc, seed)
        d = [_dev(a) for a in xs]
        dcs = _dev(cs.astype(np.uint32).view(np.int32))
        ctx = P.Context(p)
        ref = torch.empty(N ** 3, dtype=torch.float64, device="cuda")
        nb_ref = ctx.deposit(*d, dcs, ref, want_norm=True)
        got = torch.full((N ** 3,), float("nan"), dtype=torch.float64, device="cuda")
        nb = P.deposit_cic_noalloc(p, *d, dcs, got, want_norm=True)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        assert nb == nb_ref
        ref_b, ref_nb = orc.deposit(N, p.length, p.charge, p.rho_bg, *xs)
        assert np.max(np.abs(got.cpu().numpy() - ref_b)) <= 1e-13 * np.abs(ref_b).max()
        ctx.close()
    # unsorted input: FP64 atomics (order not deterministic), against the oracle
    p, xs, cs = _sorted_case(orc, 32, 2, 93)
    shuf = np.random.default_rng(4).permutation(xs[0].size)
    got = torch.empty(32 ** 3, dtype=torch.float64, device="cuda")
    P.deposit_cic_noalloc(p, *[_dev(a[shuf]) for a in xs], None, got)
    ref_b, _ = orc.deposit(32, p.length, p.charge, p.rho_bg, *xs)
    torch.cuda.synchronize()
    assert np.max(np.abs(got.cpu().numpy() - ref_b)) <= 1e-12 * np.abs(ref_b).max()


def test_noalloc_deposit_rejects_oversize_grid():
    import paper_2605_05469_amd as P
    p = P.landau_params(P.NOALLOC_MAX_N * 2, 1)
    x = torch.zeros(8, dtype=torch.float64, device="cuda")
    rho = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(P.PicError):
        P.deposit_cic_noalloc(p, x, x, x, None, rho)
    assert torch.count_nonzero(rho) == 0
