"""Parity of the network kernels (BF16 MFMA convolutions, pooling, loss, Adam,
the whole U-Net and the flexible-PCG solver) with the FP64 oracle on the same
BF16-rounded operands."""
import hashlib
import json
import math
import os

import numpy as np
import pytest

from oracle import unet
from paper_2605_05469_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PAIRS = [(16, 16), (16, 32), (32, 32), (32, 64), (64, 32), (32, 16)]


@pytest.fixture(scope="module")
def pic():
    import paper_2605_05469_amd as P
    P.lib()
    return P


def cl_bf16(a):
    """Oracle [C, z, y, x] (BF16-valued FP64) -> device channels-last bfloat16."""
    return torch.from_numpy(np.ascontiguousarray(a.transpose(1, 2, 3, 0))).to(torch.bfloat16).cuda()


def from_cl(t):
    torch.cuda.synchronize()
    a = t.float().cpu().numpy().astype(np.float64)
    return a.transpose(3, 0, 1, 2)


def f32dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _layer(rng, ci, co, n):
    x = unet.bf16(rng.standard_normal((ci, n, n, n)))
    W = rng.standard_normal((co, ci, 3, 3, 3)).astype(np.float32).astype(np.float64) / math.sqrt(27 * ci)
    b = rng.standard_normal(co).astype(np.float32).astype(np.float64) * 0.1
    return x, W, b


@pytest.mark.parametrize("ci,co", PAIRS)
def test_conv3d_forward_backward_parity(pic, ci, co):
    n = 8
    rng = np.random.default_rng(ci * 100 + co)
    x, W, b = _layer(rng, ci, co, n)
    skip = unet.bf16(rng.standard_normal((co, n, n, n)))
    Wd = f32dev(W.reshape(co, ci, 27))
    ff = torch.empty(pic.conv3d_frag_elems(ci, co), dtype=torch.int16, device="cuda")
    fb = torch.empty(pic.conv3d_frag_elems(co, ci), dtype=torch.int16, device="cuda")
    pic.conv3d_pack(ci, co, Wd, ff, fb)
    # forward: relu(conv + bias + skip), BF16 out
    y = torch.empty((n, n, n, co), dtype=torch.bfloat16, device="cuda")
    pic.conv3d_fwd(n, ci, co, cl_bf16(x), ff, f32dev(b), y, skip=cl_bf16(skip), relu=True)
    ref = np.maximum(unet.conv3_fwd(x, unet.bf16(W), b) + skip, 0.0)
    got = from_cl(y)
    assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-6 * np.abs(ref).max())
    # backward data: FP32 out, no output rounding -> tight
    gy = unet.bf16(rng.standard_normal((co, n, n, n)))
    gx = torch.empty((n, n, n, ci), dtype=torch.float32, device="cuda")
    pic.conv3d_bwd_data(n, ci, co, cl_bf16(gy), fb, gx)
    refx = unet.conv3_bwd_data(gy, unet.bf16(W))
    assert rel(from_cl(gx), refx) <= 1e-5
    # accumulate mode adds to what is there
    pic.conv3d_bwd_data(n, ci, co, cl_bf16(gy), fb, gx, accumulate=True)
    assert rel(from_cl(gx), 2 * refx) <= 1e-5
    # weight gradient
    scratch = torch.empty(pic.conv3d_wgrad_scratch_elems(n, ci, co), dtype=torch.float32, device="cuda")
    grad = torch.empty(27 * ci * co + co, dtype=torch.float32, device="cuda")
    pic.conv3d_bwd_weight(n, ci, co, cl_bf16(x), cl_bf16(gy), scratch, grad)
    dW, db = unet.conv3_bwd_weight(x, gy)
    g = grad.cpu().numpy().astype(np.float64)
    assert rel(g[:27 * ci * co], dW.reshape(-1)) <= 1e-5
    assert rel(g[27 * ci * co:], db) <= 1e-5


@pytest.mark.parametrize("n,ci,co", [(64, a, b) for a, b in PAIRS] + [(128, 16, 16), (128, 32, 16)])
def test_conv3d_zmarch_parity(pic, n, ci, co):
    """Grids that are multiples of 64 take the z-marching kernels (several
    column tiles, z ranges and periodic wraps at these sizes)."""
    rng = np.random.default_rng(n + ci * 100 + co)
    x, W, b = _layer(rng, ci, co, n)
    skip = unet.bf16(rng.standard_normal((co, n, n, n)))
    Wd = f32dev(W.reshape(co, ci, 27))
    ff = torch.empty(pic.conv3d_frag_elems(ci, co), dtype=torch.int16, device="cuda")
    fb = torch.empty(pic.conv3d_frag_elems(co, ci), dtype=torch.int16, device="cuda")
    pic.conv3d_pack(ci, co, Wd, ff, fb)
    y = torch.empty((n, n, n, co), dtype=torch.bfloat16, device="cuda")
    pic.conv3d_fwd(n, ci, co, cl_bf16(x), ff, f32dev(b), y, skip=cl_bf16(skip), relu=True)
    ref = np.maximum(unet.conv3_fwd(x, unet.bf16(W), b) + skip, 0.0)
    got = from_cl(y)
    assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-6 * np.abs(ref).max())
    # linear output (no relu, no skip) must keep negative values
    pic.conv3d_fwd(n, ci, co, cl_bf16(x), ff, f32dev(b), y, relu=False)
    ref = unet.conv3_fwd(x, unet.bf16(W), b)
    got = from_cl(y)
    assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-6 * np.abs(ref).max())
    gy = unet.bf16(rng.standard_normal((co, n, n, n)))
    gx = torch.empty((n, n, n, ci), dtype=torch.float32, device="cuda")
    pic.conv3d_bwd_data(n, ci, co, cl_bf16(gy), fb, gx)
    refx = unet.conv3_bwd_data(gy, unet.bf16(W))
    assert rel(from_cl(gx), refx) <= 1e-5
    pic.conv3d_bwd_data(n, ci, co, cl_bf16(gy), fb, gx, accumulate=True)
    assert rel(from_cl(gx), 2 * refx) <= 1e-5


def test_conv3d_rejects_unsupported(pic):
    assert pic.conv3d_frag_elems(8, 16) == 0
    w = torch.zeros(27 * 16 * 8, dtype=torch.float32, device="cuda")
    with pytest.raises(pic.PicError):
        pic.conv3d_pack(8, 16, w)


def test_adam_parity(pic):
    rng = np.random.default_rng(3)
    th = rng.standard_normal(1000).astype(np.float32).astype(np.float64)
    m = np.zeros(1000)
    v = np.zeros(1000)
    dth, dm, dv = f32dev(th), f32dev(m), f32dev(v)
    for step in range(1, 4):
        g = rng.standard_normal(1000).astype(np.float32).astype(np.float64)
        th, m, v = unet.adam(th, g, m, v, step, lr=1e-2)
        pic.adam_step(dth, dm, dv, f32dev(g), 1e-2, step)
    assert rel(dth.cpu().numpy(), th) <= 1e-6


def _params(seed):
    p = unet.init_params(seed=seed)
    rng = np.random.default_rng(seed + 1)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.05 * rng.standard_normal(p[k].shape)
        p[k] = p[k].astype(np.float32).astype(np.float64)
    return p


@pytest.mark.parametrize("n", [16, 64])
def test_network_forward_backward_parity(pic, n):
    specs = unet.layer_specs()
    p = _params(5)
    flat = unet.flatten(p, specs)
    assert flat.size == pic.unet_param_count()
    net = pic.Net(n, training=True)
    net.set_params(f32dev(flat))
    rng = np.random.default_rng(6)
    x = rng.standard_normal((n, n, n)).astype(np.float32).astype(np.float64)
    out = torch.empty(n ** 3, dtype=torch.float32, device="cuda")
    net.forward(f32dev(x), out)
    ref, acts = unet.forward(p, x, specs)
    got = out.cpu().numpy().astype(np.float64).reshape(n, n, n)
    assert rel(got, ref) <= 1e-2
    dout = rng.standard_normal((n, n, n)).astype(np.float32).astype(np.float64)
    grads = torch.empty(flat.size, dtype=torch.float32, device="cuda")
    net.backward(f32dev(dout), grads)
    rg, _ = unet.backward(p, acts, dout, specs)
    gg = unet.unflatten(grads.cpu().numpy().astype(np.float64), specs)
    # BF16 rounding of activations and gradients makes the emulated network's
    # gradients sensitive to rounding-level changes of its input (a ReLU mask
    # or a rounding decision flips).  The bar: the GPU agrees with the oracle
    # as well as the oracle agrees with itself after a 1e-6 relative
    # perturbation of the input (measured here), and never worse than 5%
    # where that spread is smaller.
    tol = {k: 5e-2 for k in rg}
    if n > 16:
        x2 = x * (1.0 + 1e-6 * np.random.default_rng(60).standard_normal(x.shape))
        _, acts2 = unet.forward(p, x2, specs)
        rg2, _ = unet.backward(p, acts2, dout, specs)
        tol = {k: max(5e-2, 2.0 * rel(rg2[k], rg[k])) for k in rg}
    for name, _, _ in specs:
        for part in (".W", ".b"):
            k = name + part
            assert rel(gg[k], rg[k]) <= tol[k], (k, rel(gg[k], rg[k]), tol[k])


def test_train_step_loss_and_descent(pic):
    n = 16
    specs = unet.layer_specs()
    p = _params(7)
    net = pic.Net(n, training=True)
    net.set_params(f32dev(unet.flatten(p, specs)))
    rng = np.random.default_rng(8)
    r = rng.standard_normal((n, n, n))
    r -= r.mean()
    # target: the exact unit-spacing solution of (-Lap_1) e = r
    m = np.arange(n)
    s = 2 - 2 * np.cos(2 * np.pi * m / n)
    lam = s[:, None, None] + s[None, :, None] + s[None, None, :]
    lam[0, 0, 0] = 1.0
    eh = np.fft.fftn(r) / lam
    eh[0, 0, 0] = 0
    t = np.real(np.fft.ifftn(eh))
    r32, t32 = r.astype(np.float32).astype(np.float64), t.astype(np.float32).astype(np.float64)
    out, _ = unet.forward(p, r32, specs)
    Lref, _ = unet.loss(out, t32, r32, lam=0.5)
    L0 = net.train_step(f32dev(r32), f32dev(t32), lam=0.5, lr=1e-3)
    assert abs(L0 - Lref) <= 1e-2 * Lref
    losses = [net.train_step(f32dev(r32), f32dev(t32), lam=0.5, lr=1e-3) for _ in range(30)]
    assert losses[-1] < 0.9 * L0


@pytest.mark.parametrize("n", [16, 64, 128])
def test_preconditioner_parity_and_homogeneity(pic, n):
    """Inference network (at 64^3 and 128^3 the decoder up-sampling is fused
    into the convolutions' staging and buffers are shared)."""
    specs = unet.layer_specs()
    p = _params(9)
    net = pic.Net(n)
    net.set_params(f32dev(unet.flatten(p, specs)))
    rng = np.random.default_rng(10)
    r = rng.standard_normal(n ** 3)
    h = 0.3
    z = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    net.precondition(torch.from_numpy(r).cuda(), h, z)
    ref = unet.precondition(p, r, h, specs)
    got = z.cpu().numpy()
    assert rel(got, ref) <= 2e-2
    assert abs(got.mean()) <= 1e-12 * np.abs(got).max()
    z4 = torch.empty_like(z)
    net.precondition(torch.from_numpy(4.0 * r).cuda(), h, z4)
    assert torch.equal(z4, 4.0 * z)


def _landau_rhs(orc, N, seed):
    P = synth.LandauParams(N=N, ppc=8)
    parts = synth.landau_particles_np(N, 8, seed=seed)
    b, _ = orc.deposit(N, P.L, P.q, P.rho_bg, *parts[:3])
    return P, b


def test_learned_fcg_converges_and_matches_oracle(pic, orc):
    N = 32
    specs = unet.layer_specs()
    p = _params(11)
    P, b = _landau_rhs(orc, N, 12)
    prm = pic.landau_params(N, 8, np_max=0, solver="fcg_learned", max_iter=2000)
    prm.flags = pic.FLAG_NO_WARM_START  # the oracle's flexible CG has no warm start
    ctx = pic.Context(prm)
    ctx.set_unet(f32dev(unet.flatten(p, specs)))
    x = torch.zeros(N ** 3, dtype=torch.float64, device="cuda")
    info = ctx.poisson(torch.from_numpy(b).cuda(), x)
    assert info["converged"] and info["rel_res"] <= 1e-10
    res = orc.residual_norm(N, P.L, b, x.cpu().numpy()) / np.linalg.norm(b)
    assert res <= 1.0001e-10
    h = P.L / N
    _, oinfo = orc.fcg(N, P.L, b, np.zeros(N ** 3), 1e-10, 2000,
                       lambda r: unet.precondition(p, r, h, specs))
    assert oinfo["converged"]
    assert info["fell_back"] == oinfo["fell_back"]
    if not info["fell_back"]:
        assert abs(info["iterations"] - oinfo["iters"]) <= max(3, 0.2 * oinfo["iters"])


def test_learned_fcg_falls_back_on_a_useless_network(pic, orc):
    N = 32
    P, b = _landau_rhs(orc, N, 13)
    prm = pic.landau_params(N, 8, np_max=0, solver="fcg_learned", max_iter=5000)
    ctx = pic.Context(prm)
    ctx.set_unet(torch.zeros(pic.unet_param_count(), dtype=torch.float32, device="cuda"))
    x = torch.zeros(N ** 3, dtype=torch.float64, device="cuda")
    info = ctx.poisson(torch.from_numpy(b).cuda(), x)
    assert info["converged"] and info["fell_back"] and not info["warm_start_used"]
    assert orc.residual_norm(N, P.L, b, x.cpu().numpy()) <= 1.0001e-10 * np.linalg.norm(b)
    _, pinfo = orc.pcg(N, P.L, b, np.zeros(N ** 3), 1e-10, 5000)
    assert abs(info["iterations"] - pinfo["iters"]) <= 1


def test_learned_warm_start_only(pic, orc):
    """FLAG_WARM_START_ONLY: the network warm start (kept only if it lowers
    the residual), then Jacobi-PCG; the residual test still decides."""
    N = 32
    specs = unet.layer_specs()
    P, b = _landau_rhs(orc, N, 14)
    prm = pic.landau_params(N, 8, np_max=0, solver="fcg_learned", max_iter=5000)
    prm.flags = pic.FLAG_WARM_START_ONLY
    ctx = pic.Context(prm)
    ctx.set_unet(f32dev(unet.flatten(_params(15), specs)))
    x = torch.zeros(N ** 3, dtype=torch.float64, device="cuda")
    info = ctx.poisson(torch.from_numpy(b).cuda(), x)
    assert info["converged"] and info["flex_iterations"] == 0 and not info["fell_back"]
    assert orc.residual_norm(N, P.L, b, x.cpu().numpy()) <= 1.0001e-10 * np.linalg.norm(b)
    if not info["warm_start_used"]:
        _, pinfo = orc.pcg(N, P.L, b, np.zeros(N ** 3), 1e-10, 5000)
        assert abs(info["iterations"] - pinfo["iters"]) <= 1
    with pytest.raises(pic.PicError):
        ctx.set_flags(256)


def test_learned_warm_start_then_mixed(pic, orc):
    """FLAG_LEARNED_MIXED: after the warm start the mixed (reliable-update)
    form finishes the solve; the FP64 true residual still decides."""
    N = 64
    specs = unet.layer_specs()
    P, b = _landau_rhs(orc, N, 16)
    prm = pic.landau_params(N, 8, np_max=0, solver="fcg_learned", inner_rtol=0.1)
    prm.flags = pic.FLAG_WARM_START_ONLY | pic.FLAG_LEARNED_MIXED | pic.FLAG_MIXED_RELIABLE
    ctx = pic.Context(prm)
    ctx.set_unet(f32dev(unet.flatten(_params(17), specs)))
    x = torch.zeros(N ** 3, dtype=torch.float64, device="cuda")
    info = ctx.poisson(torch.from_numpy(b).cuda(), x)
    assert info["converged"] and info["outer_iterations"] >= 1 and info["flex_iterations"] == 0
    assert orc.residual_norm(N, P.L, b, x.cpu().numpy()) <= 1.0001e-10 * np.linalg.norm(b)


# ---------------------------------------------- the trained network -----

_GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fcg_trained.json")
_WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2605_05469_amd", "weights", "unet_landau128.npy")


def _trained():
    with open(_GOLD) as f:
        gold = json.load(f)
    with open(_WEIGHTS, "rb") as f:
        assert hashlib.sha256(f.read()).hexdigest() == gold["weights_sha256"], \
            "fcg_trained.json was written for other weights"
    return gold, np.load(_WEIGHTS)


@pytest.mark.parametrize("N", [32, 64, 128])
def test_trained_fcg_matches_oracle(pic, orc, N):
    """Flexible PCG with the committed trained network (no warm start, as
    in the oracle's flexible CG) against the oracle's flexible CG with the
    same weights (tests/golden/fcg_trained.json, written by
    make_fcg_trained.py from the oracle alone): neither side falls back,
    the iteration counts agree within 2 (the BF16 network with FP32
    accumulation against its FP64 emulation), the true residual under the
    oracle's operator meets 1e-10, and both need far fewer iterations than
    Jacobi-PCG."""
    gold, w = _trained()
    case = gold["cases"][str(N)]
    P = synth.LandauParams(N=N, ppc=8)
    parts = synth.landau_particles_np(N, 8, seed=7000 + N)
    b, _ = orc.deposit(N, P.L, P.q, P.rho_bg, *parts[:3])
    prm = pic.landau_params(N, 8, np_max=0, solver="fcg_learned", max_iter=gold["max_iter"],
                            fcg_window=gold["window"], rtol=gold["rtol"])
    prm.flags = pic.FLAG_NO_WARM_START
    ctx = pic.Context(prm)
    ctx.set_unet(f32dev(w))
    x = torch.zeros(N ** 3, dtype=torch.float64, device="cuda")
    info = ctx.poisson(torch.from_numpy(b).cuda(), x)
    assert info["converged"], info
    assert orc.residual_norm(N, P.L, b, x.cpu().numpy()) <= 1.0001e-10 * np.linalg.norm(b)
    assert not case["fcg_fell_back"] and case["fcg_converged"]
    assert not info["fell_back"], (info, case)
    assert info["flex_iterations"] == info["iterations"]
    assert abs(info["iterations"] - case["fcg_iters"]) <= 2, (info["iterations"], case)
    assert case["fcg_iters"] <= case["pcg_iters"] / 2


def test_training_pair_and_loss(pic):
    """pic_net_make_pair (the scale-free pair the training uses) against its
    definition in FP64, and pic_net_loss against the oracle's loss of the
    oracle's forward pass."""
    n = 16
    specs = unet.layer_specs()
    p = _params(21)
    net = pic.Net(n, training=True)
    net.set_params(f32dev(unet.flatten(p, specs)))
    rng = np.random.default_rng(22)
    rho, phi, rho0, phi0 = (rng.standard_normal(n ** 3) for _ in range(4))
    h = 0.25
    dev = [torch.from_numpy(a).cuda() for a in (rho, phi, rho0, phi0)]
    r_t = torch.empty(n ** 3, dtype=torch.float32, device="cuda")
    t_t = torch.empty_like(r_t)
    for prev in (False, True):
        if prev:
            s = net.make_pair(dev[0], dev[1], h, r_t, t_t, dev[2], dev[3])
            u, e = h * h * (rho - rho0), phi - phi0
        else:
            s = net.make_pair(dev[0], dev[1], h, r_t, t_t)
            u, e = h * h * rho, phi
        s_ref = math.sqrt(np.mean(u * u))
        assert abs(s - s_ref) <= 1e-13 * s_ref
        assert rel(r_t.cpu().numpy().astype(np.float64), u / s_ref) <= 1e-7
        assert rel(t_t.cpu().numpy().astype(np.float64), e / s_ref) <= 1e-7
    r32 = r_t.cpu().numpy().astype(np.float64)
    t32 = t_t.cpu().numpy().astype(np.float64)
    out, _ = unet.forward(p, r32.reshape(n, n, n), specs)
    Lref, _ = unet.loss(out, t32.reshape(n, n, n), r32.reshape(n, n, n), lam=0.5)
    L = net.loss(r_t, t_t, lam=0.5)
    assert abs(L - Lref) <= 1e-2 * Lref
    # no update: the same loss again
    assert net.loss(r_t, t_t, lam=0.5) == L
