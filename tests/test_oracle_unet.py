"""Pins of the network oracle (oracle.unet) against library convolutions,
adjoint identities, finite differences and torch's Adam.  CPU only."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import unet


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a))


def test_bf16_rounding_matches_library():
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -2.5e-3, 3.0e5, 1e-30, 65504.0, 0.0])
    exp = torch.tensor(vals, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(unet.bf16(vals), exp)
    assert unet.bf16(1 + 2 ** -8) == 1.0 and unet.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6
    rng = np.random.default_rng(0)
    x = rng.standard_normal(10000) * 10.0 ** rng.integers(-5, 5, 10000)
    exp = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(unet.bf16(x), exp)


def test_conv3_matches_torch_circular():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 6, 6, 6))
    W = rng.standard_normal((4, 3, 3, 3, 3))
    b = rng.standard_normal(4)
    ref = F.conv3d(F.pad(_t(x)[None], (1, 1, 1, 1, 1, 1), mode="circular"), _t(W), _t(b))[0].numpy()
    assert np.allclose(unet.conv3_fwd(x, W, b), ref, rtol=1e-12, atol=1e-12)


def test_pool_up_match_torch():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((3, 8, 8, 8))
    ref = F.avg_pool3d(_t(x)[None], 2)[0].numpy()
    assert np.allclose(unet.pool_fwd(x), ref, rtol=1e-13, atol=1e-14)
    xc = rng.standard_normal((5, 4, 4, 4))
    ref = F.interpolate(_t(xc)[None], scale_factor=2, mode="nearest")[0].numpy()
    assert np.array_equal(unet.up_fwd(xc), ref)


def test_adjoint_identities():
    rng = np.random.default_rng(3)
    ci, co = 3, 4
    W = rng.standard_normal(unet.weight_shape(ci, co))
    x = rng.standard_normal((ci, 8, 8, 8))
    y = unet.conv3_fwd(x, W, np.zeros(co))
    dy = rng.standard_normal(y.shape)
    lhs = np.sum(y * dy)
    assert np.isclose(lhs, np.sum(x * unet.conv3_bwd_data(dy, W)), rtol=1e-12)
    dW, db = unet.conv3_bwd_weight(x, dy)
    assert np.isclose(lhs, np.sum(W * dW), rtol=1e-12)
    assert np.allclose(db, dy.sum(axis=(1, 2, 3)))
    g = rng.standard_normal((ci, 4, 4, 4))
    assert np.isclose(np.sum(unet.pool_fwd(x) * g), np.sum(x * unet.pool_bwd(g)), rtol=1e-12)
    assert np.isclose(np.sum(unet.up_fwd(g) * x), np.sum(g * unet.up_bwd(x)), rtol=1e-12)


def test_network_gradient_finite_differences():
    specs = unet.layer_specs(2, 3, 4)
    p = unet.init_params(seed=4, c1=2, c2=3, c3=4)
    rng = np.random.default_rng(5)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((8, 8, 8))
    dout = rng.standard_normal((8, 8, 8))
    out, acts = unet.forward(p, x, specs, round_bf16=False)
    grads, _ = unet.backward(p, acts, dout, specs, round_bf16=False)

    def f(pp):
        return np.sum(unet.forward(pp, x, specs, round_bf16=False)[0] * dout)

    eps = 1e-6
    for name in ("e1a.W", "e2a.W", "b3a.W", "b3b.W", "d2a.b", "out.W", "d2b.b", "d1a.W", "e1b.b"):
        flat = p[name].ravel()
        for j in rng.choice(flat.size, size=min(3, flat.size), replace=False):
            pp = {k: v.copy() for k, v in p.items()}
            pp[name].ravel()[j] += eps
            fp = f(pp)
            pp[name].ravel()[j] -= 2 * eps
            fm = f(pp)
            fd = (fp - fm) / (2 * eps)
            an = grads[name].ravel()[j]
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (name, j, fd, an)


def test_loss_gradient_finite_differences():
    rng = np.random.default_rng(6)
    o, t, r = rng.standard_normal((3, 6, 6, 6))
    L, g = unet.loss(o, t, r, lam=0.7)
    eps = 1e-6
    for j in rng.choice(o.size, 5, replace=False):
        op = o.copy(); op.ravel()[j] += eps
        om = o.copy(); om.ravel()[j] -= eps
        fd = (unet.loss(op, t, r, 0.7)[0] - unet.loss(om, t, r, 0.7)[0]) / (2 * eps)
        assert abs(fd - g.ravel()[j]) <= 1e-7 * max(1.0, abs(fd))


def test_adam_matches_torch():
    rng = np.random.default_rng(7)
    th = rng.standard_normal(50)
    tt = torch.tensor(th.copy(), requires_grad=True)
    opt = torch.optim.Adam([tt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50); v = np.zeros(50)
    for step in range(1, 6):
        g = rng.standard_normal(50)
        th, m, v = unet.adam(th, g, m, v, step)
        tt.grad = torch.tensor(g)
        opt.step()
    assert np.allclose(th, tt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_preconditioner_scale_equivariance_and_zero_mean():
    specs = unet.layer_specs(2, 3, 4)
    p = unet.init_params(seed=8, c1=2, c2=3, c3=4)
    r = np.random.default_rng(9).standard_normal(8 ** 3)
    z = unet.precondition(p, r, 0.3, specs)
    assert abs(z.mean()) < 1e-14 * np.abs(z).max()
    assert np.array_equal(unet.precondition(p, 4.0 * r, 0.3, specs), 4.0 * z)
    assert np.all(unet.precondition(p, 0 * r, 0.3, specs) == 0)


def test_flatten_roundtrip_and_sizes():
    specs = unet.layer_specs()
    p = unet.init_params(seed=1)
    flat = unet.flatten(p, specs)
    q = unet.unflatten(flat, specs)
    assert all(np.array_equal(p[k], q[k]) for k in p)
    n = sum(int(np.prod(unet.weight_shape(a, b))) + b for (_, a, b) in specs)
    assert flat.size == n


@pytest.mark.slow
def test_trained_fcg_golden_values_reproduce(orc):
    """tests/golden/fcg_trained.json holds the oracle's flexible CG with the
    committed trained weights (written by make_fcg_trained.py); the 32^3
    entry is recomputed here so the stored values stay tied to the oracle
    as it is."""
    import hashlib
    import json
    import os
    from paper_2605_05469_amd import synth
    here = os.path.dirname(os.path.abspath(__file__))
    wpath = os.path.join(os.path.dirname(here), "paper_2605_05469_amd", "weights",
                         "unet_landau128.npy")
    with open(os.path.join(here, "golden", "fcg_trained.json")) as f:
        gold = json.load(f)
    with open(wpath, "rb") as f:
        assert hashlib.sha256(f.read()).hexdigest() == gold["weights_sha256"]
    N = 32
    case = gold["cases"][str(N)]
    P = synth.LandauParams(N=N, ppc=8)
    parts = synth.landau_particles_np(N, 8, seed=7000 + N)
    b, _ = orc.deposit(N, P.L, P.q, P.rho_bg, *parts[:3])
    specs = unet.layer_specs()
    params = unet.unflatten(np.load(wpath).astype(np.float64), specs)
    h = P.L / N
    _, info = orc.fcg(N, P.L, b, np.zeros(N ** 3), gold["rtol"], gold["max_iter"],
                      lambda r: unet.precondition(params, r, h, specs), window=gold["window"])
    assert info["converged"] and not info["fell_back"]
    assert abs(info["iters"] - case["fcg_iters"]) <= 1
    _, pinfo = orc.pcg(N, P.L, b, np.zeros(N ** 3), gold["rtol"], 20000)
    assert pinfo["iters"] == case["pcg_iters"]
    # the trained network is a real preconditioner: far fewer iterations
    assert info["iters"] <= 0.4 * pinfo["iters"]
