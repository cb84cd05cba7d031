"""What the trained network gains over the method without it.

The same right-hand side (a CIC deposit of Landau-damping particles, 8 per
cell) is solved to relative residual 1e-10 from zero by
  * Jacobi-PCG in FP64 (the plain method of Sec. 3.2),
  * flexible PCG with the trained network as preconditioner,
  * the mixed form (FP32 inner solves, FP64 refinement, reliable updates),
  * the network's warm start followed by the mixed form,
and each solve's iterations and wall time (second call, after a warm-up
call) are recorded and asserted: at 128^3, the size the network was trained
at, flexible PCG needs at most 0.4x Jacobi-PCG's iterations, but one network
application costs more than the iterations it saves, so it is slower; at
512^3 (the headline workload) the 128^3-trained network stalls, flexible PCG
falls back and the residual test still decides, and its warm start saves
the mixed form no inner iterations (out of distribution it costs a few) nor
time; plain FP64 PCG (s-step form) and the mixed form take about the same
time there, both moving about 21 bytes per grid point per iteration.  Every solution
meets the tolerance under the oracle's operator.  The figures are printed
(and written to $PIC_GAIN_OUT as JSON lines when that is set)."""
import json
import os
import time

import numpy as np
import pytest

from paper_2605_05469_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

_WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2605_05469_amd", "weights", "unet_landau128.npy")


def _record(rec):
    print(json.dumps(rec), flush=True)
    out = os.environ.get("PIC_GAIN_OUT")
    if out:
        with open(out, "a") as f:
            f.write(json.dumps(rec) + "\n")


def _forms(P):
    FR = P.FLAG_MIXED_RELIABLE
    return {
        "pcg_fp64": ("pcg_fp64", 0),
        "fcg_learned": ("fcg_learned", P.FLAG_NO_WARM_START),
        "pcg_mixed": ("pcg_mixed", FR),
        "learned_warm_start_mixed": ("fcg_learned",
                                     P.FLAG_WARM_START_ONLY | P.FLAG_LEARNED_MIXED | FR),
    }


def _solve_all(P, orc, N, rho, L, weights):
    res = {}
    for name, (solver, flags) in _forms(P).items():
        prm = P.landau_params(N, 8, np_max=0, solver=solver, flags=flags, inner_rtol=0.1,
                              check_every=32)
        ctx = P.Context(prm)
        if solver == "fcg_learned":
            ctx.set_unet(weights)
        times = []
        for _ in range(2):  # the first call warms up (code objects, buffers)
            x = torch.zeros_like(rho)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = ctx.poisson(rho, x)
            times.append(time.perf_counter() - t0)
        assert info["converged"], (name, info)
        b = rho.cpu().numpy()
        res_true = orc.residual_norm(N, L, b, x.cpu().numpy()) / np.linalg.norm(b)
        assert res_true <= 1.001e-10, (name, res_true)
        res[name] = dict(iterations=info["iterations"], seconds=times[1],
                         fell_back=bool(info["fell_back"]),
                         outer=info["outer_iterations"], rel_res=res_true)
        ctx.close()
    return res


def test_gain_at_training_size(orc):
    import paper_2605_05469_amd as P
    N = 128
    L = synth.box_length()
    Pp = synth.LandauParams(N=N, ppc=8)
    parts = synth.landau_particles_np(N, 8, seed=7300)
    b, _ = orc.deposit(N, L, Pp.q, Pp.rho_bg, *parts[:3])
    rho = torch.from_numpy(b).cuda()
    w = torch.from_numpy(np.load(_WEIGHTS)).cuda()
    r = _solve_all(P, orc, N, rho, L, w)
    _record({"grid": N, "forms": r})
    plain, learned = r["pcg_fp64"], r["fcg_learned"]
    assert not learned["fell_back"]
    assert learned["iterations"] <= 0.4 * plain["iterations"]
    # the measured cost: at 128^3 a network application costs about 16
    # single-reduction PCG iterations, so fewer iterations are still slower
    assert learned["seconds"] > plain["seconds"]


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_gain_at_headline_size(orc):
    import paper_2605_05469_amd as P
    if torch.cuda.get_device_properties(0).total_memory < 200 * 2 ** 30:
        pytest.skip("needs ~120 GiB of device memory")
    N = 512
    p = P.landau_params(N, 8, check_every=32)
    ctx = P.Context(p)
    sim = P.Simulation(ctx, *synth.landau_particles_torch(N, 8, seed=20262, device="cuda"))
    info = sim.init()
    assert info["converged"]
    rho = sim.rho.clone()
    del sim, ctx
    torch.cuda.empty_cache()
    w = torch.from_numpy(np.load(_WEIGHTS)).cuda()
    r = _solve_all(P, orc, N, rho, p.length, w)
    _record({"grid": N, "forms": r})
    plain, mixed = r["pcg_fp64"], r["pcg_mixed"]
    ws = r["learned_warm_start_mixed"]
    # the 128^3-trained network stalls here: flexible PCG falls back
    assert r["fcg_learned"]["fell_back"]
    # its warm start saves the mixed form less than 3% of the inner
    # iterations, and no wall time beyond the box-to-box spread
    assert ws["iterations"] >= 0.97 * mixed["iterations"]
    assert ws["seconds"] >= 0.95 * mixed["seconds"]
    # plain FP64 (s-step form) and the mixed form: within 20% of each other
    assert abs(mixed["seconds"] - plain["seconds"]) <= 0.2 * plain["seconds"]
