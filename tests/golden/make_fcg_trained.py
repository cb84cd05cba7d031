"""Write fcg_trained.json: the oracle's flexible PCG with the committed
trained network (paper_2605_05469_amd/weights/unet_landau128.npy) as its
preconditioner, on seeded Landau-damping right-hand sides (32^3, 64^3,
128^3, 8 particles per cell), next to the oracle's Jacobi-PCG on the same
right-hand side.  Only the oracle computes here; the inputs come from the
seeded generator.  The network's FP64 emulation takes about 25 s per
application at 128^3, so the whole script takes about an hour.

    python tests/golden/make_fcg_trained.py [N ...]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import unet  # noqa: E402
from paper_2605_05469_amd import synth  # noqa: E402

WEIGHTS = os.path.join(ROOT, "paper_2605_05469_amd", "weights", "unet_landau128.npy")
OUT = os.path.join(HERE, "fcg_trained.json")
RTOL, MAX_ITER, WINDOW = 1e-10, 2000, 10


def seed_for(N):
    return 7000 + N


def rhs(N):
    P = synth.LandauParams(N=N, ppc=8)
    parts = synth.landau_particles_np(N, 8, seed=seed_for(N))
    b, _ = oracle.deposit(N, P.L, P.q, P.rho_bg, *parts[:3])
    return P, b


def main(sizes):
    with open(WEIGHTS, "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    w = np.load(WEIGHTS).astype(np.float64)
    specs = unet.layer_specs()
    params = unet.unflatten(w, specs)
    out = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            out = json.load(f)
        if out.get("weights_sha256") != digest:
            out = {}
    out.update({"weights_sha256": digest, "rtol": RTOL, "max_iter": MAX_ITER, "window": WINDOW,
                "ppc": 8, "seed": "7000 + N"})
    cases = out.setdefault("cases", {})
    for N in sizes:
        P, b = rhs(N)
        h = P.L / N
        t0 = time.time()
        napp = [0]

        def M(r):
            napp[0] += 1
            return unet.precondition(params, r, h, specs)

        _, info = oracle.fcg(N, P.L, b, np.zeros(N ** 3), RTOL, MAX_ITER, M, window=WINDOW)
        _, pinfo = oracle.pcg(N, P.L, b, np.zeros(N ** 3), RTOL, 20000)
        cases[str(N)] = {
            "fcg_iters": info["iters"], "fcg_flex_iters": info["flex_iters"],
            "fcg_fell_back": info["fell_back"], "fcg_converged": info["converged"],
            "fcg_true_rel_res": float(info["true_rel_res"]),
            "pcg_iters": pinfo["iters"], "pcg_converged": pinfo["converged"],
            "network_applications": napp[0], "seconds": round(time.time() - t0, 1),
        }
        print(N, cases[str(N)], flush=True)
        with open(OUT, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [32, 64, 128])
