"""Write the stored reference values used by the GPU tests and the benchmark.

Calls only ``synth`` and ``oracle`` (FP64 CPU).  Outputs, next to this file:

* ``c1_counts.npz``      Poisson counts y (uint16, K x 128 x 128) of the joint workload with a
                         512x512 object, 128x128 probe and 40x40 raster: expected counts from
                         the oracle's far-field model at the true object and probe, drawn
                         with numpy's PCG64 seeded 1001001.
* ``c1_oracle_lm.json``  the oracle's truncated LM on that data from the workload's initial
                         guess: D = Dg(G) with the App. B diagonal, Jacobi PCG, cg_max 10,
                         Sec. 5 hyper-parameters, T outer iterations; loss per iteration, wall
                         time and the host it ran on.
* ``c0_oracle_lm.json``  the same for the noise-free object-only 64x64 workload (plain LM).

    python tests/golden/make_golden.py [c0] [c1] [--T 50]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import ptycho, solver  # noqa: E402

C1_NOISE_SEED = 1001001


def c1_counts():
    pr = synth.make_c1()
    h = ptycho.intensity(pr.O_true, pr.P_true, pr.pos, pr.background)
    y = np.random.default_rng(C1_NOISE_SEED).poisson(h)
    assert y.max() < 65536
    return pr, y.astype(np.uint16)


def host():
    """The machine the oracle ran on: CPU model, logical cores, and the NumPy FFT's threads (1)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "cpu_count": os.cpu_count(), "threads_used": 1}


def run_lm(pr, y, params, T, joint, O0, P0, label):
    t0 = time.time()
    prog = lambda t, f: print("  %s t=%d f=%.6e  %.0fs" % (label[:3], t, f, time.time() - t0), flush=True)
    res = solver.lm_solve(O0.astype(np.complex128), P0.astype(np.complex128), pr.pos, y.astype(np.float64),
                          pr.background, "gauss", joint, params, T, progress=prog)
    return {"label": label, "T": T, "f_per_iter": res.f_per_iter + [res.f], "f_final": res.f,
            "attempts": [[h.t, h.cg_iters, h.rho, h.lam, bool(h.accepted)] for h in res.history],
            "cg_total": int(sum(h.cg_iters for h in res.history)),
            "seconds": round(time.time() - t0, 1), "host": host()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="*", default=["c0", "c1"])
    ap.add_argument("--T", type=int, default=50)
    ap.add_argument("--out", default=HERE, help="directory of the LM records (the counts stay here)")
    a = ap.parse_args()
    if "c0" in a.which:
        pr = synth.make_c0()
        O0 = pr.O_init.astype(np.complex64)
        P = pr.P_true.astype(np.complex64)
        y = ptycho.intensity(pr.O_true.astype(np.complex64).astype(np.complex128),
                             P.astype(np.complex128), pr.pos, pr.background).astype(np.float32)
        out = run_lm(pr, y, solver.LMParams(), 20, False, O0, P, "c0 plain LM, noise-free, object only")
        json.dump(out, open(os.path.join(a.out, "c0_oracle_lm.json"), "w"), indent=1)
        print("c0 final", out["f_final"], flush=True)
    if "c1" in a.which:
        pr, y = c1_counts()
        path = os.path.join(HERE, "c1_counts.npz")
        if not (os.path.exists(path) and np.array_equal(np.load(path)["y"], y)):
            np.savez_compressed(path, y=y, seed=C1_NOISE_SEED)
            print("c1 counts written", flush=True)
        O0 = pr.O_init.astype(np.complex64)
        P0 = pr.P_init.astype(np.complex64)
        params = solver.LMParams(scaling=1, precond=1, cg_max=10)
        out = run_lm(pr, y, params, a.T, True, O0, P0,
                     "c1 joint LM, D = Dg(G), Jacobi PCG, cg_max 10, Gaussian metric")
        json.dump(out, open(os.path.join(a.out, "c1_oracle_lm.json"), "w"), indent=1)
        print("c1 final", out["f_final"], out["seconds"], flush=True)


if __name__ == "__main__":
    main()
