"""Writes the oracle's reference solutions of the full-size workloads.

Calls only ``oracle/`` (the C/OpenMP FP64 CGLS of ``oracle/ref.py``) and
``synth/`` (the seeded media).  Each run starts from u = 0 and stops at the
requested relative residual ||Q - A u|| / ||Q|| (the carried CGLS residual;
the recomputed one is reported beside it).  Solutions are stored in FP32,
whose rounding (6e-8 relative per entry) is far below the 1e-5 accuracy they
are used to check.

  p3_64   P3 64^3 fBm medium (sigma_t = 50 fBm, albedo U[0.8,0.99], g = 0.3,
          Gaussian blob of std 4 cells), seed 1  ->  tests/golden/ref_p3_64.npz
  p5_128  P5 128^3 nebula (32 Gaussian blobs x fBm, sigma_t in [0,200],
          albedo 0.95, 2 point sources), seed 3, g = 0 or 0.5
          ->  <outdir>/ref_p5_128_g<g>.npy (305 MB, not committed)

Every run also writes a JSON summary (iterations, the iteration at which the
residual first reached 1e-8, tolerance reached, wall time, threads, host,
date, command) next to the solution, and for p5_128 into profiles/.

Usage:  python tests/golden/make_references.py p3_64 [--threads 8]
        python tests/golden/make_references.py p5_128 --g 0 [--outdir refdata]
"""
import argparse
import datetime
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.assemble import rhs_isotropic  # noqa: E402
from oracle.ref import CRef  # noqa: E402
from synth import config_p3_fbm, config_p5_nebula  # noqa: E402

GOLDEN = os.path.dirname(os.path.abspath(__file__))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def run(m, tol, threads, progress):
    t0 = time.perf_counter()
    R = CRef(m.order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=m.bc, threads=threads)
    b = rhs_isotropic(R.layout, m.q00[0])
    t_setup = time.perf_counter() - t0
    u, info = R.cgls(b, tol=tol, max_iter=200000, progress=progress)
    h = info["history"]
    first = {}
    for t in (1e-6, 1e-8, 1e-10, 1e-12):
        hit = np.nonzero(h <= t)[0]
        first["%g" % t] = int(hit[0]) if hit.size else None
    summary = {
        "workload": m.name, "order": m.order, "dims": list(m.dims), "g": m.g, "sigma_t_min": m.sigma_t_min,
        "unknowns": R.n, "solver": "oracle CGLS (C, OpenMP, FP64) from u = 0",
        "tol": tol, "iters": info["iters"], "carried_rel_residual": info["carried_rel_residual"],
        "rel_residual": info["rel_residual"], "iters_to": first, "seconds": info["seconds"],
        "seconds_per_iteration": info["seconds"] / max(info["iters"], 1), "setup_seconds": t_setup,
        "threads": info["threads"], "cpu": cpu_model(), "nproc": os.cpu_count(),
        "date": datetime.datetime.now(datetime.timezone.utc).strftime("%Y-%m-%d %H:%M UTC"),
        "command": "python tests/golden/make_references.py " + " ".join(sys.argv[1:]),
    }
    return u, summary


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=("p3_64", "p5_128"))
    ap.add_argument("--g", type=float, default=0.0, help="HG g of the P5 nebula (0 or 0.5)")
    ap.add_argument("--tol", type=float, default=1e-12)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--outdir", default=os.path.join(ROOT, "refdata"))
    ap.add_argument("--progress", type=int, default=100)
    args = ap.parse_args()
    if args.workload == "p3_64":
        m = config_p3_fbm(n=64, seed=1)
        u, summary = run(m, args.tol, args.threads, args.progress)
        np.savez_compressed(os.path.join(GOLDEN, "ref_p3_64.npz"), u=u.astype(np.float32))
        with open(os.path.join(GOLDEN, "ref_p3_64.json"), "w") as fh:
            json.dump(summary, fh, indent=1)
    else:
        m = config_p5_nebula(n=128, seed=3, g=args.g)
        u, summary = run(m, args.tol, args.threads, args.progress)
        os.makedirs(args.outdir, exist_ok=True)
        tag = "ref_p5_128_g%g" % args.g
        np.save(os.path.join(args.outdir, tag + ".npy"), u.astype(np.float32))
        with open(os.path.join(args.outdir, tag + ".json"), "w") as fh:
            json.dump(summary, fh, indent=1)
        with open(os.path.join(ROOT, "profiles", "oracle_" + tag[4:] + ".json"), "w") as fh:
            json.dump(summary, fh, indent=1)
    print(json.dumps({k: v for k, v in summary.items() if k != "history"}))


if __name__ == "__main__":
    main()
