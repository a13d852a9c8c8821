"""Profiling driver for rocprofv3: runs each kernel of the FP32 Krylov loop
of the P5 128^3 nebula workload (plain apply, equilibrated apply q = W A p,
s -= alpha A^T q, x/p update) a fixed number of times in its in-loop form,
then a plain 1 GiB device copy whose counter readings calibrate FETCH_SIZE /
WRITE_SIZE.

    rocprofv3 --pmc FETCH_SIZE -- python3 paper_1807_00410_amd/prof_stencil.py
"""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--order", type=int, default=5)
    ap.add_argument("--iters", type=int, default=10)
    ap.add_argument("--kernels", default="apply,apply_eq,supd,update",
                    help="comma-separated: apply, apply_t, apply_eq, supd, update")
    ap.add_argument("--zchunk", type=int, default=2, help="launch z-chunk (the autotuner's choice at P5 128^3)")
    args = ap.parse_args()
    import torch
    from synth import config_p5_nebula
    from paper_1807_00410_amd.solver import Solver
    m = config_p5_nebula(n=args.n, order=args.order, g=0.0)
    s = Solver(m.order, m.dims, torch.as_tensor(m.sigma_t).cuda(), torch.as_tensor(m.albedo).cuda(),
               g=m.g, sigma_t_min=m.sigma_t_min)
    s.set_zchunk(args.zchunk)
    cells = m.dims[0] * m.dims[1] * m.dims[2]
    per_unknown = {"apply": 8, "apply_t": 8, "apply_eq": 8, "supd": 12, "update": 20}
    for k in args.kernels.split(","):
        ms = s.bench_kernel(k, args.iters)
        alg = per_unknown[k] * s.n + (8 * cells if k != "update" else 0)
        print("%s %.4f ms, %.1f GB/s algorithmic (%d unknowns)" % (k, ms, alg / ms / 1e6, s.n), flush=True)
    a = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)  # calibration: 1 GiB read + 1 GiB written per copy
    torch.cuda.synchronize()
    s.close()


if __name__ == "__main__":
    main()
