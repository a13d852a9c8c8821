"""Benchmark: time to an FP64-equivalent relative residual of 1e-8 for P5 on a
128^3 heterogeneous (nebula-like) medium, on one MI355X.

One step = one complete solve A u = Q from u = 0 to ||Q - A u|| <= 1e-8 ||Q||
(FP32 stencil + Krylov vectors, FP64 dot products, scalars and refinement
residual), inputs resident in HBM.  Prints one JSON line.

Also reported (JSON keys):
  roofline      the kernel of the Krylov loop that takes the most time per
                iteration (s -= alpha A^T q at P5 128^3), timed in its in-loop
                form with HIP events on the stream it runs on: algorithmic
                bytes per launch / mean launch time, against the 8 TB/s HBM
                peak; traffic = HBM bytes per launch from the committed
                rocprofv3 FETCH_SIZE / WRITE_SIZE summary when it was taken
                on the current kernel sources.
  loop_kernels  the same figures for every kernel of the loop (the plain
                apply, q = W A p, s -= alpha A^T q, the x/p update).
  cpu_baseline  the FP64 oracle (NumPy, one thread) timed for one CGLS
                iteration at the full size, scaled by the GPU solve's
                iteration count.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "P5 128^3 time-to-1e-8 residual (plain vs learned+mixed); stencil HBM GB/s"
HBM_PEAK_GBS = 8000.0


def source_hash():
    h = hashlib.sha256()
    for f in ("pn_kernels.h", "pn_tables.h", "pn_launch.h"):
        with open(os.path.join(ROOT, "paper_1807_00410_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_hash, kernel):
    """HBM bytes per launch of one loop kernel from the committed rocprofv3
    counter summary, or None when the kernel sources changed since the
    counters were taken."""
    path = os.path.join(ROOT, "profiles", "krylov_p5_128_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != kernel_hash:
        return None
    return d.get("kernels", {}).get(kernel, {}).get("hbm_bytes_per_launch")


# algorithmic HBM bytes of the Krylov-loop kernels: per unknown (FP32 vector
# elements read + written) and whether the medium (8 B per cell) is read
LOOP_KERNELS = (
    ("apply", 8, True, "k_stencil<5,float,APPLY>: y = A x"),
    ("apply_eq", 8, True, "k_stencil<5,float,APPLY_EQ>: q = W A p, <A p, W A p> partials"),
    ("supd", 12, True, "k_stencil<5,float,SUPD>: s -= alpha A^T q, ||s||^2 partials"),
    ("update", 20, False, "k_update_xp<float>: x += alpha p, p = s + beta p"),
)


def cpu_baseline(medium, gpu_iters):
    """One FP64 CGLS iteration of the oracle at the full size (A p, A^T r and
    the vector updates), scaled by the number of iterations the GPU solve
    took.  NumPy element-wise work runs on one thread."""
    import numpy as np
    from oracle.apply import Operator
    op = Operator(medium.order, medium.dims, medium.sigma_t, medium.albedo, medium.g, medium.sigma_t_min)
    rng = np.random.default_rng(0)
    p = rng.normal(size=op.n)
    r = rng.normal(size=op.n)
    x = np.zeros(op.n)
    t0 = time.perf_counter()
    q = op.matvec(p)
    alpha = float(r @ r) / float(q @ q)
    x += alpha * p
    r -= alpha * q
    s = op.rmatvec(r)
    gamma = float(s @ s)
    p = s + (gamma / (gamma + 1.0)) * p
    t_iter = time.perf_counter() - t0
    return {"value": t_iter * gpu_iters, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": "one FP64 CGLS iteration (A p, A^T r, vector updates) of the NumPy oracle on the full "
                      "P5 128^3 system (%.1f s), scaled by the %d iterations of the GPU solve" % (t_iter, gpu_iters),
            "seconds_per_iteration": t_iter}


def bench_batch(args):
    """The batched workload: 48 seeded media (n in {32,48,64,96}, orders
    P1/P3/P5/P7, fBm sigma_t in [0,100], albedo 0.9, g = 0), 8 Gaussian
    emission fields each, solved together to tol with autotuned launch shapes.
    Prints one JSON line."""
    import numpy as np
    import torch
    from synth import config_batch
    from paper_1807_00410_amd.solver import Batch

    t0 = time.perf_counter()
    media = config_batch(seed=7, nmedia=args.batch_media, nrhs=8)
    print("[bench] %d media generated in %.1fs" % (len(media), time.perf_counter() - t0), file=sys.stderr, flush=True)
    probs = [(m.order, m.dims, torch.as_tensor(m.sigma_t).cuda(), torch.as_tensor(m.albedo).cuda(), m.g,
              m.sigma_t_min, m.bc) for m in media]
    t0 = time.perf_counter()
    B = Batch(probs, 8, tune=True)
    t_setup = time.perf_counter() - t0
    rhs = []
    for p, m in enumerate(media):
        lay = B.layouts[p]
        for q in m.q00:
            b = torch.zeros(lay.n, dtype=torch.float32, device="cuda")
            b[lay.offset[0]:lay.offset[1]] = torch.as_tensor(q).cuda().reshape(-1)
            rhs.append(b)
    xs = [torch.zeros(B.layouts[i // 8].n, dtype=torch.float64, device="cuda") for i in range(len(rhs))]
    print("[bench] batch set up in %.1fs: %d systems, %d unknowns" % (t_setup, len(rhs), B.unknowns),
          file=sys.stderr, flush=True)
    ms_apply = B.bench_apply(iters=5)
    cells = sum(m.dims[0] * m.dims[1] * m.dims[2] for m in media)
    alg = 8 * B.unknowns + 8 * cells  # every system's x and y once; each medium once per tile
    print("[bench] batched apply %.3f ms (%.0f GB/s algorithmic)" % (ms_apply, alg / ms_apply / 1e6),
          file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    xs, infos = B.solve(rhs, x=xs, tol=args.tol, inner_tol=args.inner_tol, raise_on_fail=False)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t1
    iters = np.array([d["inner_iters"] for d in infos])
    status = [d["status"] for d in infos]
    unk_it = sum(B.layouts[i // 8].n * int(iters[i]) for i in range(len(infos)))
    print("[bench] batched solve %.2fs, iterations min/mean/max %d/%.0f/%d, %d converged" % (
        sec, iters.min(), iters.mean(), iters.max(), status.count(0)), file=sys.stderr, flush=True)
    out = {
        "metric": "batched solve: unknown-iterations per second (48 media x 8 RHS to tol)",
        "value": unk_it / sec, "unit": "unknown-iterations/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "%d seeded fBm media, n in {32,48,64,96}, P1/P3/P5/P7, 8 RHS each, vacuum, tol %g"
                               % (len(media), args.tol), "systems": len(rhs), "unknowns": B.unknowns},
        "solve_seconds": sec, "setup_seconds": t_setup, "converged": status.count(0),
        "iters_min": int(iters.min()), "iters_mean": float(iters.mean()), "iters_max": int(iters.max()),
        "batched_apply_ms": ms_apply, "batched_apply_algorithmic_GBs": alg / ms_apply / 1e6,
        "zchunks": [B.zchunk(p) for p in range(len(media))],
    }
    B.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--order", type=int, default=5)
    ap.add_argument("--g", type=float, default=0.0)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--inner-tol", type=float, default=1e-2)
    ap.add_argument("--apply-iters", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the pure FP64 Krylov comparison solve")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned + mixed-precision solve")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_1807_00410_amd", "weights", "unet_p3.bin"))
    ap.add_argument("--workload", choices=("p5", "batch"), default="p5")
    ap.add_argument("--batch-media", type=int, default=48)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (requested --gpus %d)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        bench_batch(args)
        return

    import numpy as np
    import torch
    from synth import config_p5_nebula
    from paper_1807_00410_amd.solver import Solver

    t0 = time.perf_counter()
    m = config_p5_nebula(n=args.n, seed=3, g=args.g, order=args.order)
    print("[bench] medium %s generated in %.1fs" % (m.name, time.perf_counter() - t0), file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    st = torch.as_tensor(m.sigma_t).to(dev)
    al = torch.as_tensor(m.albedo).to(dev)
    q00 = torch.as_tensor(m.q00[0]).to(dev)
    s = Solver(m.order, m.dims, st, al, g=m.g, sigma_t_min=m.sigma_t_min)
    zchunk, ms_tuned = s.autotune(10)  # launch shape from the project's autotuner
    print("[bench] autotuned zchunk %d (%.4f ms per apply)" % (zchunk, ms_tuned), file=sys.stderr, flush=True)
    rhs = s.rhs_from_q00(q00)
    x = torch.zeros(s.n, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    def one_solve():
        return s.solve(rhs, x=x, tol=args.tol, inner_tol=args.inner_tol, raise_on_fail=True)

    for i in range(args.warmup):
        _, info = one_solve()
        print("[bench] warmup %d: %.3fs iters %d rel %.3g" % (i, info["seconds"], info["inner_iters"],
                                                              info["rel_residual"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    times, infos = [], []
    t_all = time.perf_counter()
    for i in range(args.steps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, info = one_solve()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
        infos.append(info)
        print("[bench] step %d: %.3fs iters %d outer %d rel %.3g" % (i, times[-1], info["inner_iters"],
                                                                     info["outer_iters"], info["rel_residual"]),
              file=sys.stderr, flush=True)
    total = time.perf_counter() - t_all
    sec = sum(times) / len(times)

    # Krylov-loop kernels in their in-loop form (HIP events on their stream)
    ms_apply = s.bench_apply(args.apply_iters, transpose=False)
    ms_apply_t = s.bench_apply(args.apply_iters, transpose=True)
    cells = m.dims[0] * m.dims[1] * m.dims[2]
    khash = source_hash()
    loop = {}
    for name, per_unknown, medium, desc in LOOP_KERNELS:
        ms = s.bench_kernel(name, args.apply_iters)
        alg = per_unknown * s.n + (8 * cells if medium else 0)
        ach = alg / (ms * 1e-3) / 1e9
        loop[name] = {"kernel": desc, "ms": ms, "algorithmic_bytes_per_launch": alg, "achieved": ach,
                      "frac": ach / HBM_PEAK_GBS, "traffic": load_traffic(khash, name)}
        print("[bench] %-8s %.4f ms  %.0f GB/s algorithmic" % (name, ms, ach), file=sys.stderr, flush=True)
    # the dominant kernel: the most time per iteration of the default solve
    dom = max(("apply_eq", "supd", "update"), key=lambda k: loop[k]["ms"])

    fp64 = None
    if not args.no_fp64:
        xx = torch.zeros_like(x)
        _, i64 = s.solve(rhs, x=xx, tol=args.tol, precision="fp64", raise_on_fail=False)
        fp64 = {"seconds": i64["seconds"], "iters": i64["inner_iters"], "rel_residual": i64["rel_residual"],
                "status": i64["status"]}
        print("[bench] fp64 CGLS: %.3fs iters %d" % (i64["seconds"], i64["inner_iters"]), file=sys.stderr,
              flush=True)

    # FP32 Krylov without refinement: one inner CGLS asked for the full
    # reduction (FP64 dots, FP32 vectors); its FP64 true residual shows where
    # FP32 alone stalls
    fp32_single = None
    if not args.no_fp64:
        xx = torch.zeros_like(x)
        _, i32 = s.solve(rhs, x=xx, tol=args.tol, inner_tol=1e-9, max_refine=1, max_iter=8000, variant="cgls",
                         raise_on_fail=False)
        fp32_single = {"seconds": i32["seconds"], "iters": i32["inner_iters"], "rel_residual": i32["rel_residual"],
                       "status": i32["status"]}
        print("[bench] fp32 CGLS without refinement: %.3fs iters %d rel %.3g" % (
            i32["seconds"], i32["inner_iters"], i32["rel_residual"]), file=sys.stderr, flush=True)

    learned = None
    if not args.no_learned and os.path.exists(args.weights):
        from paper_1807_00410_amd.net import Net
        net = Net(seed=0)
        net.load(args.weights)
        s.attach_net(net)
        for mode in ("guess", "guess+correct"):
            s.solve(rhs, x=x, tol=args.tol, inner_tol=args.inner_tol, learned=mode)  # warm-up
        res = {}
        for mode in ("guess", "guess+correct"):
            lt, li = [], None
            for i in range(args.steps):
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                _, li = s.solve(rhs, x=x, tol=args.tol, inner_tol=args.inner_tol, learned=mode)
                torch.cuda.synchronize()
                lt.append(time.perf_counter() - t1)
            res[mode] = {"seconds": sum(lt) / len(lt), "iters": li["inner_iters"], "outer_iters": li["outer_iters"],
                         "learned_steps": li["learned_steps"], "guess_residual_ratio": li["learned_ratio"],
                         "rel_residual": li["rel_residual"], "speedup_vs_plain": sec / (sum(lt) / len(lt))}
            print("[bench] learned %s: %.3fs iters %d outer %d (guess ratio %.3f)" % (
                mode, res[mode]["seconds"], li["inner_iters"], li["outer_iters"], li["learned_ratio"]),
                file=sys.stderr, flush=True)
        learned = {"weights": os.path.relpath(args.weights, ROOT),
                   "network": "4-level 3D conv U-Net, 32 channels, BF16 MFMA, trained on solver-generated "
                              "P3 64^3 fBm samples (P3 channels; l = 4, 5 start at 0)", **res}
        s.attach_net(None)
        net.close()

    out = {
        "metric": METRIC,
        "value": sec,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "P%d nebula %d^3 (32 Gaussian blobs x fBm, sigma_t in [0,200], albedo 0.95, "
                               "g=%g, 2 point sources), vacuum boundary, tol %g"
                               % (m.order, args.n, m.g, args.tol),
                   "unknowns": s.n, "solver": "FP32 CG on the row-equilibrated normal equations + FP64 dots/refinement (plain)",
                   "inner_tol": args.inner_tol, "zchunk": zchunk},
        "iters": infos[-1]["inner_iters"],
        "outer_iters": infos[-1]["outer_iters"],
        "rel_residual": infos[-1]["rel_residual"],
        "wall_s_timed_region": total,
        "apply_ms": ms_apply,
        "apply_t_ms": ms_apply_t,
        "fp64_krylov": fp64,
        "fp32_krylov_no_refinement": fp32_single,
        "learned_mixed": learned,
        "roofline": {"bound": "hbm", "achieved": loop[dom]["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": loop[dom]["frac"], "traffic": loop[dom]["traffic"],
                     "algorithmic_bytes_per_launch": loop[dom]["algorithmic_bytes_per_launch"],
                     "ms_per_launch": loop[dom]["ms"], "kernel": loop[dom]["kernel"], "source_hash": khash},
        "loop_kernels": loop,
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle, ~20-30 s)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(m, infos[-1]["inner_iters"])
        # the FP64 oracle's own residual of the GPU solution (one CPU matvec)
        from oracle.apply import Operator
        xs = x.cpu().numpy()
        op = Operator(m.order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min)
        b = np.zeros(op.n)
        b[:m.dims[0] * m.dims[1] * m.dims[2]] = m.q00[0].astype(np.float64).reshape(-1)
        out["oracle_rel_residual"] = float(np.linalg.norm(b - op.matvec(xs)) / np.linalg.norm(b))
    s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
