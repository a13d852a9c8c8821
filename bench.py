"""Benchmark: time to an FP64-equivalent relative residual of 1e-8 for P5 on a
128^3 heterogeneous (nebula-like) medium, on one MI355X.

One step = one complete solve A u = Q from u = 0 to ||Q - A u|| <= 1e-8 ||Q||
(FP32 stencil + Krylov vectors, FP64 dot products, scalars and refinement
residual; the inner solver is the even-parity PCG on the Schur complement of
the even bands), inputs resident in HBM.  Prints one JSON line.

Also reported (JSON keys):
  roofline      the kernel of the Krylov loop that takes the most time per
                iteration, timed in its in-loop form with HIP events on the
                stream it runs on: algorithmic bytes per launch / mean launch
                time, against the 8 TB/s HBM peak; traffic = HBM bytes per
                launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
                summary when it was taken on the current kernel sources.
  loop_kernels  the same figures for every kernel of the loop (the plain
                apply; w_o = -D_o^-1 T_oe p_e, r_e -= alpha S p_e and the PCG
                x/p pass; and the kernels of the normal-equation loop,
                q = W A p, s -= alpha A^T q, the x/p update).
  cg_eq_normal_equations  the previous default inner solver (CG on the
                row-equilibrated normal equations) on the same system.
  cpu_baseline  the C/OpenMP FP64 oracle's CGLS (oracle/pn_ref.c) timed for a
                bounded number of iterations on the full P5 128^3 system on
                this host's cores, scaled by the iterations the oracle's CGLS
                needs to reach 1e-8 on it (its full run, profiles/).
  accuracy      relative L2 error of the GPU solution against the oracle's
                FP64 solution to 1e-12 (when the reference file is present)
                and the oracle's residual of the GPU solution.
  configs       the other workloads: P1 16^3 (FP64 Krylov to 1e-10, error vs
                SuperLU), P3 64^3 (error vs the committed oracle reference),
                P5 128^3 with g = 0.5, the batched workload (48 media x 8
                right-hand sides) and the held-out P3 96^3 medium, plain vs
                learned.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "P5 128^3 time-to-1e-8 residual (plain vs learned+mixed); stencil HBM GB/s"
HBM_PEAK_GBS = 8000.0


def source_hash():
    h = hashlib.sha256()
    for f in ("pn_kernels.h", "pn_tables.h", "pn_launch.h", "pn_mg.h", "pn_mg_kernels.h"):
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


def mg_level_points(layout):
    """Points per level (1, 2, ...) of the multigrid preconditioner: the even
    coefficients' lattices halved (rounding up) until every axis has at most
    5 points and the level at most 2048 (the library's coarsening rule)."""
    ext = [list(layout.ext[k]) for k in range(layout.ncoeff) if math.isqrt(k) % 2 == 0]  # band l = isqrt(k)
    out = []
    while True:
        ext = [[(e + 1) // 2 for e in x] for x in ext]
        out.append(sum(x[0] * x[1] * x[2] for x in ext))
        if (max(max(x) for x in ext) <= 5 and out[-1] <= 2048) or len(out) + 1 >= 12:
            return out


def mg_vcycle_bytes(ne, lv):
    """Algorithmic bytes of one V-cycle (FP32 elements, the 16-byte operator
    {diag, w_x, w_y, w_z} per point): restriction (read fine r; read the
    level-1 diagonal; write r_1, z_1), per level L below the coarsest a down
    pass (read operator, r, z; read the next diagonal; write its r, z) and an
    up pass (read operator, r, z, the coarser correction; write z), the
    coarsest solve (read operator, r, z; write z).  The levels that one
    launch handles in LDS (the tail) are counted the same way: their share is
    below 0.5%."""
    b = 4 * ne + 12 * lv[0]
    for i in range(len(lv) - 1):
        b += 24 * lv[i] + 12 * lv[i + 1]          # down
        b += 28 * lv[i] + 4 * lv[i + 1]           # up
    b += 28 * lv[-1]
    return b


# algorithmic HBM bytes of the Krylov-loop kernels as a function of the
# unknowns n, the even-band unknowns ne, the cells and the multigrid level
# sizes: FP32 vector elements read + written, and the medium (8 B per cell)
# for the stencil passes
LOOP_KERNELS = (
    ("apply", lambda n, ne, c, lv: 8 * n + 8 * c, "k_stencil<5,float,APPLY>: y = A x"),
    ("odd_w", lambda n, ne, c, lv: 4 * ne + 4 * (n - ne) + 8 * c,
     "k_stencil<5,float,ODD_W>: w_o = -D_o^-1 T_oe p_e (odd rows), <p, S p> partials"),
    ("even_r", lambda n, ne, c, lv: 4 * n + 4 * ne + 2 * ne + 4 * ne + 8 * c,
     "k_stencil<5,float,EVEN_SR>: r_e -= alpha (D_e p_e + T_eo w_o) (even rows), <r, M r>, <r, r> partials"),
    ("mg_vcycle", lambda n, ne, c, lv: mg_vcycle_bytes(ne, lv),
     "the V-cycle on P^T r (k_mg_restrict0, k_mg_down, k_mg_tail or k_mg_coarsest, k_mg_up), timed as one"),
    ("pcg_xp_mg", lambda n, ne, c, lv: 22 * ne + 4 * lv[0],
     "k_pcg_vec_mg<2>: x += alpha p, p = 0.6 M r + P z_1 + beta p (M in bfloat16)"),
    ("pcg_xp", lambda n, ne, c, lv: 22 * ne, "k_pcg_vec<2>: x += alpha p, p = M r + beta p (Jacobi loop)"),
    ("apply_eq", lambda n, ne, c, lv: 8 * n + 8 * c, "k_stencil<5,float,APPLY_EQ>: q = W A p (normal-equation loop)"),
    ("supd", lambda n, ne, c, lv: 12 * n + 8 * c, "k_stencil<5,float,SUPD>: s -= alpha A^T q (normal-equation loop)"),
    ("update", lambda n, ne, c, lv: 20 * n, "k_update_xp<float>: x += alpha p, p = s + beta p (normal-equation loop)"),
)
# single kernels of the default solve's loop (the multigrid V-cycle is a group of kernels)
DEFAULT_LOOP = ("odd_w", "even_r", "pcg_xp_mg")


def oracle_run(tag):
    """Summary of the oracle's full reference run of a workload (profiles/)."""
    path = os.path.join(ROOT, "profiles", "oracle_%s.json" % tag)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh)


def cpu_baseline(medium, iters):
    """The C/OpenMP FP64 oracle's CGLS (A p, A^T r and the vector updates of
    oracle/pn_ref.c) on the full system for `iters` iterations on this host's
    cores, scaled by the iterations the oracle's own CGLS takes to reach 1e-8
    on this workload (its full run to 1e-12, profiles/oracle_p5_128_g0.json)."""
    import numpy as np
    from oracle.assemble import rhs_isotropic
    from oracle.ref import CRef
    R = CRef(medium.order, medium.dims, medium.sigma_t, medium.albedo, medium.g, medium.sigma_t_min)
    b = rhs_isotropic(R.layout, medium.q00[0])
    _, info = R.cgls(b, tol=0.0, max_iter=iters)
    per_it = info["seconds"] / max(info["iters"], 1)
    full = oracle_run("p5_128_g%g" % medium.g)
    n8 = full["iters_to"]["1e-08"] if full else None
    out = {"value": per_it * n8 if n8 else None, "unit": "s", "cores": info["threads"], "kind": "oracle",
           "sample": "%d FP64 CGLS iterations of the C/OpenMP oracle on the full P5 128^3 system (%.1f s, %d threads), "
                     "scaled by the %s iterations the oracle's CGLS takes to 1e-8 on it"
                     % (info["iters"], info["seconds"], info["threads"], n8),
           "seconds_per_iteration": per_it, "oracle_iters_to_1e-8": n8}
    if full:
        out["full_run"] = {k: full.get(k) for k in ("iters", "tol", "rel_residual", "seconds", "threads", "cpu", "date",
                                                    "command")}
    return out, R


def rel_l2(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def reference_error(x, tag):
    """rel-L2 error of a GPU solution against the oracle's stored FP64 (1e-12)
    solution, when that file is present (refdata/, not in the repository)."""
    import numpy as np
    path = os.path.join(ROOT, "refdata", "ref_%s.npy" % tag)
    if not os.path.exists(path):
        return None
    return rel_l2(x, np.load(path).astype(np.float64))


def timed_solve(s, rhs, x, warmup=1, **kw):
    import torch
    for _ in range(warmup):
        s.solve(rhs, x=x, **kw)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, info = s.solve(rhs, x=x, **kw)
    torch.cuda.synchronize()
    return time.perf_counter() - t, info


def extra_configs(args):
    """The workloads beside the headline one, each with its time, iterations
    and accuracy against the oracle."""
    import numpy as np
    import torch
    from oracle.assemble import assemble, rhs_isotropic
    from oracle.solve import direct
    from synth import config_p1_homogeneous, config_p3_fbm, config_p5_nebula
    from paper_1807_00410_amd.solver import Solver
    dev = torch.device("cuda:0")
    out = {}

    def mk(m):
        return Solver(m.order, m.dims, torch.as_tensor(m.sigma_t).to(dev), torch.as_tensor(m.albedo).to(dev), g=m.g,
                      sigma_t_min=m.sigma_t_min)

    # P1 16^3 homogeneous: FP64 Krylov to 1e-10, error against SuperLU
    m = config_p1_homogeneous(16)
    s = mk(m)
    rhs = s.rhs_from_q00(torch.as_tensor(m.q00[0]).to(dev))
    x = torch.zeros(s.n, dtype=torch.float64, device=dev)
    sec, info = timed_solve(s, rhs, x, tol=1e-10, precision="fp64")
    A, lay = assemble(m.order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min)
    u = direct(A, rhs_isotropic(lay, m.q00[0]))
    out["p1_16"] = {"workload": "P1 16^3 homogeneous (sigma_t 10, albedo 0.9), FP64 CGLS to 1e-10",
                    "seconds": sec, "iters": info["inner_iters"], "rel_residual": info["rel_residual"],
                    "rel_l2_vs_oracle": rel_l2(x.cpu().numpy(), u), "oracle": "SuperLU"}
    s.close()
    print("[bench] P1 16^3: %.4fs iters %d err %.2e" % (sec, info["inner_iters"], out["p1_16"]["rel_l2_vs_oracle"]),
          file=sys.stderr, flush=True)
    # P3 64^3 fBm: error against the committed oracle reference (CGLS to 1e-12)
    m = config_p3_fbm(n=64, seed=1)
    s = mk(m)
    rhs = s.rhs_from_q00(torch.as_tensor(m.q00[0]).to(dev))
    x = torch.zeros(s.n, dtype=torch.float64, device=dev)
    sec, info = timed_solve(s, rhs, x, tol=args.tol, inner_tol=args.inner_tol)
    ref = np.load(os.path.join(ROOT, "tests", "golden", "ref_p3_64.npz"))["u"].astype(np.float64)
    out["p3_64"] = {"workload": "P3 64^3 fBm (sigma_t 50 fBm, albedo U[0.8,0.99], g 0.3, Gaussian blob), to %g"
                                % args.tol, "seconds": sec, "iters": info["inner_iters"],
                    "rel_residual": info["rel_residual"], "rel_l2_vs_oracle": rel_l2(x.cpu().numpy(), ref),
                    "oracle": "oracle CGLS to 1e-12 (tests/golden/ref_p3_64.npz)"}
    s.close()
    print("[bench] P3 64^3: %.3fs iters %d err %.2e" % (sec, info["inner_iters"], out["p3_64"]["rel_l2_vs_oracle"]),
          file=sys.stderr, flush=True)
    # P5 128^3 nebula, g = 0.5
    m = config_p5_nebula(n=args.n, seed=3, g=0.5, order=args.order)
    s = mk(m)
    s.autotune(10)
    rhs = s.rhs_from_q00(torch.as_tensor(m.q00[0]).to(dev))
    x = torch.zeros(s.n, dtype=torch.float64, device=dev)
    sec, info = timed_solve(s, rhs, x, tol=args.tol, inner_tol=args.inner_tol)
    xs = x.cpu().numpy()
    out["p5_128_g0.5"] = {"workload": "P5 128^3 nebula, g 0.5, to %g" % args.tol, "seconds": sec,
                          "iters": info["inner_iters"], "outer_iters": info["outer_iters"],
                          "rel_residual": info["rel_residual"], "rel_l2_vs_oracle": reference_error(xs, "p5_128_g0.5")}
    s.close()
    print("[bench] P5 128^3 g=0.5: %.3fs iters %d" % (sec, info["inner_iters"]), file=sys.stderr, flush=True)
    # held-out P3 96^3 medium: plain vs learned
    if os.path.exists(args.weights):
        from paper_1807_00410_amd.net import Net
        m = config_p3_fbm(n=96, seed=90002, order=3)
        s = mk(m)
        rhs = s.rhs_from_q00(torch.as_tensor(m.q00[0]).to(dev))
        x = torch.zeros(s.n, dtype=torch.float64, device=dev)
        sec, info = timed_solve(s, rhs, x, tol=args.tol, inner_tol=args.inner_tol)
        r = {"workload": "P3 96^3 fBm, held-out seed 90002, to %g" % args.tol,
             "plain": {"seconds": sec, "iters": info["inner_iters"]}}
        net = Net(seed=0)
        net.load(args.weights)
        s.attach_net(net)
        for mode in ("guess", "guess+correct"):
            sl, li = timed_solve(s, rhs, x, tol=args.tol, inner_tol=args.inner_tol, learned=mode)
            r[mode] = {"seconds": sl, "iters": li["inner_iters"], "learned_steps": li["learned_steps"],
                       "guess_residual_ratio": li["learned_ratio"], "speedup_vs_plain": sec / sl}
        s.attach_net(None)
        net.close()
        s.close()
        out["p3_96_heldout"] = r
        print("[bench] P3 96^3 held-out: plain %.3fs, guess %.3fs" % (sec, r["guess"]["seconds"]), file=sys.stderr,
              flush=True)
    out.update(validation_workloads(args))
    # the batched workload
    out["batch"] = bench_batch(args, quiet=True)
    return out


def validation_workloads(args):
    """The validation problems of section "Results": the 2D checkerboard
    (P1-P5, 71 x 71 cells, to the residual 1e-10 the paper quotes) and the 80^3
    point source (P1-P5, to the same residual; its P1 fluence against the
    oracle's CDA solution).  Optionally writes the fluence along the x axis
    through the source for every order and the CDA."""
    import numpy as np
    import torch
    from oracle.assemble import assemble, rhs_isotropic
    from oracle.cda import cda_solve
    from oracle.solve import direct
    from oracle.stagger import Layout
    from synth import config_checkerboard, config_point_source
    from paper_1807_00410_amd.solver import Solver
    dev = torch.device("cuda:0")
    tol = 1e-10
    paper_cb = {1: 0.27, 5: 25.0}           # seconds on the paper's CPU (hardware not stated)
    paper_ps = {1: 600.0, 5: 2700.0}
    out = {"checkerboard_71": {}, "point_source_80": {}}
    lines = {}
    for name, mk_cfg in (("checkerboard_71", lambda o: config_checkerboard(o, n=71)),
                         ("point_source_80", lambda o: config_point_source(o, n=80))):
        for order in range(1, 6):
            m = mk_cfg(order)
            s = Solver(m.order, m.dims, torch.as_tensor(m.sigma_t).to(dev), torch.as_tensor(m.albedo).to(dev),
                       g=m.g, sigma_t_min=m.sigma_t_min, bc=m.bc, h=m.h)
            rhs = s.rhs_from_q00(torch.as_tensor(m.q00[0]).to(dev))
            x = torch.zeros(s.n, dtype=torch.float64, device=dev)
            sec, info = timed_solve(s, rhs, x, tol=tol, inner_tol=args.inner_tol)
            xs = x.cpu().numpy()
            s.close()
            r = {"seconds": sec, "iters": info["inner_iters"], "outer_iters": info["outer_iters"],
                 "rel_residual": info["rel_residual"], "unknowns": int(xs.size)}
            paper = (paper_cb if name.startswith("checker") else paper_ps).get(order)
            if paper is not None:
                r["paper_seconds_cpu"] = paper
            lay = Layout(m.order, m.dims, m.bc)
            if name.startswith("checker") and order <= 3:
                A, _ = assemble(m.order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=m.bc, h=m.h)
                r["rel_l2_vs_oracle"] = rel_l2(xs, direct(A, rhs_isotropic(lay, m.q00[0])))
                r["oracle"] = "SuperLU"
            if name.startswith("point"):
                c = m.dims[0] // 2
                lines["P%d" % order] = lay.view(xs, 0)[c, c, c:].copy()
                if order == 1:
                    phi = cda_solve(m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, m.q00[0])
                    r["rel_l2_vs_cda"] = rel_l2(lay.view(xs, 0), phi)
                    lines["CDA"] = phi[c, c, c:].copy()
            out[name]["P%d" % order] = r
            print("[bench] %s P%d: %.4fs iters %d" % (name, order, sec, info["inner_iters"]), file=sys.stderr,
                  flush=True)
    out["checkerboard_71"]["workload"] = ("2D checkerboard, 7 x 7 unit blocks on 71 x 71 cells (one z-periodic "
                                          "cell), absorbers sigma_a 10, scatterers sigma_s 1, central unit "
                                          "source; to %g" % tol)
    out["point_source_80"]["workload"] = ("point source, 80^3 cells of size 1/80, sigma_t 8, albedo 0.9, "
                                          "isotropic, Q00 = 1 in the central 2^3 cells; to %g" % tol)
    if args.lineplot:
        with open(args.lineplot, "w") as f:
            f.write("# Point source 80^3: fluence coefficient L00 along +x through the source\n\n")
            f.write("Cells (40..79, 40, 40); sigma_t 8, albedo 0.9, isotropic; every order solved to the "
                    "relative residual 1e-10; CDA by the oracle.\n\nCommand: `python bench.py --no-cpu-baseline "
                    "--lineplot %s`\n\n" % os.path.relpath(args.lineplot, ROOT))
            keys = ["P1", "CDA", "P2", "P3", "P4", "P5"]
            f.write("| r / h | " + " | ".join(keys) + " |\n|" + "---|" * (len(keys) + 1) + "\n")
            for i in range(len(lines["P1"])):
                f.write("| %.1f | " % (i + 0.5) + " | ".join("%.6e" % lines[k][i] for k in keys) + " |\n")
    return out


def bench_batch(args, quiet=False):
    """The batched workload: 48 seeded media (n in {32,48,64,96}, orders
    P1/P3/P5/P7, fBm sigma_t in [0,100], albedo 0.9, g = 0), 8 Gaussian
    emission fields each, solved to tol with autotuned launch shapes; variant
    `--batch-variant` (default schur_mg: every system by the multigrid
    even-parity solve; cg_eq: the batched normal-equation CG, all systems in
    shared launches).  Prints one JSON line (returns the dict instead when
    quiet)."""
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
    xs, infos = B.solve(rhs, x=xs, tol=args.tol, inner_tol=args.inner_tol, raise_on_fail=False,
                        variant=args.batch_variant)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t1
    iters = np.array([d["inner_iters"] for d in infos])
    status = [d["status"] for d in infos]
    unk_it = sum(B.layouts[i // 8].n * int(iters[i]) for i in range(len(infos)))
    print("[bench] batched solve (%s) %.2fs, iterations min/mean/max %d/%.0f/%d, %d converged" % (
        args.batch_variant, sec, iters.min(), iters.mean(), iters.max(), status.count(0)), file=sys.stderr, flush=True)
    out = {
        "metric": "batched solve: time to solve every system (48 media x 8 RHS) to tol",
        "value": sec, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": sec * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "variant": args.batch_variant, "unknown_iterations_per_s": unk_it / sec,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "%d seeded fBm media, n in {32,48,64,96}, P1/P3/P5/P7, 8 RHS each, vacuum, tol %g"
                               % (len(media), args.tol), "systems": len(rhs), "unknowns": B.unknowns},
        "solve_seconds": sec, "setup_seconds": t_setup, "converged": status.count(0),
        "iters_min": int(iters.min()), "iters_mean": float(iters.mean()), "iters_max": int(iters.max()),
        "batched_apply_ms": ms_apply, "batched_apply_algorithmic_GBs": alg / ms_apply / 1e6,
        "zchunks": [B.zchunk(p) for p in range(len(media))],
    }
    B.close()
    if quiet:
        return out
    print(json.dumps(out), flush=True)


def profile_kernels(args):
    """Profiling mode for rocprofv3 (--profile-kernels): runs each listed
    kernel of the FP32 Krylov loops of the P5 nebula workload (the plain
    apply; the even-parity loop odd_w, even_r, pcg_xp; the
    normal-equation loop apply_eq, supd, update) `--profile-iters` times in its in-loop form
    at a fixed z-chunk, then three plain 1 GiB device copies whose counter
    readings calibrate FETCH_SIZE / WRITE_SIZE (bytes per copy known).  Prints
    the live timings; the counters come from the profiler."""
    import torch
    from synth import config_p5_nebula
    from paper_1807_00410_amd.solver import Solver
    m = config_p5_nebula(n=args.n, order=args.order, g=args.g)
    s = Solver(m.order, m.dims, torch.as_tensor(m.sigma_t).cuda(), torch.as_tensor(m.albedo).cuda(),
               g=m.g, sigma_t_min=m.sigma_t_min)
    s.set_zchunk(args.profile_zchunk)
    cells = m.dims[0] * m.dims[1] * m.dims[2]
    ne = s.even_unknowns()
    nbytes = {name: f for name, f, _ in LOOP_KERNELS}
    nbytes["apply_t"] = nbytes["apply"]
    lv = mg_level_points(s.layout)
    geo = {"n": s.n, "ne": ne, "cells": cells, "mg_level_points": lv, "algorithmic_bytes": {}, "ms": {}}
    for k in args.profile_kernels.split(","):
        ms = s.bench_kernel(k, args.profile_iters)
        alg = nbytes[k](s.n, ne, cells, lv)
        geo["algorithmic_bytes"][k] = alg
        geo["ms"][k] = ms
        print("%s %.4f ms, %.1f GB/s algorithmic (%d unknowns)" % (k, ms, alg / ms / 1e6, s.n), flush=True)
    print("GEOMETRY " + json.dumps(geo), flush=True)
    a = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)  # calibration: 1 GiB read + 1 GiB written per copy
    torch.cuda.synchronize()
    s.close()


# kernels of each profiled loop kernel in the rocprofv3 output (the V-cycle:
# every kernel of the group, per V-cycle)
PROFILE_NAMES = {
    "apply": ("k_stencil<5, float, 0, float,",),
    "odd_w": ("k_stencil<5, float, 6, float,",),
    "even_r": ("k_stencil<5, float, 11, float,",),
    "pcg_xp_mg": ("k_pcg_vec_mg<2>",),
    "mg_vcycle": ("k_mg_restrict0", "k_mg_down", "k_mg_tail", "k_mg_coarsest", "k_mg_up"),
}


def counters_summary(args):
    """--counters-summary DIR: reads the outputs of the three rocprofv3 runs
    of `bench.py --profile-kernels` (DIR/fetch, DIR/write: --pmc FETCH_SIZE /
    WRITE_SIZE in csv; DIR/ktrace: --kernel-trace in csv, its stdout in
    DIR/ktrace.log) and writes profiles/krylov_p5_128_counters.json and .md:
    per loop kernel the HBM bytes per launch (counters scaled by the three
    1 GiB copies of the same run), the algorithmic bytes and the trace's mean
    duration.  Runs on the CPU."""
    import csv
    d = args.counters_summary
    geo = None
    with open(os.path.join(d, "ktrace.log")) as fh:
        for line in fh:
            if line.startswith("GEOMETRY "):
                geo = json.loads(line[len("GEOMETRY "):])
    rows = {c: list(csv.DictReader(open(os.path.join(d, c, c + "_counter_collection.csv")))) for c in ("fetch", "write")}
    trace = list(csv.DictReader(open(os.path.join(d, "ktrace", "ktrace_kernel_trace.csv"))))
    cal = {}
    for c in ("fetch", "write"):
        big = sorted(float(r["Counter_Value"]) for r in rows[c] if "copyBuffer" in r["Kernel_Name"])[-3:]
        cal[c] = (1 << 30) / (sum(big) / len(big) * 1024.0)
    out = {"workload": "P5 nebula 128^3, zchunk 2", "source_hash": source_hash(), "fetch_factor": cal["fetch"],
           "write_factor": cal["write"], "summary": "profiles/krylov_p5_128_counters.md", "kernels": {}}
    for name, pats in PROFILE_NAMES.items():
        if name not in geo["algorithmic_bytes"]:
            continue
        match = lambda kn: any(p in kn for p in pats)
        launches = sum(1 for r in rows["fetch"] if pats[0] in r["Kernel_Name"])
        tot = {c: sum(float(r["Counter_Value"]) for r in rows[c] if match(r["Kernel_Name"])) for c in rows}
        durs = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in trace if match(r["Kernel_Name"])]
        ntrace = sum(1 for r in trace if pats[0] in r["Kernel_Name"])
        hf = tot["fetch"] / launches * 1024 * cal["fetch"]
        hw = tot["write"] / launches * 1024 * cal["write"]
        alg = geo["algorithmic_bytes"][name]
        out["kernels"][name] = {"kernels": list(pats), "launches": launches,
                                "fetch_KiB_per_launch": tot["fetch"] / launches,
                                "write_KiB_per_launch": tot["write"] / launches,
                                "hbm_fetch_bytes_per_launch": hf, "hbm_write_bytes_per_launch": hw,
                                "hbm_bytes_per_launch": hf + hw, "algorithmic_bytes_per_launch": alg,
                                "traffic_over_algorithmic": (hf + hw) / alg,
                                "mean_us_trace": sum(durs) / max(ntrace, 1) / 1e3}
    with open(os.path.join(ROOT, "profiles", "krylov_p5_128_counters.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    cmd = "python3 bench.py --profile-kernels " + ",".join(geo["algorithmic_bytes"])
    lines = ["# Krylov-loop kernels, P5 128^3: HBM traffic counters (rocprofv3 --pmc)", "",
             "Commands (from the repository root, `TMPDIR=/tmp`; `bench.py --profile-kernels` runs each listed",
             "loop kernel of the nebula workload in its in-loop form, 1 warm-up + 10 timed iterations at",
             "zchunk 2, then three 1 GiB device copies that calibrate the counters):", "",
             "    timeout -s KILL 150 rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/prof/fetch -o fetch -- \\",
             "        " + cmd,
             "    timeout -s KILL 150 rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/prof/write -o write -- \\",
             "        " + cmd,
             "    timeout -k 10 150 rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof/ktrace -o ktrace -- \\",
             "        " + cmd + " > gpurun_out/prof/ktrace.log",
             "    python3 bench.py --counters-summary gpurun_out/prof      # this file and its .json", "",
             "Calibration (the three 1 GiB `copyBuffer` dispatches): HBM bytes = FETCH_SIZE x 1024 x %.3f and"
             % cal["fetch"], "WRITE_SIZE x 1024 x %.3f.  The V-cycle row sums all kernels of one V-cycle (restriction, "
             "the down and up passes of the large levels, the one-launch tail of the small ones)." % cal["write"], "",
             "| loop kernel | launches | HBM read MB | HBM write MB | algorithmic MB | traffic / algorithmic | trace mean us | algorithmic GB/s |",
             "|---|---|---|---|---|---|---|---|"]
    for name, k in out["kernels"].items():
        lines.append("| %s | %d | %.1f | %.1f | %.1f | %.2f | %.1f | %.0f |" % (
            name, k["launches"], k["hbm_fetch_bytes_per_launch"] / 1e6, k["hbm_write_bytes_per_launch"] / 1e6,
            k["algorithmic_bytes_per_launch"] / 1e6, k["traffic_over_algorithmic"], k["mean_us_trace"],
            k["algorithmic_bytes_per_launch"] / k["mean_us_trace"] / 1e3))
    lines += ["", "Geometry: n = %d unknowns, ne = %d in the even bands, %d cells; multigrid level points %s." % (
        geo["n"], geo["ne"], geo["cells"], geo["mg_level_points"]),
        "Algorithmic bytes: see `LOOP_KERNELS` and `mg_vcycle_bytes` in bench.py.",
        "", "Kernel source hash (pn_kernels.h, pn_tables.h, pn_launch.h, pn_mg.h, pn_mg_kernels.h): %s" % out["source_hash"]]
    with open(os.path.join(ROOT, "profiles", "krylov_p5_128_counters.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))
    solve_stats = os.path.join(d, "solve", "solve_kernel_stats.csv")
    if os.path.exists(solve_stats):
        stats = list(csv.DictReader(open(solve_stats)))
        log = open(os.path.join(d, "solve.log")).read().strip().splitlines() if os.path.exists(
            os.path.join(d, "solve.log")) else []
        sl = ["# P5 128^3 nebula solve: kernel time (rocprofv3 kernel trace)", "",
              "Command (from the repository root, `TMPDIR=/tmp`):", "",
              "    timeout -k 10 150 rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof/solve "
              "-o solve -- \\", "        python3 bench.py --profile-solve --profile-iters 2 > gpurun_out/prof/solve.log",
              "    python3 bench.py --counters-summary gpurun_out/prof", "",
              "Three solves (one untimed, two profiled) of the P5 128^3 nebula (76,237,059 unknowns, 31,753,344 in "
              "the even bands) with the default solver: the even-parity PCG with the multigrid preconditioner, "
              "FP32 vectors, FP64 dots and refinement, tol 1e-8, inner_tol 1e-2, zchunk 2.  The program's "
              "output:", ""] + ["    " + x for x in log if x.startswith("solve ")] + [
              "", "All dispatches (loop kernels launched after a solve's stop flag return at once and pull the "
              "averages down; each captured graph holds 8 iterations):", "",
              "| kernel | calls | total ms | avg us | min us | max us | % of GPU time |", "|---|---|---|---|---|---|---|"]
        for r in stats[:20]:
            nm = r["Name"].split("(")[0]
            sl.append("| `%s` | %s | %.2f | %.1f | %.1f | %.1f | %.1f |" % (
                nm, r["Calls"], float(r["TotalDurationNs"]) / 1e6, float(r["AverageNs"]) / 1e3,
                float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
        with open(os.path.join(ROOT, "profiles", "solve_p5_128_kernel_stats.md"), "w") as fh:
            fh.write("\n".join(sl) + "\n")


def net_kernels(args):
    """--net-kernels: the U-Net's 3x3x3 32 -> 32 convolution (forward with
    ReLU, input gradient, weight gradient) at the U-Net's level sizes for a
    batch of 4 64^3 volumes, each timed over 20 launches with HIP events on
    the current stream; 55,296 flop per voxel against the 2.5 PFLOP/s dense
    BF16 peak."""
    import torch
    from paper_1807_00410_amd import net as N
    torch.manual_seed(0)
    rows = []
    for n in (64, 32, 16, 8):
        x = (torch.randn(4, n, n, n, 32, device="cuda") * 0.5).to(torch.bfloat16)
        g = (torch.randn(4, n, n, n, 32, device="cuda") * 0.5).to(torch.bfloat16)
        w = (torch.randn(27, 32, 32, device="cuda") * 0.05).to(torch.bfloat16)
        b = torch.zeros(32, device="cuda")
        for name, fn in (("forward", lambda: N.conv3d(x, w, b, relu=True)), ("input gradient", lambda: N.conv3d_dgrad(g, w)),
                         ("weight gradient", lambda: N.conv3d_wgrad(x, g))):  # the API call: with its temporary partials buffer
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(20):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 20
            tf = 55296.0 * 4 * n ** 3 / ms / 1e9
            rows.append({"kernel": name, "voxels": 4 * n ** 3, "ms": ms, "TFLOPs": tf, "frac": tf / 2500.0})
            print("%-15s 4 x %2d^3  %.4f ms  %6.0f TFLOP/s  %.3f of peak" % (name, n, ms, tf, tf / 2500.0), flush=True)
    print(json.dumps({"net_kernels": rows}), flush=True)


def variant_sweep(args):
    """--variant-sweep: the even-parity PCG with the Jacobi and with the
    multigrid preconditioner on the validation problems and on fBm / nebula
    media of several sizes and orders (best of 3 solves after a warm-up each);
    writes the table (default profiles/variant_sweep.md), the measurement
    behind AUTO's choice."""
    import torch
    from synth import config_checkerboard, config_point_source, config_p3_fbm, config_p5_nebula
    from paper_1807_00410_amd.solver import Solver
    dev = torch.device("cuda:0")
    cases = [("checkerboard 71 x 71 P%d" % o, config_checkerboard(o, n=71), 1e-10) for o in range(1, 6)]
    cases += [("point source 80^3 P%d" % o, config_point_source(o, n=80), 1e-10) for o in range(1, 6)]
    for n in (24, 32, 48):
        cases += [("P3 fBm %d^3" % n, config_p3_fbm(n=n), 1e-8), ("P5 nebula %d^3" % n, config_p5_nebula(n=n), 1e-8)]
    for n in (24, 32, 48):
        cases += [("P2 fBm %d^3" % n, config_p3_fbm(n=n, order=2), 1e-8),
                  ("P4 fBm %d^3" % n, config_p3_fbm(n=n, order=4), 1e-8)]
    cases += [("P4 nebula 64^3", config_p5_nebula(n=64, order=4), 1e-8),
              ("P6 nebula 64^3", config_p5_nebula(n=64, order=6), 1e-8)]
    lines = ["# Jacobi vs multigrid preconditioner of the even-parity PCG", "",
             "Command (repository root, one GPU): `python3 bench.py --variant-sweep`", "",
             "Each problem solved from u = 0 with `variant=\"schur\"` (Jacobi) and `variant=\"schur_mg\"`; best of 3",
             "timed solves after one warm-up each; tolerance 1e-10 for the validation problems, 1e-8 otherwise.",
             "AUTO takes the multigrid form for odd orders with at least 2^17 even-band unknowns.", "",
             "| problem | even-band unknowns | Jacobi ms | Jacobi iterations | multigrid ms | multigrid iterations "
             "| multigrid / Jacobi time | AUTO |", "|---|---|---|---|---|---|---|---|"]
    for name, m, tol in cases:
        s = Solver(m.order, m.dims, torch.as_tensor(m.sigma_t).to(dev), torch.as_tensor(m.albedo).to(dev),
                   g=m.g, sigma_t_min=m.sigma_t_min, bc=m.bc, h=m.h)
        rhs = s.rhs_from_q00(torch.as_tensor(m.q00[0]).to(dev))
        res = {}
        for v in ("schur", "schur_mg"):
            x = torch.zeros(s.n, dtype=torch.float64, device=dev)
            best, info = min((timed_solve(s, rhs, x, warmup=1 if k == 0 else 0, tol=tol, variant=v) for k in range(3)),
                             key=lambda r: r[0])
            res[v] = (best, info["inner_iters"])
        ne = s.even_unknowns()
        auto = "multigrid" if (m.order % 2 == 1 and ne >= 1 << 17) else "Jacobi"
        s.close()
        lines.append("| %s | %d | %.2f | %d | %.2f | %d | %.2f | %s |" % (
            name, ne, res["schur"][0] * 1e3, res["schur"][1], res["schur_mg"][0] * 1e3, res["schur_mg"][1],
            res["schur_mg"][0] / res["schur"][0], auto))
        print(lines[-1], file=sys.stderr, flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(args.sweep_out)), exist_ok=True)
    with open(args.sweep_out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def profile_solve(args):
    """Profiling mode for rocprofv3 (--profile-solve): the headline workload
    (P5 nebula) solved by the default solver once untimed, then
    `--profile-iters` times, nothing else -- the kernel trace of a real solve
    (every kernel of the Krylov loop and the preconditioner, with their
    per-launch durations)."""
    import torch
    from synth import config_p5_nebula
    from paper_1807_00410_amd.solver import Solver
    m = config_p5_nebula(n=args.n, order=args.order, g=args.g)
    s = Solver(m.order, m.dims, torch.as_tensor(m.sigma_t).cuda(), torch.as_tensor(m.albedo).cuda(),
               g=m.g, sigma_t_min=m.sigma_t_min)
    s.set_zchunk(args.profile_zchunk)
    rhs = s.rhs_from_q00(torch.as_tensor(m.q00[0]).cuda())
    for i in range(1 + args.profile_iters):
        x, info = s.solve(rhs, tol=args.tol, inner_tol=args.inner_tol)
        print("solve %d: %.4f s, %d iterations, %d refinement steps, rel %.3g" % (
            i, info["seconds"], info["inner_iters"], info["outer_iters"], info["rel_residual"]), flush=True)
    s.close()


def accuracy_check(args):
    """--accuracy: the P5 128^3 nebula (g = 0 and 0.5) solved to 1e-8 by the
    default inner solver, the equilibrated normal equations and FP64 CGLS,
    each compared with the oracle's FP64 solution to 1e-12
    (refdata/ref_p5_128_g<g>.npy, written by tests/golden/make_references.py;
    workloads without that file are skipped).  Prints one JSON line."""
    import numpy as np
    import torch
    from synth import config_p5_nebula
    from paper_1807_00410_amd.solver import Solver
    out = {}
    for g in (0.0, 0.5):
        path = os.path.join(ROOT, "refdata", "ref_p5_128_g%g.npy" % g)
        if not os.path.exists(path):
            continue
        ref = np.load(path).astype(np.float64)
        m = config_p5_nebula(n=128, seed=3, g=g)
        s = Solver(m.order, m.dims, torch.as_tensor(m.sigma_t).cuda(), torch.as_tensor(m.albedo).cuda(), g=m.g,
                   sigma_t_min=m.sigma_t_min)
        rhs = s.rhs_from_q00(torch.as_tensor(m.q00[0]).cuda())
        res = {}
        for name, kw in (("even-parity PCG, multigrid (default)", {}),
                         ("even-parity PCG, Jacobi", {"variant": "schur"}),
                         ("CG, equilibrated normal equations", {"variant": "cg_eq"}),
                         ("CGLS in FP64", {"precision": "fp64"})):
            x, info = s.solve(rhs, tol=args.tol, **kw)
            xs = x.cpu().numpy()
            res[name] = {"iters": info["inner_iters"], "rel_residual": info["rel_residual"], "seconds": info["seconds"],
                         "rel_l2_vs_oracle": float(np.linalg.norm(xs - ref) / np.linalg.norm(ref)),
                         "max_abs_err_over_max": float(np.max(np.abs(xs - ref)) / np.max(np.abs(ref)))}
            print("[bench] g=%g %-34s iters %5d rel %.3g rel-L2 vs oracle %.3e" % (
                g, name, info["inner_iters"], info["rel_residual"], res[name]["rel_l2_vs_oracle"]), file=sys.stderr,
                flush=True)
        out["p5_128_g%g" % g] = res
        s.close()
    print(json.dumps({"accuracy_vs_oracle": out, "tol": args.tol}), flush=True)


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
    ap.add_argument("--cpu-iters", type=int, default=12, help="oracle CGLS iterations timed for the CPU baseline")
    ap.add_argument("--no-configs", action="store_true", help="skip the other workloads (P1, P3 64^3, P5 g=0.5, "
                                                             "batch, P3 96^3 held-out)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the pure FP64 Krylov comparison solve")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned + mixed-precision solve")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_1807_00410_amd", "weights", "unet_p3.bin"))
    ap.add_argument("--workload", choices=("p5", "batch"), default="p5")
    ap.add_argument("--batch-media", type=int, default=48)
    ap.add_argument("--batch-variant", default="schur_mg", choices=("schur_mg", "cg_eq"),
                    help="inner solver of the batched workload")
    ap.add_argument("--lineplot", default=None, metavar="PATH",
                    help="write the point-source fluence along +x for P1-P5 and the CDA as a markdown table")
    ap.add_argument("--profile-kernels", default=None, metavar="LIST",
                    help="profiling mode: comma-separated loop kernels (apply, apply_t, odd_w, even_r, pcg_xp, "
                         "apply_eq, supd, update) "
                         "run in their in-loop form for rocprofv3, then the counter-calibration copies")
    ap.add_argument("--profile-iters", type=int, default=10)
    ap.add_argument("--net-kernels", action="store_true",
                    help="time the U-Net convolution kernels (forward, input and weight gradient) per level")
    ap.add_argument("--counters-summary", default=None, metavar="DIR",
                    help="write profiles/krylov_p5_128_counters.{json,md} from the rocprofv3 outputs in DIR")
    ap.add_argument("--profile-solve", action="store_true",
                    help="solve the P5 nebula 1 + --profile-iters times with the default solver, nothing else "
                         "(the kernel trace of a real solve for rocprofv3)")
    ap.add_argument("--accuracy", action="store_true",
                    help="compare the P5 128^3 solutions with the oracle's reference solutions in refdata/")
    ap.add_argument("--profile-zchunk", type=int, default=2)
    ap.add_argument("--variant-sweep", action="store_true",
                    help="Jacobi vs multigrid preconditioner over problem sizes and orders "
                         "(writes the table to --sweep-out)")
    ap.add_argument("--sweep-out", default=os.path.join(ROOT, "profiles", "variant_sweep.md"))
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (requested --gpus %d)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.profile_kernels:
        profile_kernels(args)
        return
    if args.profile_solve:
        profile_solve(args)
        return
    if args.variant_sweep:
        variant_sweep(args)
        return
    if args.counters_summary:
        counters_summary(args)
        return
    if args.net_kernels:
        net_kernels(args)
        return
    if args.accuracy:
        accuracy_check(args)
        return
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
    xs = x.cpu().numpy()  # the solution of the last timed step

    # Krylov-loop kernels in their in-loop form (HIP events on their stream)
    ms_apply = s.bench_apply(args.apply_iters, transpose=False)
    ms_apply_t = s.bench_apply(args.apply_iters, transpose=True)
    cells = m.dims[0] * m.dims[1] * m.dims[2]
    khash = source_hash()
    loop = {}
    ne = s.even_unknowns()
    lv = mg_level_points(s.layout)
    for name, nbytes, desc in LOOP_KERNELS:
        ms = s.bench_kernel(name, args.apply_iters)
        alg = nbytes(s.n, ne, cells, lv)
        ach = alg / (ms * 1e-3) / 1e9
        loop[name] = {"kernel": desc, "ms": ms, "algorithmic_bytes_per_launch": alg, "achieved": ach,
                      "frac": ach / HBM_PEAK_GBS, "traffic": load_traffic(khash, name)}
        print("[bench] %-8s %.4f ms  %.0f GB/s algorithmic" % (name, ms, ach), file=sys.stderr, flush=True)
    # the dominant kernel: the most time per iteration of the default (even-parity) solve
    dom = max(DEFAULT_LOOP, key=lambda k: loop[k]["ms"])

    # the even-parity PCG with the Jacobi preconditioner alone
    tj, ij = timed_solve(s, rhs, torch.zeros_like(x), warmup=0, tol=args.tol, inner_tol=args.inner_tol,
                         variant="schur")
    jac = {"seconds": tj, "iters": ij["inner_iters"], "rel_residual": ij["rel_residual"],
           "speedup_of_default": tj / sec}
    print("[bench] even-parity PCG, Jacobi preconditioner: %.3fs iters %d" % (tj, ij["inner_iters"]),
          file=sys.stderr, flush=True)
    # CG on the row-equilibrated normal equations on the same system
    ti, ii = timed_solve(s, rhs, torch.zeros_like(x), warmup=0, tol=args.tol, inner_tol=args.inner_tol,
                         variant="cg_eq")
    cg_eq = {"seconds": ti, "iters": ii["inner_iters"], "rel_residual": ii["rel_residual"],
             "speedup_of_default": ti / sec}
    print("[bench] CG on the equilibrated normal equations: %.3fs iters %d" % (ti, ii["inner_iters"]),
          file=sys.stderr, flush=True)
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
                   "unknowns": s.n, "solver": "FP32 even-parity PCG (CG on the Schur complement of the even bands, "
                                             "preconditioner 0.6 Jacobi + one aggregation V-cycle per even "
                                             "coefficient) + FP64 dots/refinement (plain)",
                   "inner_tol": args.inner_tol, "zchunk": zchunk},
        "iters": infos[-1]["inner_iters"],
        "outer_iters": infos[-1]["outer_iters"],
        "rel_residual": infos[-1]["rel_residual"],
        "wall_s_timed_region": total,
        "apply_ms": ms_apply,
        "apply_t_ms": ms_apply_t,
        "phases_ms": infos[-1]["t_ms"], "solve_algorithmic_bytes": infos[-1]["bytes"],
        "solve_achieved_GBs": infos[-1]["achieved_gbs"],
        "even_parity_jacobi": jac,
        "cg_eq_normal_equations": cg_eq,
        "fp64_krylov": fp64,
        "fp32_krylov_no_refinement": fp32_single,
        "learned_mixed": learned,
        "roofline": {"bound": "hbm", "achieved": loop[dom]["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": loop[dom]["frac"], "traffic": loop[dom]["traffic"],
                     "algorithmic_bytes_per_launch": loop[dom]["algorithmic_bytes_per_launch"],
                     "ms_per_launch": loop[dom]["ms"], "kernel": loop[dom]["kernel"], "source_hash": khash},
        "loop_kernels": loop,
    }
    s.close()
    out["accuracy"] = {"rel_l2_vs_oracle": reference_error(xs, "p5_128_g%g" % m.g),
                       "oracle": "oracle CGLS (C, FP64) to 1e-12 from u = 0; refdata/ref_p5_128_g%g.npy "
                                 "(not in the repository: null when absent; its figure is in profiles/)" % m.g}
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (C oracle, %d CGLS iterations)" % args.cpu_iters, file=sys.stderr, flush=True)
        from oracle.assemble import rhs_isotropic
        out["cpu_baseline"], R = cpu_baseline(m, args.cpu_iters)
        # the FP64 oracle's own residual of the GPU solution (one CPU matvec)
        b = rhs_isotropic(R.layout, m.q00[0])
        out["accuracy"]["oracle_rel_residual"] = float(np.linalg.norm(b - R.matvec(xs)) / np.linalg.norm(b))
        del R
    if not args.no_configs:
        out["configs"] = extra_configs(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
