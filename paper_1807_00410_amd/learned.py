"""Training and evaluation of the learned initial guess / preconditioner.

The data are pairs the solver itself produces: seeded P3 fBm media on a 64^3
grid (the P3 generator: sigma_t = 50 fBm, albedo ~ U[0.8, 0.99], g = 0.3,
Gaussian emission blobs of std 4 cells; or, with --data mixed, a per-medium
extinction scale and point / narrow sources), 8 emission fields each, solved together by
the batched solver; the network input and the target of every solution come
from the library (pn_net_features / pn_net_targets) and the network is
trained by the library's own forward / backward / Adam kernels.  This module
only schedules that work and moves tensors.

    python -m paper_1807_00410_amd.learned --out weights.bin

writes the FP32 parameters (pn_net_save) and prints the training and
evaluation log.
"""
import argparse
import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from synth import config_p3_fbm, config_p3_train, config_p5_nebula  # noqa: E402

from .net import Net  # noqa: E402
from .solver import Batch, Solver  # noqa: E402

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "unet_p3.bin")


def _medium(args):
    n, seed, nrhs, data = args
    if data == "mixed":
        return config_p3_train(n=n, seed=seed, nrhs=nrhs)
    return config_p3_fbm(n=n, seed=seed, order=3, nrhs=nrhs)


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def generate(n=64, nmedia=250, nrhs=8, seed0=1000, chunk=16, tol=1e-5, workers=12, data="p3", log=print):
    """Solves nmedia x nrhs P3 problems; returns (X, T, stats): X [N, n, n, n,
    32] and T [N, n, n, n, 16] bfloat16 on the GPU, sample order shuffled by
    medium."""
    N = nmedia * nrhs
    X = torch.empty((N, n, n, n, 32), dtype=torch.bfloat16, device="cuda")
    T = torch.empty((N, n, n, n, 16), dtype=torch.bfloat16, device="cuda")
    t0 = time.time()
    iters = []
    with ProcessPoolExecutor(max_workers=workers) as ex:
        media_iter = ex.map(_medium, [(n, seed0 + i, nrhs, data) for i in range(nmedia)])
        k = 0
        solve_s = 0.0
        for c0 in range(0, nmedia, chunk):
            media = [next(media_iter) for _ in range(min(chunk, nmedia - c0))]
            probs = [(m.order, m.dims, _dev(m.sigma_t), _dev(m.albedo), m.g, m.sigma_t_min, m.bc) for m in media]
            with Batch(probs, nrhs, tune=(c0 == 0)) as B:
                rhs = []
                for p in range(len(media)):
                    lay = B.layouts[p]
                    for q in media[p].q00:
                        b = torch.zeros(lay.n, dtype=torch.float32, device="cuda")
                        b[lay.offset[0]:lay.offset[1]] = _dev(q).reshape(-1)
                        rhs.append(b)
                ts = time.time()
                xs, infos = B.solve(rhs, tol=tol, raise_on_fail=False, variant="schur_mg")
                solve_s += time.time() - ts
                for i, d in enumerate(infos):
                    if d["status"] != 0:
                        raise RuntimeError("training solve %d did not converge: %s" % (i, d))
                    iters.append(d["inner_iters"])
                for p in range(len(media)):
                    for r in range(nrhs):
                        i = p * nrhs + r
                        X[k] = B.net_features(p, rhs[i])[0]
                        B.net_targets(p, xs[i], out=T[k:k + 1])
                        k += 1
                del xs, rhs
            log("  data: %d/%d samples, %.1f s (batched solves %.1f s, mean %.0f iterations)" % (
                k, N, time.time() - t0, solve_s, float(np.mean(iters))))
    torch.cuda.synchronize()
    return X, T, dict(samples=N, seconds=time.time() - t0, solve_seconds=solve_s, mean_iters=float(np.mean(iters)))


def generate_corrections(n=64, nmedia=64, nrhs=8, seed0=5000, stages=(1e-2, 1e-4), tol=1e-5, workers=12,
                         data="p3", log=print):
    """Correction pairs for the learned refinement step: for every system the
    FP64 residual r_j = Q - A x_j after a partial solve to stages[j] and the
    remaining correction x* - x_j (x* solved to tol).  Returns (X, T, stats)
    as generate(); the residual feeds all 16 source channels."""
    N = nmedia * nrhs * len(stages)
    X = torch.empty((N, n, n, n, 32), dtype=torch.bfloat16, device="cuda")
    T = torch.empty((N, n, n, n, 16), dtype=torch.bfloat16, device="cuda")
    t0 = time.time()
    k = 0
    with ProcessPoolExecutor(max_workers=workers) as ex:
        for m in ex.map(_medium, [(n, seed0 + i, nrhs, data) for i in range(nmedia)]):
            s = Solver(m.order, m.dims, _dev(m.sigma_t), _dev(m.albedo), g=m.g, sigma_t_min=m.sigma_t_min, bc=m.bc)
            r = torch.empty(s.n, dtype=torch.float64, device="cuda")
            for q in m.q00:
                b = s.rhs_from_q00(_dev(q))
                parts = [s.solve(b, tol=st, raise_on_fail=False)[0] for st in stages]
                xs, d = s.solve(b, x=parts[-1].clone(), tol=tol, use_guess=True)
                for xj in parts:
                    s.residual64(b, xj, r)
                    X[k] = s.net_features(r.float())[0]
                    T[k] = s.net_targets(xs, sub=xj)[0]
                    k += 1
            s.close()
            if k % (nrhs * len(stages) * 16) == 0:
                log("  corrections: %d/%d samples, %.1f s" % (k, N, time.time() - t0))
    torch.cuda.synchronize()
    return X, T, dict(samples=N, seconds=time.time() - t0)


def train(net, X, T, epochs=10, batch=4, lr=2e-3, val=16, seed=0, log=print):
    """Adam with a cosine learning-rate decay; the last `val` samples are held
    out for the validation loss.  Batches are contiguous runs of samples, in a
    fresh random order every epoch."""
    N = X.shape[0] - val
    nb = N // batch
    total = epochs * nb
    rng = np.random.default_rng(seed)
    step = 0
    hist = []
    t0 = time.time()
    for ep in range(epochs):
        losses = []
        for b in rng.permutation(nb):
            s = int(b) * batch
            lr_t = lr * 0.5 * (1.0 + math.cos(math.pi * step / total))
            losses.append(net.train_step(X[s:s + batch], T[s:s + batch], lr_t))
            step += 1
        vl = [net.train_step(X[i:i + 1], T[i:i + 1], 0.0) for i in range(N, N + val)]
        hist.append((float(np.mean(losses)), float(np.mean(vl))))
        log("  epoch %2d: train loss %.3e  validation loss %.3e  (%.1f s)" % (ep, hist[-1][0], hist[-1][1],
                                                                            time.time() - t0))
    return hist


def evaluate(net, cases, tol=1e-8, log=print):
    """Plain solve against the learned guess and guess+correction."""
    out = {}
    for name, m in cases:
        s = Solver(m.order, m.dims, _dev(m.sigma_t), _dev(m.albedo), g=m.g, sigma_t_min=m.sigma_t_min, bc=m.bc)
        rhs = s.rhs_from_q00(_dev(m.q00[0]))
        s.solve(rhs, tol=1e-3)  # warm-up (graph capture, network buffers)
        s.attach_net(net)
        s.solve(rhs, tol=1e-3, learned="guess")
        res = {}
        for mode in ("off", "guess", "guess+correct"):
            x, d = s.solve(rhs, tol=tol, learned=mode)
            res[mode] = dict(iters=d["inner_iters"], outer=d["outer_iters"], seconds=d["seconds"],
                             learned_steps=d["learned_steps"], guess_ratio=d["learned_ratio"],
                             rel_residual=d["rel_residual"])
            log("  %-22s %-14s iters %5d  outer %2d  learned steps %d  guess residual ratio %.3f  %.3f s" % (
                name, mode, d["inner_iters"], d["outer_iters"], d["learned_steps"], d["learned_ratio"],
                d["seconds"]))
        out[name] = res
        s.attach_net(None)
        s.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--media", type=int, default=250)
    ap.add_argument("--nrhs", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--eval", action="store_true", help="evaluate on held-out P3 96^3 and P5 128^3 media")
    ap.add_argument("--corrections", type=int, default=0,
                    help="media whose partially solved residuals add (residual -> correction) samples")
    ap.add_argument("--data", choices=("p3", "mixed"), default="p3",
                    help="p3: the P3 fBm generator (sigma_t 50 fBm, blobs of std 4 cells); mixed: per-medium "
                         "extinction scale and point / narrow sources")
    args = ap.parse_args()
    log = lambda *a: print(*a, flush=True)
    log("generating %d x %d P3 %d^3 samples" % (args.media, args.nrhs, args.n))
    X, T, st = generate(n=args.n, nmedia=args.media, nrhs=args.nrhs, data=args.data, log=log)
    if args.corrections > 0:
        log("generating correction samples from %d media" % args.corrections)
        Xc, Tc, _ = generate_corrections(n=args.n, nmedia=args.corrections, nrhs=args.nrhs, data=args.data, log=log)
        # the validation tail stays a guess sample set; corrections go in front
        X = torch.cat([Xc, X])
        T = torch.cat([Tc, T])
        del Xc, Tc
    net = Net(seed=1)
    log("training: %d epochs, batch %d, lr %g" % (args.epochs, args.batch, args.lr))
    train(net, X, T, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    net.save(args.out)
    log("saved %s" % args.out)
    del X, T
    torch.cuda.empty_cache()
    if args.eval:
        cases = [("P3 96^3 fBm s90002", config_p3_fbm(n=96, seed=90002, order=3)),
                 ("P5 128^3 nebula g=0", config_p5_nebula(n=128, seed=3, g=0.0))]
        evaluate(net, cases, log=log)
    net.close()


if __name__ == "__main__":
    main()
