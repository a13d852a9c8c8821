"""Python handle around the C ABI (include/pn.h).  Marshals torch device
tensors into pointers; every step of the solve runs in the HIP library."""
import ctypes as C

import torch

from . import _lib as L


class PnError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (status %d): %s" % (L.load().pn_status_string(status).decode(), status, msg))
        self.status = status


def _ptr(t, dtype):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if t.dtype != dtype:
        raise TypeError("expected %s, got %s" % (dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def make_grid(dims, h, bc):
    """pn_grid for a boundary type (int: the same on every axis) or a 3-tuple
    of types per axis (x, y, z)."""
    if isinstance(bc, (tuple, list)):
        if len(bc) != 3:
            raise ValueError("bc must be one type or three")
        axes = tuple(int(v) for v in bc)
        code = axes[0] if axes[0] == axes[1] == axes[2] else L.PN_BC_PER_AXIS
    else:
        code, axes = int(bc), (0, 0, 0)
    return L.PnGrid(int(dims[0]), int(dims[1]), int(dims[2]), float(h), code, (C.c_int * 3)(*axes))


class Layout:
    """Staggered SoA layout reported by pn_layout_query."""

    def __init__(self, raw):
        self.order = raw.order
        self.ncoeff = raw.ncoeff
        self.dims = (raw.nx, raw.ny, raw.nz)
        self.bc = raw.bc
        self.bc_axis = tuple(raw.bc_axis)
        self.n = int(raw.n_unknowns)
        self.cls = [tuple(raw.cls[k]) for k in range(self.ncoeff)]
        self.ext = [tuple(raw.ext[k]) for k in range(self.ncoeff)]
        self.offset = [int(raw.offset[k]) for k in range(self.ncoeff + 1)]

    def view(self, vec, k):
        ex, ey, ez = self.ext[k]
        return vec[self.offset[k]:self.offset[k + 1]].view(ez, ey, ex)


class Solver:
    """One medium on one grid: pn_setup ... pn_destroy."""

    def __init__(self, order, dims, sigma_t, albedo, g=0.0, sigma_t_min=0.0, bc=L.PN_BC_VACUUM, h=0.0,
                 stream=None):
        self.lib = L.load()
        st = sigma_t.contiguous()
        al = albedo.contiguous()
        grid = make_grid(dims, h, bc)
        med = L.PnMedium(_ptr(st, torch.float32), _ptr(al, torch.float32), float(g), float(sigma_t_min))
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        ctx = C.c_void_p()
        rc = self.lib.pn_setup(int(order), C.byref(grid), C.byref(med), C.c_void_p(s.cuda_stream), C.byref(ctx))
        if rc != L.PN_OK:
            raise PnError(rc, self.lib.pn_last_error(None).decode())
        self.ctx = ctx
        raw = L.PnLayout()
        self._check(self.lib.pn_layout_query(self.ctx, C.byref(raw)))
        self.layout = Layout(raw)

    def _check(self, rc):
        if rc != L.PN_OK:
            raise PnError(rc, self.lib.pn_last_error(self.ctx).decode())

    @property
    def n(self):
        return self.layout.n

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.pn_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------ kernels --
    def apply(self, x, y=None, transpose=False):
        y = torch.empty_like(x) if y is None else y
        self._check(self.lib.pn_apply(self.ctx, _ptr(x, torch.float32), _ptr(y, torch.float32), int(transpose)))
        return y

    def single_scatter(self, light, power=1.0, out=None):
        """Packed FP32 right-hand side of the single-scattered light of a point
        light at `light` (physical coordinates) with `power` (pn_single_scatter)."""
        q = torch.empty(self.n, dtype=torch.float32, device="cuda") if out is None else out
        pos = (C.c_double * 3)(*[float(v) for v in light])
        self._check(self.lib.pn_single_scatter(self.ctx, pos, float(power), _ptr(q, torch.float32)))
        return q

    def unstagger(self, x):
        """[ncoeff, nz, ny, nx] FP32 coefficients at the voxel centres of the
        packed FP64 solution x (pn_unstagger)."""
        nx, ny, nz = self.layout.dims
        out = torch.empty((self.layout.ncoeff, nz, ny, nx), dtype=torch.float32, device=x.device)
        self._check(self.lib.pn_unstagger(self.ctx, _ptr(x, torch.float64), C.c_void_p(out.data_ptr())))
        return out

    def apply_precond(self, r, variant="schur_mg", z=None):
        """z = B r on the even-band entries (0 elsewhere): the Jacobi (variant
        "schur") or multigrid ("schur_mg") preconditioner of the even-parity
        solve (pn_apply_precond)."""
        z = torch.empty_like(r) if z is None else z
        code = {"schur": 4, "schur_mg": 5}.get(variant, variant)  # or a PN_VARIANT_* code
        self._check(self.lib.pn_apply_precond(self.ctx, code, _ptr(r, torch.float32), _ptr(z, torch.float32)))
        return z

    def apply_schur(self, x, y=None):
        """y_o = -D_o^-1 T_oe x_e and y_e = S x_e (pn_apply_schur); x packed FP32."""
        y = torch.empty_like(x) if y is None else y
        self._check(self.lib.pn_apply_schur(self.ctx, _ptr(x, torch.float32), _ptr(y, torch.float32)))
        return y

    def row_weights(self):
        """Diagonal of W in the equilibrated CG variant (pn_row_weights)."""
        w = torch.empty(self.n, dtype=torch.float32, device="cuda")
        self._check(self.lib.pn_row_weights(self.ctx, _ptr(w, torch.float32)))
        return w

    def apply64(self, x, y=None, transpose=False):
        y = torch.empty_like(x) if y is None else y
        self._check(self.lib.pn_apply64(self.ctx, _ptr(x, torch.float64), _ptr(y, torch.float64), int(transpose)))
        return y

    def residual64(self, rhs, x, r=None):
        rel = C.c_double()
        self._check(self.lib.pn_residual64(self.ctx, _ptr(rhs, torch.float32), _ptr(x, torch.float64),
                                           _ptr(r, torch.float64) if r is not None else None, C.byref(rel)))
        return rel.value

    KERNELS = {"apply": 0, "apply_t": 1, "apply_eq": 2, "supd": 3, "update": 4, "mg_vcycle": 8, "pcg_xp_mg": 9,
               "odd_w": 5, "even_r": 6, "pcg_xp": 7}

    def bench_kernel(self, kernel, iters=20):
        """Mean milliseconds of one launch of a Krylov-loop kernel in its
        in-loop form (pn_bench_kernel): "apply", "apply_t", "apply_eq",
        "supd", "update" (the normal-equation loop) or "odd_w",
        "even_r", "pcg_xp" (the even-parity loop)."""
        ms = C.c_double()
        self._check(self.lib.pn_bench_kernel(self.ctx, self.KERNELS[kernel], int(iters), C.byref(ms)))
        return ms.value

    def bench_apply(self, iters=20, transpose=False):
        """Mean milliseconds of one in-loop FP32 apply (HIP events)."""
        ms = C.c_double()
        self._check(self.lib.pn_bench_apply(self.ctx, int(iters), int(transpose), C.byref(ms)))
        return ms.value

    def attach_net(self, net):
        """Attaches a paper_1807_00410_amd.net.Net (None detaches)."""
        self._net = net
        self._check(self.lib.pn_attach_net(self.ctx, net.n if net is not None else None))

    def net_grid(self):
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        self._check(self.lib.pn_net_grid(self.ctx, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def net_features(self, src):
        nx8, ny8, nz8 = self.net_grid()
        x = torch.empty((1, nz8, ny8, nx8, 32), dtype=torch.bfloat16, device=src.device)
        self._check(self.lib.pn_net_features(self.ctx, _ptr(src, torch.float32), C.c_void_p(x.data_ptr())))
        return x

    def net_targets(self, sol, sub=None):
        """Training target of a packed FP64 solution (of sol - sub when sub is
        given: the remaining correction of a partial iterate)."""
        nx8, ny8, nz8 = self.net_grid()
        t = torch.empty((1, nz8, ny8, nx8, 16), dtype=torch.bfloat16, device=sol.device)
        self._check(self.lib.pn_net_targets_diff(self.ctx, _ptr(sol, torch.float64),
                                                 _ptr(sub, torch.float64) if sub is not None else None,
                                                 C.c_void_p(t.data_ptr())))
        return t

    def autotune(self, iters=10):
        """Times the candidate launch z-chunks, keeps the fastest (also in the
        process-wide tune cache).  Returns (zchunk, ms per apply)."""
        z, ms = C.c_int(), C.c_double()
        self._check(self.lib.pn_autotune(self.ctx, int(iters), C.byref(z), C.byref(ms)))
        return z.value, ms.value

    def set_zchunk(self, z):
        self._check(self.lib.pn_set_zchunk(self.ctx, int(z)))

    def zchunk(self):
        return self.lib.pn_get_zchunk(self.ctx)

    def set_tiles(self, tx, ty, zchunk=0):
        self._check(self.lib.pn_set_tiles(self.ctx, int(tx), int(ty), int(zchunk)))

    def tiles(self):
        tx, ty, z = C.c_int(), C.c_int(), C.c_int()
        self._check(self.lib.pn_get_tiles(self.ctx, C.byref(tx), C.byref(ty), C.byref(z)))
        return tx.value, ty.value, z.value

    def solve(self, rhs, x=None, tol=1e-8, precision="fp32_ir", max_iter=200000, max_refine=40,
              inner_tol=1e-2, use_guess=False, graph_iters=8, variant="auto", learned="off", raise_on_fail=True):
        """Solves A x = rhs.  learned: "off", "guess" or "guess+correct" (needs
        attach_net).  Returns (x, info dict)."""
        if x is None:
            x = torch.zeros(self.n, dtype=torch.float64, device=rhs.device)
        opts = _opts(self.lib, precision, max_iter, max_refine, inner_tol, use_guess, graph_iters, variant)
        opts.learned = {"off": 0, "guess": 1, "guess+correct": 2}[learned]
        info = L.PnSolveInfo()
        rc = self.lib.pn_solve(self.ctx, _ptr(rhs, torch.float32), _ptr(x, torch.float64), float(tol),
                               C.byref(opts), C.byref(info))
        d = _info(rc, info)
        if rc != L.PN_OK and raise_on_fail:
            raise PnError(rc, self.lib.pn_last_error(self.ctx).decode())
        return x, d

    # ---------------------------------------------------------- marshalling --
    def even_unknowns(self):
        """Unknowns of the even bands l (the even-parity solve's vectors)."""
        lay = self.layout
        return sum(lay.offset[k + 1] - lay.offset[k] for k in range(lay.ncoeff) if int(k ** 0.5 + 1e-9) % 2 == 0)

    def rhs_from_q00(self, q00):
        """Right-hand side vector for an isotropic emission Q^{00} per cell
        (coefficient 0 sits at the cell centres; all other entries zero)."""
        rhs = torch.zeros(self.n, dtype=torch.float32, device=q00.device)
        rhs[self.layout.offset[0]:self.layout.offset[1]] = q00.reshape(-1).to(torch.float32)
        return rhs


def _opts(lib, precision, max_iter, max_refine, inner_tol, use_guess, graph_iters, variant):
    opts = L.PnSolveOpts()
    lib.pn_default_opts(C.byref(opts))
    opts.precision = L.PN_FP64 if precision == "fp64" else L.PN_FP32_IR
    opts.max_iter = int(max_iter)
    opts.max_refine = int(max_refine)
    opts.inner_tol = float(inner_tol)
    opts.use_guess = int(bool(use_guess))
    opts.graph_iters = int(graph_iters)
    opts.variant = {"auto": 0, "cgls": 1, "cg": 2, "cg_eq": 3, "schur": 4, "schur_mg": 5}[variant]
    return opts


def _info(rc, info):
    return dict(status=rc, outer_iters=info.outer_iters, inner_iters=info.inner_iters,
                rel_residual=info.rel_residual, bnorm=info.bnorm, seconds=info.seconds,
                history=[info.history[i] for i in range(info.nhistory)],
                learned_steps=info.learned_steps, learned_ratio=info.learned_ratio,
                t_ms={name: info.t_ms[i] for i, name in enumerate(L.PHASES)}, bytes=info.bytes,
                achieved_gbs=info.achieved_gbs)


class Batch:
    """Many media (problems), each with `nrhs` right-hand sides, solved
    together: pn_batch_setup ... pn_batch_destroy.  `problems` is a list of
    (order, dims, sigma_t, albedo, g, sigma_t_min, bc) with device FP32 cell
    arrays."""

    def __init__(self, problems, nrhs, tune=False, h=0.0, stream=None):
        self.lib = L.load()
        n = len(problems)
        arr = (L.PnProblem * n)()
        keep = []
        for i, (order, dims, st, al, g, stmin, bc) in enumerate(problems):
            st = st.contiguous()
            al = al.contiguous()
            keep += [st, al]
            arr[i].order = int(order)
            arr[i].grid = make_grid(dims, h, bc)
            arr[i].medium = L.PnMedium(_ptr(st, torch.float32), _ptr(al, torch.float32), float(g), float(stmin))
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        b = C.c_void_p()
        rc = self.lib.pn_batch_setup(n, arr, int(nrhs), int(bool(tune)), C.c_void_p(s.cuda_stream), C.byref(b))
        if rc != L.PN_OK:
            raise PnError(rc, self.lib.pn_batch_last_error(None).decode())
        self.b = b
        self.nprob = n
        self.nrhs = int(nrhs)
        self.layouts = []
        for i in range(n):
            raw = L.PnLayout()
            self._check(self.lib.pn_batch_layout(self.b, i, C.byref(raw)))
            self.layouts.append(Layout(raw))

    def _check(self, rc):
        if rc != L.PN_OK:
            raise PnError(rc, self.lib.pn_batch_last_error(self.b).decode())

    @property
    def unknowns(self):
        return self.lib.pn_batch_unknowns(self.b)

    def zchunk(self, prob):
        return self.lib.pn_batch_zchunk(self.b, int(prob))

    def net_features(self, prob, src):
        """Network input of problem `prob` for a packed FP32 source vector."""
        ctx = self.lib.pn_batch_problem(self.b, int(prob))
        g = [C.c_int() for _ in range(3)]
        self._check(self.lib.pn_net_grid(ctx, *[C.byref(v) for v in g]))
        nx8, ny8, nz8 = (v.value for v in g)
        x = torch.empty((1, nz8, ny8, nx8, 32), dtype=torch.bfloat16, device=src.device)
        self._check(self.lib.pn_net_features(ctx, _ptr(src, torch.float32), C.c_void_p(x.data_ptr())))
        return x

    def net_targets(self, prob, sol, out=None):
        """Training target of problem `prob` for a packed FP64 solution."""
        ctx = self.lib.pn_batch_problem(self.b, int(prob))
        g = [C.c_int() for _ in range(3)]
        self._check(self.lib.pn_net_grid(ctx, *[C.byref(v) for v in g]))
        nx8, ny8, nz8 = (v.value for v in g)
        t = out if out is not None else torch.empty((1, nz8, ny8, nx8, 16), dtype=torch.bfloat16, device=sol.device)
        self._check(self.lib.pn_net_targets(ctx, _ptr(sol, torch.float64), C.c_void_p(t.data_ptr())))
        return t

    def close(self):
        if getattr(self, "b", None):
            self.lib.pn_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def bench_apply(self, iters=10, transpose=False):
        ms = C.c_double()
        self._check(self.lib.pn_batch_bench_apply(self.b, int(iters), int(transpose), C.byref(ms)))
        return ms.value

    def solve(self, rhs, x=None, tol=1e-8, max_iter=200000, max_refine=40, inner_tol=1e-2, use_guess=False,
              graph_iters=8, variant="auto", raise_on_fail=True):
        """rhs: list over systems (problem-major, nrhs per problem) of device
        FP32 vectors in the problem's packed layout.  Returns (x list, info list)."""
        ns = self.nprob * self.nrhs
        if len(rhs) != ns:
            raise ValueError("expected %d right-hand sides" % ns)
        if x is None:
            x = [torch.zeros(self.layouts[i // self.nrhs].n, dtype=torch.float64, device=rhs[i].device)
                 for i in range(ns)]
        rp = (C.c_void_p * ns)(*[_ptr(r, torch.float32).value for r in rhs])
        xp = (C.c_void_p * ns)(*[_ptr(v, torch.float64).value for v in x])
        opts = _opts(self.lib, "fp32_ir", max_iter, max_refine, inner_tol, use_guess, graph_iters, variant)
        info = (L.PnSolveInfo * ns)()
        rc = self.lib.pn_batch_solve(self.b, rp, xp, float(tol), C.byref(opts), info)
        infos = [_info(info[i].status, info[i]) for i in range(ns)]
        if rc != L.PN_OK and raise_on_fail:
            raise PnError(rc, self.lib.pn_batch_last_error(self.b).decode())
        return x, infos


def tune_cache_save(path):
    rc = L.load().pn_tune_cache_save(str(path).encode())
    if rc != L.PN_OK:
        raise PnError(rc, "cannot write %s" % path)


def tune_cache_load(path):
    rc = L.load().pn_tune_cache_load(str(path).encode())
    if rc != L.PN_OK:
        raise PnError(rc, "cannot read %s" % path)


def tune_cache_size():
    return L.load().pn_tune_cache_size()


def tune_cache_clear():
    L.load().pn_tune_cache_clear()


def coupling_table(order):
    """(k, d, k', value) list compiled into the library for `order`."""
    lib = L.load()
    cap = 1024
    k = (C.c_int * cap)()
    d = (C.c_int * cap)()
    kp = (C.c_int * cap)()
    v = (C.c_double * cap)()
    n = lib.pn_coupling_table(int(order), k, d, kp, v, cap)
    if n < 0:
        raise ValueError("bad order")
    return [(k[i], d[i], kp[i], v[i]) for i in range(n)]
