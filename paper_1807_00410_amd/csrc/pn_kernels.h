// HIP kernels of the staggered real P_N solver (gfx950).
//
// Stencil apply (matrix-free A x, A^T x).  One thread owns one (x, y) column
// of the staggered lattice and marches a chunk of z planes.  Per input
// coefficient it keeps a two-plane register window in z (the plane above for
// z-face classes, the plane below for z-centred ones), so every vector entry
// is fetched from memory once for its own row and the z-difference; the x/y
// neighbours are re-reads of lines that adjacent lanes / rows already pulled
// into L1/L2.  The RTE parameters (sigma_t, albedo per cell, 8 bytes) are
// averaged on the fly from the 1/2/4/8 cells adjacent to each staggered
// location, with the previous plane of cells kept in registers.
//
// The coupling structure is a compile-time table (pn_tables.h), so the
// per-class bookkeeping, the differences and the coupling weights unroll into
// straight-line FMA code with literal constants.
//
// Krylov bookkeeping: dot products are accumulated in FP64 per thread,
// reduced per wavefront with cross-lane shuffles, per block through LDS in a
// fixed order, and per grid by a one-block finalize kernel that also forms
// the CGLS scalars on the device (no host round trip per iteration).
#pragma once
#include <hip/hip_runtime.h>

#include <utility>

#include "pn_tables.h"

namespace pn {

constexpr int kBlock = 256;
constexpr int kMaxCoeff = 64;

// Minimum waves per SIMD the stencil kernels are compiled for (caps VGPRs).
#ifndef PN_STENCIL_WPE
#define PN_STENCIL_WPE 1
#endif

// ------------------------------------------------------------------ state --
struct DevState {
  double gamma;   // ||s||^2 of the current normal-equation residual s = A^T r
  double alpha;   // step length
  double beta;    // direction update factor
  double rr;      // ||r||^2 of the (recursive) residual
  double rr0;     // ||r||^2 at the start of the current inner solve
  double tol2;    // inner stop threshold on rr
  double qq;      // ||A p||^2
  double rtrue2;  // ||Q - A x||^2 from the FP64 residual kernel
  double bb2;     // ||Q||^2
  double nonfinite;
  double itol2;   // batch: squared relative tolerance of the next inner solve
  double rzf;     // multigrid PCG: <r, M r> of the current residual (its Jacobi part)
  int iters;      // Krylov iterations so far (all inner solves)
  int max_iters;
  int stop;       // set when the iteration must end after this step's update
  int done;       // set one step later: every kernel returns at once
  int breakdown;
  int frozen;     // batch: the system is finished; every kernel skips it
  int pad[2];
};

// M_SUPD: s <- s - alpha * op(x) (the normal-equation residual update of CG
// on A^T A).  M_APPLY_EQ / M_EQS: the row-equilibrated forms (w = 1 / ||row
// of A||^2 per unknown, formed from the medium in the kernel).
enum Mode {
  M_APPLY = 0, M_TRANSR = 1, M_RESID = 2, M_SUPD = 3, M_APPLY_EQ = 4, M_EQS = 5,
  // even-parity (Schur complement) solve, rows of one band parity only
  M_ODD_W = 6, M_EVEN_S = 7, M_EVEN_RHS = 8, M_ODD_BACK = 9, M_EVEN_JAC = 10, M_EVEN_SR = 11
};

// Band parity of the rows a mode computes: 0 all, 1 even l, 2 odd l.  The
// band parity of a coefficient is the parity of its staggering class
// (px + py + pz): even bands sit at cell centres and edges, odd ones on faces
// and corners, and the transport couples only bands l and l +- 1, so A is
// [[D_e, T_eo], [T_oe, D_o]] with D_e, D_o diagonal (and T_oe = -T_eo^T when
// no axis is Neumann).
constexpr int mode_rows(int m) {
  return (m == M_EVEN_S || m == M_EVEN_RHS || m == M_EVEN_JAC || m == M_EVEN_SR) ? 1
         : (m == M_ODD_W || m == M_ODD_BACK) ? 2 : 0;
}
constexpr int class_parity(int c) { return ((c & 1) + ((c >> 1) & 1) + ((c >> 2) & 1)) & 1; }

// Internal vectors live on a padded lattice shared by every coefficient:
// coefficient k occupies [k*cs, (k+1)*cs); lattice point (x, y, z) of any
// class sits at ((z+1)*PY + (y+1))*PX + (x+1) with PX = Ex + 2, PY = Ey + 2,
// where Ex = nx + 1 (vacuum / Neumann along x) or nx (periodic along x).
// Entries outside a coefficient's class extent -- the one-point halo and, for
// a class centred along d, the position x_d = n_d -- are zero and stay zero:
// kernels never store there and every element-wise update maps 0 to 0.
// That makes every neighbour load unconditional (vacuum: an out-of-domain read
// hits a zero).  Cells are padded the same way, their halo holding clamped
// (vacuum, Neumann) or wrapped (periodic) copies, so the parameter reads need
// no clamping either.
//
// Boundary types per axis (BC_*): vacuum = the paper's Dirichlet mode (an
// entry referencing a location outside the domain is dropped: the zero halo);
// periodic = wrap-around; Neumann = the entry moves to the coefficient at the
// closest location inside the domain (section "Runtime").  Only the
// differences of face-centred rows on a boundary face reach outside, and there
// the two samples of the centred input land on the same coefficient, so under
// Neumann those differences vanish from A; in A^T the face values on the two
// boundary faces drop out of the differences of the centred rows next to them.
enum { BC_VACUUM = 0, BC_PERIODIC = 1, BC_NEUMANN = 2 };
struct StencilArgs {
  int nx, ny, nz;
  int Ex, Ey, Ez;      // lattice points per axis
  int PX, PY, plane;   // padded pitches of a coefficient array, plane = PX*PY
  int CX, cplane;      // padded cell pitches: CX = nx + 2, cplane = CX*(ny + 2)
  long long cs;        // coefficient stride (elements)
  int zchunk, nzc, ncb, nblocks;
  int bcx, bcy, bcz;   // boundary type per axis (the general-boundary kernels)
  double invh;         // 1 / h
  double tsign;        // +1: A, -1: A^T
  double omg[8];       // 1 - g^l, l = 0..7
  const float2* med32; // padded cells (sigma_a, sigma_s) in FP32
  const float2* med;   // padded cells (sigma_t, albedo) as given (FP64 kernels)
  const uint16_t* m16; // M_EVEN_SR: bfloat16 preconditioner on the padded lattice
  const void* x;       // input vector (T); M_TRANSR: r
  const void* x2;      // M_TRANSR: q;  M_RESID: right-hand side (float)
  void* y;             // output vector
  void* y2;            // M_TRANSR: updated r
  DevState* st;        // device scalars (alpha for M_TRANSR, stop/done flags), may be null
  double* partials;    // [nblocks][2] FP64 partial sums, may be null
  // LDS-tiled kernel only: tile of TX x TY columns, ntx x nty tiles per plane
  int TX, TY, ntx, nty;
};

template <class F, int... I>
__device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// Blocks are handed to the 8 XCDs round-robin; give each XCD a contiguous
// range of logical tiles so neighbouring columns / chunks share an L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int xcd = b & 7, slot = b >> 3;
  return (xcd < r) ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Access at a uniform base pointer plus a 32-bit byte offset (lets the
// compiler use the scalar-base + vector-offset addressing mode).
template <typename U>
__device__ __forceinline__ U ldb(const U* base, unsigned boff) {
  return *reinterpret_cast<const U*>(reinterpret_cast<const char*>(base) + boff);
}
template <typename U>
__device__ __forceinline__ void stb(U* base, unsigned boff, U v) {
  *reinterpret_cast<U*>(reinterpret_cast<char*>(base) + boff) = v;
}

template <typename T>
__device__ __forceinline__ T fmadd(T a, T b, T c);
template <>
__device__ __forceinline__ float fmadd<float>(float a, float b, float c) { return __fmaf_rn(a, b, c); }
template <>
__device__ __forceinline__ double fmadd<double>(double a, double b, double c) { return __fma_rn(a, b, c); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Deterministic block sum of two FP64 values; result valid in thread 0.
__device__ __forceinline__ void block_sum2(double& a, double& b) {
  __shared__ double red[2][kBlock / 64];
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) { red[0][w] = a; red[1][w] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) { s0 += red[0][i]; s1 += red[1][i]; }
    a = s0; b = s1;
  }
}

// --------------------------------------------------------------- stencil --
// T: arithmetic / vector type of the input (float or double).  TO: output
// element type.  GEN: general boundary types per axis (a.bcx, a.bcy, a.bcz);
// otherwise vacuum on every axis.  NORM: write the FP64 block partial
// sums of the squares below to a.partials (per thread, squares are summed in
// T over the rows of one class -- at most 10 terms -- then added in FP64).
//   M_APPLY  y = op(x)                         [||y||^2]
//   M_TRANSR r' = r - alpha q, y = A^T r'      [writes r' to y2; ||y||^2, ||r'||^2]
//   M_RESID  y = Q - A x                       [||y||^2, ||Q||^2]
//   M_SUPD   y = y - alpha op(x)               [||y||^2]
//   M_APPLY_EQ  y = W A x                      [<A x, W A x>]
//   M_EQS    y = W x                           [<x, W x>]
// Even-parity Schur complement S = D_e - T_eo D_o^-1 T_oe (rows of one band
// parity; T the transport part of A, (T x) on those rows reads only the other
// parity of x):
//   M_ODD_W    y_o = -(T x)_o / d_o            (x even: p_e)
//              [NORM: <x_e, D_e x_e> + <y_o, D_o y_o> = <p_e, S p_e>]
//   M_EVEN_S   y_e = d_e x_e + (T x)_e         [<x_e, y_e>]  (x odd: w_o)
//   M_EVEN_SR  q_e = d_e x_e + (T x)_e, y_e -= alpha q_e   (y: the PCG
//              residual r; m: the bfloat16 preconditioner)
//              [<y_e, m y_e>, <y_e, y_e>]
//   M_EVEN_RHS y_e = x2_e - (T x)_e            (x odd: D_o^-1 r_o; x2: r)
//   M_ODD_BACK y_o = (x2_o - (T x)_o) / d_o    (x even: d_e; x2: r)
//   M_EVEN_JAC y_e = 1 / (d_e + sum over the row's transport entries (T)_ij^2 x_j)
//              (x odd: 1 / d_o): the inverse diagonal of S
// W is diagonal: w = 1 / (d^2 + sum of the squared transport entries of the
// row), d the row's diagonal -- the inverse squared 2-norm of the row of A
// away from the boundary.
template <int N, typename T, int MODE, typename TO, bool GEN, bool NORM>
__device__ __forceinline__ void stencil_body(const StencilArgs& a, const int L) {
  using TB = Table<N>;
  constexpr int NC = TB::NC;
  const int cb = L % a.ncb, zc = L / a.ncb;
  const int col = cb * kBlock + threadIdx.x;
  const bool act = col < a.Ex * a.Ey;
  const int x = act ? col % a.Ex : 0;
  const int y = act ? col / a.Ex : 0;
  const int z0 = zc * a.zchunk;
  const int z1 = min(z0 + a.zchunk, a.Ez);

  const T* __restrict__ X = static_cast<const T*>(a.x);
  const T* __restrict__ X2 = static_cast<const T*>(a.x2);
  const float* __restrict__ RHS = static_cast<const float*>(a.x2);
  TO* __restrict__ Y = static_cast<TO*>(a.y);
  TO* __restrict__ Y2 = static_cast<TO*>(a.y2);
  T alpha = T(0);
  if constexpr (MODE == M_TRANSR || MODE == M_SUPD || MODE == M_EVEN_SR) alpha = T(a.st->alpha);
  const T tinvh = T(a.tsign * a.invh);
  const T invh2 = T(a.invh * a.invh);
  const long long cs = a.cs;

  // Lane offsets inside a padded plane (own point and the four in-plane
  // neighbours), kept as 32-bit BYTE offsets: every access is then a uniform
  // 64-bit base (coefficient, plane) in SGPRs plus one 32-bit VGPR offset.
  const bool perx = GEN && a.bcx == BC_PERIODIC, pery = GEN && a.bcy == BC_PERIODIC;
  const bool perz = GEN && a.bcz == BC_PERIODIC;
  unsigned o, oxp, oxm, oyp, oym;
  {
    const int oi = (y + 1) * a.PX + (x + 1);
    int ixp = oi + 1, ixm = oi - 1, iyp = oi + a.PX, iym = oi - a.PX;
    if constexpr (GEN) {
      if (perx) {
        ixp = (y + 1) * a.PX + (x + 1 == a.nx ? 0 : x + 1) + 1;
        ixm = (y + 1) * a.PX + (x == 0 ? a.nx - 1 : x - 1) + 1;
      }
      if (pery) {
        iyp = ((y + 1 == a.ny ? 0 : y + 1) + 1) * a.PX + x + 1;
        iym = ((y == 0 ? a.ny - 1 : y - 1) + 1) * a.PX + x + 1;
      }
    }
    o = (unsigned)oi * (unsigned)sizeof(T);
    oxp = (unsigned)ixp * (unsigned)sizeof(T);
    oxm = (unsigned)ixm * (unsigned)sizeof(T);
    oyp = (unsigned)iyp * (unsigned)sizeof(T);
    oym = (unsigned)iym * (unsigned)sizeof(T);
  }
  const unsigned oo = o / (unsigned)sizeof(T) * (unsigned)sizeof(TO);  // own point, output type
  const unsigned orhs = o / (unsigned)sizeof(T) * 4u;                 // own point, float rhs
  // padded cell (x-1, y-1) of a cell plane, bytes
  const unsigned mo = (unsigned)(y * a.CX + x) * (unsigned)sizeof(float2);
  const unsigned mcx = (unsigned)a.CX * (unsigned)sizeof(float2);
  const bool okx0 = perx || x < a.nx;  // store predicate of classes centred in x
  const bool oky0 = pery || y < a.ny;
  // Neumann weights of the differences along x and y (1 elsewhere): A drops
  // the backward difference of face rows on a boundary face (nb); A^T drops
  // the boundary-face samples from the forward difference of centred rows
  // (nl: the face below the row, nh: the face above it)
  T nbx = T(1), nlx = T(1), nhx = T(1), nby = T(1), nly = T(1), nhy = T(1);
  if constexpr (GEN) {
    const bool fwd = a.tsign > 0.0;
    if (a.bcx == BC_NEUMANN) {
      if (fwd) nbx = (x == 0 || x == a.nx) ? T(0) : T(1);
      else { nlx = x == 0 ? T(0) : T(1); nhx = x + 1 == a.nx ? T(0) : T(1); }
    }
    if (a.bcy == BC_NEUMANN) {
      if (fwd) nby = (y == 0 || y == a.ny) ? T(0) : T(1);
      else { nly = y == 0 ? T(0) : T(1); nhy = y + 1 == a.ny ? T(0) : T(1); }
    }
  }

  // padded plane offset (elements) of lattice plane z (periodic planes wrap)
  // The offset goes through readfirstlane: it is uniform anyway, and the
  // opaque value keeps loop strength reduction from turning every one of the
  // ~100 address streams into its own 64-bit induction variable in VGPRs.
  auto zoff = [&](int z) -> long long {
    if (perz) z = wrapi(z, a.nz);
    return (long long)__builtin_amdgcn_readfirstlane((z + 1) * a.plane);
  };
  // Element offset of (coefficient, plane) as an opaque uniform 32-bit value:
  // recomputed with two scalar ops per use instead of ~36 loop-invariant 64-bit
  // bases being hoisted out of the z loop and spilled into vector registers.
  auto cbase = [&](int k, long long zo) -> long long {
    return (long long)__builtin_amdgcn_readfirstlane((int)((long long)k * cs + zo));
  };
  auto load = [&](auto KPc, long long zo, unsigned lo) -> T {
    constexpr int KP = decltype(KPc)::value;
    const long long base = cbase(KP, zo);
    if constexpr (MODE == M_TRANSR) return fmadd<T>(-alpha, ldb(X2 + base, lo), ldb(X + base, lo));
    else return ldb(X + base, lo);
  };
  const float2* __restrict__ MED = (sizeof(T) == 4) ? a.med32 : a.med;
  auto cells = [&](int z, T* sa, T* ss) {  // 4 cells (x-1|x, y-1|y) of cell plane z
    const float2* __restrict__ mp = MED + (long long)(z + 1) * a.cplane;
    const float2 c[4] = {ldb(mp, mo), ldb(mp, mo + 8u), ldb(mp, mo + mcx), ldb(mp, mo + mcx + 8u)};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if constexpr (sizeof(T) == 4) {
        sa[q] = c[q].x; ss[q] = c[q].y;
      } else {  // exact in FP64: sigma_t (1 - albedo), sigma_t albedo
        sa[q] = T(c[q].x) * (T(1) - T(c[q].y));
        ss[q] = T(c[q].x) * T(c[q].y);
      }
    }
  };

  double nrm0 = 0.0, nrm1 = 0.0;
  // coefficients whose window is kept: every one, or for the one-parity
  // modes the other parity (their transport inputs) and, for M_EVEN_S, the
  // rows' own values
  constexpr int kRows = mode_rows(MODE);
  constexpr auto in_window = [](int K) constexpr {
    return kRows == 0 || class_parity(cls_id(K)) != kRows - 1 || MODE == M_EVEN_S || MODE == M_EVEN_SR;
  };
  {  // lanes past the last column recompute column 0 and store nothing
    T cur[NC], nb[NC];
    {
      const long long zo0 = zoff(z0), zom = zoff(z0 - 1);
      sfor<NC>([&](auto KPc) {
        constexpr int KP = decltype(KPc)::value;
        if constexpr (in_window(KP)) {
          if constexpr (cls_z(KP) == 1) nb[KP] = load(KPc, zo0, o);
          else cur[KP] = load(KPc, zom, o);
        }
      });
    }
    T msa[8], mss[8];  // cells of the plane below (0..3) and of this plane (4..7)
    cells(perz ? wrapi(z0 - 1, a.nz) : z0 - 1, msa, mss);

#pragma clang loop unroll(disable)
    for (int z = z0; z < z1; ++z) {
      const long long zo = zoff(z), zon = zoff(z + 1);
      sfor<NC>([&](auto KPc) {
        constexpr int KP = decltype(KPc)::value;
        if constexpr (in_window(KP)) {
          if constexpr (cls_z(KP) == 1) { cur[KP] = nb[KP]; nb[KP] = load(KPc, zon, o); }
          else { nb[KP] = cur[KP]; cur[KP] = load(KPc, zo, o); }
        }
      });
      cells(z, msa + 4, mss + 4);
      // Class means of sigma_a and sigma_s (cells visited z-major, lower
      // neighbour first).  The row diagonal sigma_t - g^l sigma_s is formed as
      // mean(sigma_a) + (1 - g^l) mean(sigma_s): the same number without the
      // cancellation of sigma_t - sigma_s at albedo close to 1.
      T csa[8], css[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int px = c & 1, py = (c >> 1) & 1, pz = (c >> 2) & 1;
        T s0 = T(0), s1 = T(0);
        int cnt = 0;
#pragma unroll
        for (int dz = 1 - pz; dz < 2; ++dz)
#pragma unroll
          for (int dy = 1 - py; dy < 2; ++dy)
#pragma unroll
            for (int dx = 1 - px; dx < 2; ++dx) {
              s0 += msa[4 * dz + 2 * dy + dx];
              s1 += mss[4 * dz + 2 * dy + dx];
              ++cnt;
            }
        const T inv = T(1) / T(cnt);
        csa[c] = s0 * inv;
        css[c] = s1 * inv;
      }

      // Rows one staggering class at a time: form each (input, axis)
      // difference once, fan it out to the rows of the class, store them.
      const bool okz0 = perz || z < a.nz;
      T nbz = T(1), nlz = T(1), nhz = T(1);  // Neumann weights along z (as for x, y)
      if constexpr (GEN) {
        if (a.bcz == BC_NEUMANN) {
          if (a.tsign > 0.0) nbz = (z == 0 || z == a.nz) ? T(0) : T(1);
          else { nlz = z == 0 ? T(0) : T(1); nhz = z + 1 == a.nz ? T(0) : T(1); }
        }
      }
      sfor<8>([&](auto Cc) {
        constexpr int c = decltype(Cc)::value;
        if constexpr (TB::class_has_rows(c) && (kRows == 0 || class_parity(c) == kRows - 1)) {
#ifdef PN_CLASS_BARRIER
          // keep each class group's loads from being hoisted above the previous
          // group (bounds the live registers)
          __builtin_amdgcn_sched_barrier(0);
#endif
          constexpr int ib = TB::class_begin(c);
          constexpr int ie = TB::class_end(c);
          T acc[NC];
          sfor<NC>([&](auto Kc) {
            constexpr int K = decltype(Kc)::value;
            if constexpr (cls_id(K) == c) acc[K] = T(0);
          });
          // M_SUPD: the class's old outputs are loaded before its differences
          // are formed, so their latency hides behind that work
          T yold[NC];
          if constexpr (MODE == M_SUPD || MODE == M_EVEN_SR) {
            sfor<NC>([&](auto Kc) {
              constexpr int K = decltype(Kc)::value;
              if constexpr (cls_id(K) == c) yold[K] = T(ldb(Y + cbase(K, zo), oo));
            });
          }
          T dcur = T(0);
          sfor<ie - ib>([&](auto Ic) {
            constexpr int I = ib + decltype(Ic)::value;
            constexpr Coupling cp = TB::cpl.v[I];
            constexpr bool first = TB::starts_difference(I);
            if constexpr (first) {
              constexpr int p = cls_axis(cp.kp, cp.d);
              if constexpr (MODE == M_EVEN_JAC) {  // the two samples summed (squared couplings)
                if constexpr (cp.d == 2) {
                  dcur = nb[cp.kp] + cur[cp.kp];
                } else {
                  const unsigned lo = (cp.d == 0) ? (p ? oxp : oxm) : (p ? oyp : oym);
                  dcur = load(std::integral_constant<int, cp.kp>{}, zo, lo) + cur[cp.kp];
                }
              } else if constexpr (cp.d == 2) {
                if constexpr (GEN) dcur = p ? nhz * nb[cp.kp] - nlz * cur[cp.kp] : nbz * (cur[cp.kp] - nb[cp.kp]);
                else dcur = p ? nb[cp.kp] - cur[cp.kp] : cur[cp.kp] - nb[cp.kp];
              } else {
                const unsigned lo = (cp.d == 0) ? (p ? oxp : oxm) : (p ? oyp : oym);
                const T v = load(std::integral_constant<int, cp.kp>{}, zo, lo);
                if constexpr (GEN) {
                  const T nh = cp.d == 0 ? nhx : nhy, nl = cp.d == 0 ? nlx : nly, nbb = cp.d == 0 ? nbx : nby;
                  dcur = p ? nh * v - nl * cur[cp.kp] : nbb * (cur[cp.kp] - v);
                } else {
                  dcur = p ? v - cur[cp.kp] : cur[cp.kp] - v;
                }
              }
            }
            if constexpr (MODE == M_EVEN_JAC) acc[cp.k] = fmadd<T>(T(cp.c * cp.c), dcur, acc[cp.k]);
            else acc[cp.k] = fmadd<T>(T(cp.c), dcur, acc[cp.k]);
          });
          constexpr int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
          const bool ok = act && (cx || okx0) && (cy || oky0) && (cz || okz0);
          if (ok) {
            // squares summed per class in T, promoted to FP64 once per class
            T cn0 = T(0), cn1 = T(0);
            sfor<NC>([&](auto Kc) {
              constexpr int K = decltype(Kc)::value;
              if constexpr (cls_id(K) == c) {
                const long long base = cbase(K, zo);
                const T dg = fmadd<T>(T(a.omg[band_of(K)]), css[c], csa[c]);
                T out;
                if constexpr (MODE == M_ODD_W) out = -(tinvh * acc[K]) / dg;
                else if constexpr (MODE == M_EVEN_RHS) out = T(ldb(X2 + base, o)) - tinvh * acc[K];
                else if constexpr (MODE == M_ODD_BACK)  // x2 == NULL reads as 1 (then y_o = 1 / d_o for x = 0)
                  out = ((X2 != nullptr ? T(ldb(X2 + base, o)) : T(1)) - tinvh * acc[K]) / dg;
                else if constexpr (MODE == M_EVEN_JAC) out = T(1) / fmadd<T>(invh2, acc[K], dg);
                else out = fmadd<T>(tinvh, acc[K], dg * cur[K]);
                if constexpr (MODE == M_EQS) out = cur[K];
                if constexpr (MODE == M_APPLY_EQ || MODE == M_EQS) {
                  constexpr T rc2 = T(TB::row_c2(K));
                  const T w = __builtin_amdgcn_rcpf(fmadd<T>(dg, dg, invh2 * rc2));
                  const T wo = w * out;
                  cn0 = fmadd<T>(wo, out, cn0);
                  out = wo;
                }
                if constexpr (MODE == M_RESID) {
                  const T q = T(ldb(RHS + base, orhs));
                  out = q - out;
                  cn1 = fmadd<T>(q, q, cn1);
                }
                if constexpr (MODE == M_SUPD || MODE == M_EVEN_SR) out = fmadd<T>(-alpha, out, yold[K]);
                stb(Y + base, oo, TO(out));
                if constexpr (MODE == M_EVEN_SR) {
                  const T mk = T(__uint_as_float((uint32_t)ldb(a.m16 + base, o / (unsigned)sizeof(T) * 2u) << 16));
                  cn0 = fmadd<T>(mk * out, out, cn0);
                  cn1 = fmadd<T>(out, out, cn1);
                } else if constexpr (MODE == M_ODD_W) {
                  cn0 = fmadd<T>(dg * out, out, cn0);  // <w_o, D_o w_o>
                } else if constexpr (MODE == M_EVEN_S) cn0 = fmadd<T>(cur[K], out, cn0);
                else if constexpr (NORM && MODE != M_APPLY_EQ && MODE != M_EQS) cn0 = fmadd<T>(out, out, cn0);
                if constexpr (MODE == M_TRANSR) {
                  stb(Y2 + base, oo, TO(cur[K]));
                  cn1 = fmadd<T>(cur[K], cur[K], cn1);
                }
              }
            });
            if constexpr (NORM) nrm0 += double(cn0);
            if constexpr (MODE == M_TRANSR || MODE == M_RESID || MODE == M_EVEN_SR) nrm1 += double(cn1);
          }
        }
      });
      // M_ODD_W: <p_e, D_e p_e> over this thread's even points of the plane
      // (with <w_o, D_o w_o> above: <p, S p>, since T_oe = -T_eo^T)
      if constexpr (MODE == M_ODD_W && NORM) {
        T ce = T(0);
        sfor<NC>([&](auto Kc) {
          constexpr int K = decltype(Kc)::value;
          constexpr int c = cls_id(K);
          if constexpr (class_parity(c) == 0) {
            constexpr int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
            const bool okk = act && (cx || okx0) && (cy || oky0) && (cz || okz0);
            const T dg = fmadd<T>(T(a.omg[band_of(K)]), css[c], csa[c]);
            ce = okk ? fmadd<T>(dg * cur[K], cur[K], ce) : ce;
          }
        });
        nrm0 += double(ce);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) { msa[q] = msa[4 + q]; mss[q] = mss[4 + q]; }
    }
  }

  if constexpr (NORM) {
    block_sum2(nrm0, nrm1);
    if (threadIdx.x == 0) {
      a.partials[2 * L] = nrm0;
      a.partials[2 * L + 1] = nrm1;
    }
  }
}

template <int N, typename T, int MODE, typename TO, bool GEN, bool NORM>
__global__ void __launch_bounds__(kBlock, PN_STENCIL_WPE) k_stencil(const StencilArgs a) {
  // In the Krylov loop the A p launch also ends once the stop flag is up.
  if (a.st != nullptr &&
      (a.st->done || ((MODE == M_APPLY || MODE == M_APPLY_EQ || MODE == M_ODD_W || MODE == M_EVEN_S) && a.st->stop)))
    return;
  stencil_body<N, T, MODE, TO, GEN, NORM>(a, xcd_remap(blockIdx.x, a.nblocks));
}

// ---------------------------------------------------------------- batch --
// Many systems (problem x right-hand side) in one launch.  Each block takes a
// work item (system, tile) from a list ordered problem-major, then tile, then
// right-hand side, so the blocks of one tile for the different right-hand
// sides of a problem run next to each other on one XCD and share the cell
// parameters through its L2.  A system's vectors are addressed by role
// through its vector table.
enum BatchVec { BV_R0 = 0, BV_R1, BV_S, BV_P, BV_Q, BV_D, BV_B, BV_X64, BV_COUNT };

struct SysArgs {
  StencilArgs a;        // geometry and medium of the problem; st, partials of the system
  void* vec[BV_COUNT];  // padded vectors of the system
  long long nv;         // padded vector length
  double itol2;         // squared relative inner tolerance of the current inner solve
};

struct BatchLaunch {
  const SysArgs* sys;
  const int2* work;     // (system, tile) per block
  int nwork;
  int ix, ix2, iy, iy2; // vector roles (-1: unused)
  double tsign;
  int gate;             // 1: skip systems whose inner solve stopped (Krylov loop)
};

template <int N, typename T, int MODE, typename TO, bool GEN, bool NORM>
__global__ void __launch_bounds__(kBlock, PN_STENCIL_WPE) k_stencil_batch(const BatchLaunch bl) {
  const int2 w = bl.work[xcd_remap(blockIdx.x, bl.nwork)];
  const SysArgs* __restrict__ s = bl.sys + w.x;
  DevState* st = s->a.st;
  if (st->frozen || (bl.gate && (st->done || ((MODE == M_APPLY || MODE == M_APPLY_EQ) && st->stop)))) return;
  StencilArgs a = s->a;
  a.x = s->vec[bl.ix];
  a.x2 = bl.ix2 >= 0 ? s->vec[bl.ix2] : nullptr;
  a.y = s->vec[bl.iy];
  a.y2 = bl.iy2 >= 0 ? s->vec[bl.iy2] : nullptr;
  a.tsign = bl.tsign;
  stencil_body<N, T, MODE, TO, GEN, NORM>(a, w.y);
}

// ------------------------------------------------------------- finalize --
// Sum of partials[2*i + j] over i < n in a fixed order by one block of
// kFinBlock threads; the sums are valid in thread 0 (the only reader).
constexpr int kFinBlock = 1024;
__device__ __forceinline__ void grid_sum2(const double* __restrict__ p, int n, double& s0, double& s1) {
  double a = 0.0, b = 0.0;
  const double2* __restrict__ p2 = reinterpret_cast<const double2*>(p);
#pragma unroll 4
  for (int i = threadIdx.x; i < n; i += kFinBlock) {
    const double2 v = p2[i];
    a += v.x;
    b += v.y;
  }
  a = wave_sum(a);
  b = wave_sum(b);
  __shared__ double red[2][kFinBlock / 64];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { red[0][w] = a; red[1][w] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = 0.0; b = 0.0;
    for (int i = 0; i < kFinBlock / 64; ++i) { a += red[0][i]; b += red[1][i]; }
  }
  s0 = a;
  s1 = b;
}

__device__ __forceinline__ bool finite_d(double v) { return v == v && v - v == 0.0; }

// After q = A p:  alpha = gamma / ||q||^2.
__device__ __forceinline__ void fin_alpha(DevState* st, const double* partials, int n) {
  if (st->done) return;
  if (st->stop) {
    if (threadIdx.x == 0) st->done = 1;
    return;
  }
  double qq, unused;
  grid_sum2(partials, n, qq, unused);
  if (threadIdx.x == 0) {
    st->qq = qq;
    if (!(qq > 0.0) || !finite_d(qq)) {
      st->breakdown = 1;
      st->alpha = 0.0;
      st->stop = 1;
      st->done = 1;
    } else {
      st->alpha = st->gamma / qq;
    }
  }
}

// After s = A^T r':  beta = ||s||^2 / gamma, convergence test on ||r'||^2.
__device__ __forceinline__ void fin_beta(DevState* st, const double* partials, int n) {
  if (st->done) return;
  double ss, rr;
  grid_sum2(partials, n, ss, rr);
  if (threadIdx.x == 0) {
    const double g0 = st->gamma;
    st->beta = (g0 > 0.0) ? ss / g0 : 0.0;
    st->gamma = ss;
    st->rr = rr;
    st->iters += 1;
    if (!finite_d(rr) || !finite_d(ss)) { st->breakdown = 1; st->stop = 1; st->nonfinite = 1.0; }
    if (rr <= st->tol2 || st->iters >= st->max_iters || !(ss > 0.0)) st->stop = 1;
  }
}

// After s = A^T r0, p = s:  start of an inner solve.
__device__ __forceinline__ void fin_init(DevState* st, const double* partials, int n, double inner_tol2) {
  double ss, unused;
  grid_sum2(partials, n, ss, unused);
  if (threadIdx.x == 0) {
    st->gamma = ss;
    st->rr0 = st->rr;
    st->tol2 = inner_tol2 * st->rr;
    st->stop = (ss > 0.0 && finite_d(ss)) ? 0 : 1;
    st->done = 0;
    st->breakdown = 0;
    st->alpha = 0.0;
    st->beta = 0.0;
  }
}

// CG on the normal equations with the recursive normal residual s
// (q = A p;  alpha = gamma / ||q||^2;  s <- s - alpha A^T q;  x += alpha p;
// p <- s + beta p).  The residual norm follows ||r'||^2 = ||r||^2 - alpha gamma
// (r' = r - alpha q and <r, q> = <s, p> = gamma), so r itself is never formed.
// After q = A p:
__device__ __forceinline__ void fin_alpha_cg(DevState* st, const double* partials, int n) {
  if (st->done) return;
  if (st->stop) {
    if (threadIdx.x == 0) st->done = 1;
    return;
  }
  double qq, unused;
  grid_sum2(partials, n, qq, unused);
  if (threadIdx.x == 0) {
    st->qq = qq;
    if (!(qq > 0.0) || !finite_d(qq)) {
      st->breakdown = 1;
      st->alpha = 0.0;
      st->stop = 1;
      st->done = 1;
    } else {
      const double al = st->gamma / qq;
      st->alpha = al;
      st->rr -= al * st->gamma;
      st->iters += 1;
      if (st->rr <= st->tol2 || st->iters >= st->max_iters) st->stop = 1;
    }
  }
}

// After s <- s - alpha A^T q (partials hold ||s||^2):
__device__ __forceinline__ void fin_beta_cg(DevState* st, const double* partials, int n) {
  if (st->done || st->stop) return;
  double ss, unused;
  grid_sum2(partials, n, ss, unused);
  if (threadIdx.x == 0) {
    const double g0 = st->gamma;
    st->beta = (g0 > 0.0) ? ss / g0 : 0.0;
    st->gamma = ss;
    if (!finite_d(ss)) { st->breakdown = 1; st->stop = 1; st->nonfinite = 1.0; }
    if (!(ss > 0.0)) st->stop = 1;
  }
}

// After r~ = W r (equilibrated CG):  the tracked residual norm is <r, W r>.
__device__ __forceinline__ void fin_rr(DevState* st, const double* partials, int n) {
  double rr, unused;
  grid_sum2(partials, n, rr, unused);
  if (threadIdx.x == 0) st->rr = rr;
}

// After r = Q - A x (FP64):  true residual and ||Q||^2.
__device__ __forceinline__ void fin_resid(DevState* st, const double* partials, int n) {
  double rr, bb;
  grid_sum2(partials, n, rr, bb);
  if (threadIdx.x == 0) {
    st->rtrue2 = rr;
    st->bb2 = bb;
    st->rr = rr;
  }
}

static __global__ void __launch_bounds__(kFinBlock) k_fin_alpha(DevState* st, const double* partials, int n) { fin_alpha(st, partials, n); }
static __global__ void __launch_bounds__(kFinBlock) k_fin_beta(DevState* st, const double* partials, int n) { fin_beta(st, partials, n); }
static __global__ void __launch_bounds__(kFinBlock) k_fin_init(DevState* st, const double* partials, int n, double inner_tol2) { fin_init(st, partials, n, inner_tol2); }
static __global__ void __launch_bounds__(kFinBlock) k_fin_alpha_cg(DevState* st, const double* partials, int n) { fin_alpha_cg(st, partials, n); }
static __global__ void __launch_bounds__(kFinBlock) k_fin_beta_cg(DevState* st, const double* partials, int n) { fin_beta_cg(st, partials, n); }
static __global__ void __launch_bounds__(kFinBlock) k_fin_resid(DevState* st, const double* partials, int n) { fin_resid(st, partials, n); }
static __global__ void __launch_bounds__(kFinBlock) k_fin_rr(DevState* st, const double* partials, int n) { fin_rr(st, partials, n); }

// ---------------------------------------------------------------- vector --
// Non-temporal float4 access for the pure streaming update: the stream is
// larger than the caches and is not re-read before the next stencil pass
// evicts it, so marking it non-temporal leaves the caches to the lines the
// stencil passes reuse (faster update, and faster stencil passes after it).
typedef float f4nt __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld_nt(const float4* p) {
  const f4nt v = __builtin_nontemporal_load(reinterpret_cast<const f4nt*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st_nt(float4* p, const float4 a) {
  const f4nt v = {a.x, a.y, a.z, a.w};
  __builtin_nontemporal_store(v, reinterpret_cast<f4nt*>(p));
}

// x += alpha p;  p = s + beta p
template <typename T>
__global__ void __launch_bounds__(kBlock) k_update_xp(T* __restrict__ x, T* __restrict__ p,
                                                      const T* __restrict__ s, long n, const DevState* st) {
  if (st->done) return;
  const T al = T(st->alpha), be = T(st->beta);
  const long stride = (long)gridDim.x * kBlock;
  if constexpr (sizeof(T) == 4) {
    const long n4 = n >> 2;
    float4* x4 = reinterpret_cast<float4*>(x);
    float4* p4 = reinterpret_cast<float4*>(p);
    const float4* s4 = reinterpret_cast<const float4*>(s);
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n4; i += stride) {
      float4 pv = ld_nt(p4 + i), xv = ld_nt(x4 + i);
      const float4 sv = ld_nt(s4 + i);
      xv.x = __fmaf_rn(al, pv.x, xv.x); xv.y = __fmaf_rn(al, pv.y, xv.y);
      xv.z = __fmaf_rn(al, pv.z, xv.z); xv.w = __fmaf_rn(al, pv.w, xv.w);
      pv.x = __fmaf_rn(be, pv.x, sv.x); pv.y = __fmaf_rn(be, pv.y, sv.y);
      pv.z = __fmaf_rn(be, pv.z, sv.z); pv.w = __fmaf_rn(be, pv.w, sv.w);
      st_nt(x4 + i, xv);
      st_nt(p4 + i, pv);
    }
    for (long i = (n4 << 2) + (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
      const T pv = p[i];
      x[i] = fmadd<T>(al, pv, x[i]);
      p[i] = fmadd<T>(be, pv, s[i]);
    }
  } else {
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
      const T pv = p[i];
      x[i] = fmadd<T>(al, pv, x[i]);
      p[i] = fmadd<T>(be, pv, s[i]);
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill(T* __restrict__ v, long n, T value) {
  const long stride = (long)gridDim.x * kBlock;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) v[i] = value;
}

// x64 += d (refinement update)
template <typename TD>
__global__ void __launch_bounds__(kBlock) k_axpy64(double* __restrict__ x, const TD* __restrict__ d, long n) {
  const long stride = (long)gridDim.x * kBlock;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) x[i] += double(d[i]);
}

// Padded cell arrays: med32 = (sigma_a, sigma_s) in FP32 and med = (sigma_t,
// albedo) with sigma_t raised to the threshold; the one-cell halo holds
// clamped (vacuum, Neumann) or wrapped (periodic) copies, per axis.  Sets
// bit 0 of *bad for NaN / Inf, bit 1 for a cell whose (thresholded)
// extinction is not positive.
static __global__ void __launch_bounds__(kBlock) k_medium_prep(const float* __restrict__ sigma_t,
                                                        const float* __restrict__ albedo, float thr,
                                                        int nx, int ny, int nz, int perx, int pery, int perz,
                                                        float2* __restrict__ med32, float2* __restrict__ med,
                                                        int* bad) {
  const long long CX = nx + 2, CY = ny + 2, n = CX * CY * (nz + 2);
  const long long stride = (long long)gridDim.x * kBlock;
  int b = 0;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    int px = (int)(i % CX) - 1, py = (int)((i / CX) % CY) - 1, pz = (int)(i / (CX * CY)) - 1;
    px = perx ? wrapi(px, nx) : min(max(px, 0), nx - 1);
    py = pery ? wrapi(py, ny) : min(max(py, 0), ny - 1);
    pz = perz ? wrapi(pz, nz) : min(max(pz, 0), nz - 1);
    const long long src = ((long long)pz * ny + py) * nx + px;
    const float s = sigma_t[src], al = albedo[src];
    if (!isfinite(s) || !isfinite(al)) b |= 1;
    const float st = fmaxf(s, thr);
    if (!(st > 0.f)) b |= 2;
    med[i] = make_float2(st, al);
    med32[i] = make_float2(st * (1.0f - al), st * al);
  }
  if (b) atomicOr(bad, b);
}

// Layout conversion between the packed API layout (coefficient k contiguous
// over its class extent) and the padded lattice.  One grid row per k.
struct PackArgs {
  int nc;
  int PX, PY, plane;
  long long cs;
  long long off[kMaxCoeff];
  int ex[kMaxCoeff], ey[kMaxCoeff], ez[kMaxCoeff];
};

// DIR 0: padded[k] <- packed;  DIR 1: packed <- padded;  DIR 2: packed += padded
template <typename TS, typename TD, int DIR>
__global__ void __launch_bounds__(kBlock) k_pack(const TS* __restrict__ src, TD* __restrict__ dst, const PackArgs p) {
  const int k = blockIdx.y;
  const int ex = p.ex[k], ey = p.ey[k];
  const long long sz = (long long)ex * ey * p.ez[k];
  const long long stride = (long long)gridDim.x * kBlock;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < sz; i += stride) {
    const int x = (int)(i % ex);
    const long long t = i / ex;
    const int y = (int)(t % ey), z = (int)(t / ey);
    const long long pi = (long long)k * p.cs + ((long long)(z + 1) * p.PY + (y + 1)) * p.PX + (x + 1);
    const long long qi = p.off[k] + i;
    if constexpr (DIR == 0) dst[pi] = TD(src[qi]);
    else if constexpr (DIR == 1) dst[qi] = TD(src[pi]);
    else dst[qi] += TD(src[pi]);
  }
}

// Flags NaN / Inf in a float vector.
static __global__ void __launch_bounds__(kBlock) k_check_finite(const float* __restrict__ v, long n, int* bad) {
  const long stride = (long)gridDim.x * kBlock;
  int b = 0;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
    if (!isfinite(v[i])) b = 1;
  if (b) atomicOr(bad, 1);
}


// ------------------------------------------------- even-parity PCG (Schur) --
// CG with a Jacobi preconditioner on S d_e = f, S = D_e - T_eo D_o^-1 T_oe
// (symmetric positive definite when T_oe = -T_eo^T), on the even-band
// coefficients of the padded vectors.  DevState: gamma = <r, M r>, rr = <r, r>,
// qq = <p, S p>.  The reduced residual equals the residual of the whole system
// once the odd part is back-substituted, so the inner stop tests <r, r>.
__device__ __forceinline__ void fin_alpha_pcg(DevState* st, const double* partials, int n) {
  if (st->done) return;
  if (st->stop) {
    if (threadIdx.x == 0) st->done = 1;
    return;
  }
  double pq, unused;
  grid_sum2(partials, n, pq, unused);
  if (threadIdx.x == 0) {
    st->qq = pq;
    if (!(pq > 0.0) || !finite_d(pq)) {
      st->breakdown = 1;
      st->alpha = 0.0;
      st->stop = 1;
      st->done = 1;
    } else {
      st->alpha = st->gamma / pq;
    }
  }
}

__device__ __forceinline__ void fin_beta_pcg(DevState* st, const double* partials, int n) {
  if (st->done || st->stop) return;
  double rz, rr;
  grid_sum2(partials, n, rz, rr);
  if (threadIdx.x == 0) {
    const double g0 = st->gamma;
    st->beta = (g0 > 0.0) ? rz / g0 : 0.0;
    st->gamma = rz;
    st->rr = rr;
    st->iters += 1;
    if (!finite_d(rr) || !finite_d(rz)) { st->breakdown = 1; st->stop = 1; st->nonfinite = 1.0; }
    if (rr <= st->tol2 || st->iters >= st->max_iters || !(rz > 0.0)) st->stop = 1;
  }
}

// start of an inner solve: gamma = <r, M r>, rr = <r, r>; stop at rr <= itol2 * ||r0||^2
__device__ __forceinline__ void fin_init_pcg(DevState* st, const double* partials, int n, double inner_tol2) {
  double rz, rr;
  grid_sum2(partials, n, rz, rr);
  if (threadIdx.x == 0) {
    st->gamma = rz;
    st->rr = rr;
    st->rr0 = st->rtrue2;
    st->tol2 = inner_tol2 * st->rtrue2;
    st->stop = (rz > 0.0 && finite_d(rz) && rr > st->tol2) ? 0 : 1;
    st->done = 0;
    st->breakdown = 0;
    st->alpha = 0.0;
    st->beta = 0.0;
  }
}

static __global__ void __launch_bounds__(kFinBlock) k_fin_alpha_pcg(DevState* st, const double* partials, int n) { fin_alpha_pcg(st, partials, n); }
static __global__ void __launch_bounds__(kFinBlock) k_fin_beta_pcg(DevState* st, const double* partials, int n) { fin_beta_pcg(st, partials, n); }
static __global__ void __launch_bounds__(kFinBlock) k_fin_init_pcg(DevState* st, const double* partials, int n, double inner_tol2) { fin_init_pcg(st, partials, n, inner_tol2); }

// bfloat16 copy (round to nearest even) of a float vector
static __global__ void __launch_bounds__(kBlock) k_to_bf16(const float* __restrict__ src, uint16_t* __restrict__ dst,
                                                           long n) {
  const long stride = (long)gridDim.x * kBlock;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const uint32_t u = __float_as_uint(src[i]);
    dst[i] = (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
  }
}

// The even-band coefficient arrays of a padded vector: array j of the list
// starts at k[j] * cs; each is cs floats (a multiple of 64).  Grid: (blocks
// per array, arrays); block partials in the order blockIdx.y * gridDim.x +
// blockIdx.x.
struct EvenSlots {
  int nk;
  int k[kMaxCoeff];
  long long cs;
};

// The preconditioner m is stored in bfloat16 (it only has to be the same
// positive diagonal in every use; 8 bits of mantissa keep it within 0.4% of
// 1 / diag(S)), which halves its share of the vector traffic.
__device__ __forceinline__ float4 ld_bf4(const uint2* p) {
  const uint2 v = *p;
  return make_float4(__uint_as_float(v.x << 16), __uint_as_float(v.x & 0xffff0000u), __uint_as_float(v.y << 16),
                     __uint_as_float(v.y & 0xffff0000u));
}

// OP 0 (init):    p = m r                              [<r, m r>, <r, r>]
// OP 2 (x, p):    x += alpha p, p = m r + beta p
// (x is advanced together with p, one pass after r -- which the even-row
// stencil pass updates: alpha is still the step of this iteration there, and
// that pass runs after the stop test too)
template <int OP>
__global__ void __launch_bounds__(kBlock) k_pcg_vec(float* __restrict__ x, float* __restrict__ r,
                                                    float* __restrict__ p, const float* __restrict__ q,
                                                    const uint16_t* __restrict__ m, const EvenSlots es,
                                                    double* __restrict__ partials, const DevState* st) {
  if (OP != 0 && st->done) return;
  const long long base = (long long)es.k[blockIdx.y] * es.cs;
  const long long n4 = es.cs >> 2;
  const long long stride = (long long)gridDim.x * kBlock;
  const float al = OP != 0 ? float(st->alpha) : 0.f, be = OP == 2 ? float(st->beta) : 0.f;
  float4* x4 = reinterpret_cast<float4*>(x + base);
  float4* r4 = reinterpret_cast<float4*>(r + base);
  float4* p4 = reinterpret_cast<float4*>(p + base);
  const uint2* m4 = reinterpret_cast<const uint2*>(m + base);
  double s0 = 0.0, s1 = 0.0;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n4; i += stride) {
    float4 rv = ld_nt(r4 + i);
    const float4 mv = ld_bf4(m4 + i);
    if constexpr (OP == 2) {
      float4 pv = ld_nt(p4 + i), xv = ld_nt(x4 + i);
      xv.x = __fmaf_rn(al, pv.x, xv.x); xv.y = __fmaf_rn(al, pv.y, xv.y);
      xv.z = __fmaf_rn(al, pv.z, xv.z); xv.w = __fmaf_rn(al, pv.w, xv.w);
      pv.x = __fmaf_rn(be, pv.x, mv.x * rv.x); pv.y = __fmaf_rn(be, pv.y, mv.y * rv.y);
      pv.z = __fmaf_rn(be, pv.z, mv.z * rv.z); pv.w = __fmaf_rn(be, pv.w, mv.w * rv.w);
      st_nt(x4 + i, xv);
      st_nt(p4 + i, pv);
    } else {
      const float4 z = make_float4(mv.x * rv.x, mv.y * rv.y, mv.z * rv.z, mv.w * rv.w);
      if constexpr (OP == 0) st_nt(p4 + i, z);
      s0 += double(fmadd<float>(z.x, rv.x, fmadd<float>(z.y, rv.y, fmadd<float>(z.z, rv.z, z.w * rv.w))));
      s1 += double(fmadd<float>(rv.x, rv.x, fmadd<float>(rv.y, rv.y, fmadd<float>(rv.z, rv.z, rv.w * rv.w))));
    }
  }
  if constexpr (OP != 2) {
    block_sum2(s0, s1);
    if (threadIdx.x == 0) {
      const int b = blockIdx.y * gridDim.x + blockIdx.x;
      partials[2 * b] = s0;
      partials[2 * b + 1] = s1;
    }
  }
}

// ------------------------------------------------------- batch (scalars) --
// One block per system; a finished (frozen) system is skipped.
enum BatchFin { BF_ALPHA = 0, BF_BETA = 1, BF_INIT = 2, BF_RESID = 3, BF_ALPHA_CG = 4, BF_BETA_CG = 5, BF_RR = 6 };

template <int WHICH>
__global__ void __launch_bounds__(kFinBlock) k_fin_batch(const SysArgs* __restrict__ sys) {
  const SysArgs* s = sys + blockIdx.x;
  DevState* st = s->a.st;
  if (st->frozen) return;
  const double* p = s->a.partials;
  const int n = s->a.nblocks;
  if constexpr (WHICH == BF_ALPHA) fin_alpha(st, p, n);
  else if constexpr (WHICH == BF_BETA) fin_beta(st, p, n);
  else if constexpr (WHICH == BF_INIT) fin_init(st, p, n, st->itol2);
  else if constexpr (WHICH == BF_ALPHA_CG) fin_alpha_cg(st, p, n);
  else if constexpr (WHICH == BF_BETA_CG) fin_beta_cg(st, p, n);
  else if constexpr (WHICH == BF_RR) fin_rr(st, p, n);
  else fin_resid(st, p, n);
}

// Number of systems whose inner solve is still running (one block).
static __global__ void __launch_bounds__(kBlock) k_batch_active(const SysArgs* __restrict__ sys, int nsys,
                                                               int* __restrict__ out) {
  __shared__ int cnt[kBlock];
  int c = 0;
  for (int i = threadIdx.x; i < nsys; i += kBlock) {
    const DevState* st = sys[i].a.st;
    c += (!st->frozen && !st->done) ? 1 : 0;
  }
  cnt[threadIdx.x] = c;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) cnt[threadIdx.x] += cnt[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = cnt[0];
}

// ------------------------------------------------------- batch (vectors) --
// Work item (system, chunk): elements [chunk*kChunk, min((chunk+1)*kChunk, nv))
// of the system's padded vectors.  nv is a multiple of 64, so a chunk is a
// whole number of float4.
constexpr int kChunk = 8192;
enum BatchOp { BO_UPDATE_XP = 0, BO_ZERO_D = 1, BO_COPY_SP = 2, BO_AXPY64 = 3 };

template <int OP>
__global__ void __launch_bounds__(kBlock) k_vec_batch(const SysArgs* __restrict__ sys, const int2* __restrict__ work,
                                                      int nwork) {
  const int2 w = work[xcd_remap(blockIdx.x, nwork)];
  const SysArgs* s = sys + w.x;
  const DevState* st = s->a.st;
  if (st->frozen) return;
  if (OP == BO_UPDATE_XP && st->done) return;
  const long long i0 = (long long)w.y * kChunk;
  const long long i1 = min(i0 + (long long)kChunk, s->nv);
  float* d = static_cast<float*>(s->vec[BV_D]);
  float* p = static_cast<float*>(s->vec[BV_P]);
  const float* sv = static_cast<const float*>(s->vec[BV_S]);
  if constexpr (OP == BO_AXPY64) {
    double* x = static_cast<double*>(s->vec[BV_X64]);
    for (long long i = i0 + threadIdx.x; i < i1; i += kBlock) x[i] += double(d[i]);
    return;
  }
  const float al = float(st->alpha), be = float(st->beta);
  float4* d4 = reinterpret_cast<float4*>(d);
  float4* p4 = reinterpret_cast<float4*>(p);
  const float4* s4 = reinterpret_cast<const float4*>(sv);
  for (long long i = (i0 >> 2) + threadIdx.x; i < (i1 >> 2); i += kBlock) {
    if constexpr (OP == BO_UPDATE_XP) {
      float4 pv = ld_nt(p4 + i), xv = ld_nt(d4 + i);
      const float4 q = ld_nt(s4 + i);
      xv.x = __fmaf_rn(al, pv.x, xv.x); xv.y = __fmaf_rn(al, pv.y, xv.y);
      xv.z = __fmaf_rn(al, pv.z, xv.z); xv.w = __fmaf_rn(al, pv.w, xv.w);
      pv.x = __fmaf_rn(be, pv.x, q.x); pv.y = __fmaf_rn(be, pv.y, q.y);
      pv.z = __fmaf_rn(be, pv.z, q.z); pv.w = __fmaf_rn(be, pv.w, q.w);
      st_nt(d4 + i, xv);
      st_nt(p4 + i, pv);
    } else if constexpr (OP == BO_ZERO_D) {
      d4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
      p4[i] = s4[i];
    }
  }
}

}  // namespace pn
