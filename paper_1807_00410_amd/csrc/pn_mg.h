// Multigrid preconditioner of the even-parity PCG.
//
// The Schur complement S = D_e + T_eo D_o^-1 T_eo^T couples each even
// coefficient k only to itself at the six lattice neighbours (T couples k to
// an odd coefficient j along one axis, j back to k along the same one):
//   (S_kk z)(x) = diag(x) z(x) - sum_d [w_d(x+) z(x + e_d) + w_d(x-) z(x - e_d)],
//   w_d(face) = h^-2 sum_j c_kj^2 / d_j(face),
// j over the odd coefficients between x and x +- e_d (the squared couplings
// of the row, section "Real-valued P_N-equations"), diag(x) = d_e(x) + the
// weights of all its faces -- a weighted diffusion operator per coefficient,
// the band-l analogue of the diffusion equation P1 collapses to (section
// "Results").  Its smooth error modes are what Jacobi-preconditioned CG
// converges on slowest; a coarse-grid correction per coefficient removes them.
//
// Preconditioner (symmetric positive definite, so plain PCG applies):
//   B r = omega_f M r + P V(P^T r),
// M the Jacobi inverse diagonal of S (bfloat16), P piecewise-constant
// prolongation over 2 x 2 x 2 aggregates of each coefficient's lattice, and V
// one V-cycle on the Galerkin coarse operators P^T S_kk P (7-point again;
// damped Jacobi before and after the coarse correction, a fixed number of
// damped Jacobi sweeps on the coarsest level).  Coarse operators are formed
// per solve from the fine diagonal and the odd inverse diagonals the Jacobi
// setup computes; every level is diagonally dominant by construction.
#pragma once
#include <hip/hip_runtime.h>

#include "pn_kernels.h"

namespace pn {

constexpr int kMgMaxEven = 28;   // even-band coefficients of P7
constexpr int kMgMaxLevels = 12;
constexpr int kMgMaxTerms = 8;   // odd coefficients coupled to one even row along one axis

// One level: even slot s holds a lattice of ext[s] points stored from off[s]
// (x fastest).  Level L + 1 has ceil(ext / 2) per axis.
struct MgGeom {
  int nk;
  int ext[kMgMaxEven][3];
  long long off[kMgMaxEven + 1];
};

// The fine level as the PCG stores it: slot s is coefficient k[s] of the
// padded lattice (cs floats per coefficient; point (x, y, z) at ((z + 1) PY +
// (y + 1)) PX + (x + 1)); cls the staggering class of the slot's coefficient.
struct MgFine {
  int nk, PX, PY;
  long long cs;
  int k[kMgMaxEven];
  int ext[kMgMaxEven][3];
  int cls[kMgMaxEven][3];
};

// Squared couplings of slot s along axis d: odd coefficients j and c^2.
struct MgTerms {
  int n[kMgMaxEven][3];
  int j[kMgMaxEven][3][kMgMaxTerms];
  float c2[kMgMaxEven][3][kMgMaxTerms];
};

// Levels L0..Lc (the coarsest) of the V-cycle run in one kernel, one block
// per slot in LDS: the geometry and the operators of every level, in device
// memory.
struct MgTail {
  int L0, Lc;
  MgGeom g[kMgMaxLevels];
  const float4* op[kMgMaxLevels];
  const float* idg[kMgMaxLevels];
};

}  // namespace pn
