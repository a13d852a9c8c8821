/*
 * Plain FP64 matrix-free operator of the staggered real P_N system and the
 * paper's solver, for grids too large for the assembled SciPy matrix.
 * ORACLE: test infrastructure only (the tests, the smoke check and the
 * benchmark's CPU baseline use it); the product never calls it.
 *
 * What it computes (section "Discretized Radiative Transfer Equation", with
 * the staggered central differences of section "Precomputation" and the
 * boundary rule of section "Runtime"):  row of coefficient k at lattice
 * point x (class extents and the flat layout as in oracle/stagger.py),
 *
 *   (A u)[k, x] = diag[k, x] u[k, x]
 *               + sum over couplings (k, d, k', c) of
 *                   (c / h) (u[k', x + e_d/2] - u[k', x - e_d/2])
 *
 * where the two samples of u[k'] along axis d are the lattice indices
 * (i+1, i) when k' is face-centred along d and (i, i-1) when it is
 * cell-centred, and an index outside k''s extent is dropped (vacuum /
 * Dirichlet), wrapped (periodic) or moved to the closest index inside
 * (Neumann).  The caller passes the couplings (quadrature values,
 * oracle/couplings.py) and the diagonal sigma_t - g^l sigma_s at every row
 * (oracle/medium.py); nothing here knows the spherical harmonics.
 *
 * ref_apply evaluates one row at a time by that formula (a gather).
 * ref_apply_t evaluates A^T literally: every entry (row, col, value) of A is
 * added to column col's output (a scatter), the threads splitting the work by
 * output coefficient so that no two threads write one entry.  No property of
 * A (symmetry of the couplings, skewness of the transport part) is assumed.
 *
 * ref_cgls is conjugate gradients on the normal equations A^T A u = A^T Q
 * without forming A^T A (sections "Runtime" and "Results"), in the usual CGLS
 * form with the residual r = Q - A u carried along, from u = 0; it stops when
 * the carried relative residual ||r|| / ||Q|| reaches tol.
 *
 * Threads: OpenMP, as many as the caller asks for.
 */
#include <math.h>
#include <omp.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define BC_VACUUM 0
#define BC_PERIODIC 1
#define BC_NEUMANN 2

typedef struct {
  int ncoeff;
  int bc[3];
  double h;
  const long long* off;    /* ncoeff + 1 offsets of the coefficient arrays */
  const int* ext;          /* ncoeff x 3: (ex, ey, ez) */
  const int* cls;          /* ncoeff x 3: (px, py, pz) */
  int ncpl;
  const int* ck;           /* couplings: row coefficient */
  const int* cd;           /*            axis 0, 1, 2 = x, y, z */
  const int* ckp;          /*            column coefficient */
  const double* cv;        /*            value of int omega_d Y^k Y^k' */
  const double* diag;      /* diagonal at every row (flat layout) */
} ref_op;

/* Index along one axis after the boundary rule; -1 when the entry is dropped. */
static long resolve(long idx, long ext, int bc) {
  if (idx >= 0 && idx < ext) return idx;
  if (bc == BC_PERIODIC) return ((idx % ext) + ext) % ext;
  if (bc == BC_NEUMANN) return idx < 0 ? 0 : ext - 1;
  return -1;
}

static long long n_of(const ref_op* op) { return op->off[op->ncoeff]; }

/* y = A u */
void ref_apply(const ref_op* op, const double* u, double* y) {
  const int nc = op->ncoeff;
  int* mine = (int*)malloc(sizeof(int) * (op->ncpl > 0 ? op->ncpl : 1));
  for (int k = 0; k < nc; ++k) {
    const int ex = op->ext[3 * k], ey = op->ext[3 * k + 1], ez = op->ext[3 * k + 2];
    int nm = 0;  /* the couplings of row coefficient k */
    for (int j = 0; j < op->ncpl; ++j)
      if (op->ck[j] == k) mine[nm++] = j;
#pragma omp parallel for schedule(static)
    for (long z = 0; z < ez; ++z) {
      for (long yy = 0; yy < ey; ++yy) {
        for (long x = 0; x < ex; ++x) {
          const long long row = op->off[k] + (z * ey + yy) * ex + x;
          double acc = op->diag[row] * u[row];
          for (int jj = 0; jj < nm; ++jj) {
            const int j = mine[jj];
            const int d = op->cd[j], kp = op->ckp[j];
            const long pt[3] = {x, yy, z};
            const long i = pt[d];
            long ip, im;
            if (op->cls[3 * kp + d] == 1) { ip = i + 1; im = i; }
            else { ip = i; im = i - 1; }
            const long e = op->ext[3 * kp + d];
            const long idx[2] = {resolve(ip, e, op->bc[d]), resolve(im, e, op->bc[d])};
            const double sgn[2] = {1.0, -1.0};
            for (int t = 0; t < 2; ++t) {
              if (idx[t] < 0) continue;
              long q[3] = {pt[0], pt[1], pt[2]};
              q[d] = idx[t];
              const long long col = op->off[kp] +
                  ((long long)q[2] * op->ext[3 * kp + 1] + q[1]) * op->ext[3 * kp] + q[0];
              acc += sgn[t] * (op->cv[j] / op->h) * u[col];
            }
          }
          y[row] = acc;
        }
      }
    }
  }
  free(mine);
}

/* y = A^T u: every entry of A scattered to its column. */
void ref_apply_t(const ref_op* op, const double* u, double* y) {
  const int nc = op->ncoeff;
#pragma omp parallel for schedule(dynamic, 1)
  for (int kp = 0; kp < nc; ++kp) {
    /* the diagonal entries of column block kp */
    for (long long i = op->off[kp]; i < op->off[kp + 1]; ++i) y[i] = op->diag[i] * u[i];
    for (int j = 0; j < op->ncpl; ++j) {
      if (op->ckp[j] != kp) continue;
      const int k = op->ck[j], d = op->cd[j];
      const int ex = op->ext[3 * k], ey = op->ext[3 * k + 1], ez = op->ext[3 * k + 2];
      const long e = op->ext[3 * kp + d];
      for (long z = 0; z < ez; ++z) {
        for (long yy = 0; yy < ey; ++yy) {
          for (long x = 0; x < ex; ++x) {
            const long long row = op->off[k] + (z * ey + yy) * ex + x;
            const double v = (op->cv[j] / op->h) * u[row];
            const long pt[3] = {x, yy, z};
            const long i = pt[d];
            long ip, im;
            if (op->cls[3 * kp + d] == 1) { ip = i + 1; im = i; }
            else { ip = i; im = i - 1; }
            const long idx[2] = {resolve(ip, e, op->bc[d]), resolve(im, e, op->bc[d])};
            const double sgn[2] = {1.0, -1.0};
            for (int t = 0; t < 2; ++t) {
              if (idx[t] < 0) continue;
              long q[3] = {pt[0], pt[1], pt[2]};
              q[d] = idx[t];
              const long long col = op->off[kp] +
                  ((long long)q[2] * op->ext[3 * kp + 1] + q[1]) * op->ext[3 * kp] + q[0];
              y[col] += sgn[t] * v;
            }
          }
        }
      }
    }
  }
}

static double dot(const double* a, const double* b, long long n) {
  double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
  for (long long i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* CGLS from u = 0.  x: output (n).  hist: optional array of max_iter + 1
 * carried relative residuals (entry i after i iterations).  Returns the
 * number of iterations; *rel_out gets the last carried relative residual.
 * progress > 0 prints a line to stderr every `progress` iterations. */
int ref_cgls(const ref_op* op, const double* b, double* x, double tol, int max_iter, double* hist,
             double* rel_out, int progress) {
  const long long n = n_of(op);
  double* r = (double*)malloc(sizeof(double) * n);
  double* s = (double*)malloc(sizeof(double) * n);
  double* p = (double*)malloc(sizeof(double) * n);
  double* q = (double*)malloc(sizeof(double) * n);
  if (!r || !s || !p || !q) {
    free(r); free(s); free(p); free(q);
    return -1;
  }
  const double bnorm = sqrt(dot(b, b, n));
#pragma omp parallel for schedule(static)
  for (long long i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; }
  int it = 0;
  double rel = bnorm > 0.0 ? 1.0 : 0.0;
  if (hist) hist[0] = rel;
  if (bnorm == 0.0) {
    free(r); free(s); free(p); free(q);
    *rel_out = 0.0;
    return 0;
  }
  ref_apply_t(op, r, s);
#pragma omp parallel for schedule(static)
  for (long long i = 0; i < n; ++i) p[i] = s[i];
  double gamma = dot(s, s, n);
  const double t0 = omp_get_wtime();
  while (rel > tol && it < max_iter && gamma > 0.0) {
    ref_apply(op, p, q);
    const double alpha = gamma / dot(q, q, n);
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < n; ++i) {
      x[i] += alpha * p[i];
      r[i] -= alpha * q[i];
    }
    ref_apply_t(op, r, s);
    const double gamma_new = dot(s, s, n);
    const double beta = gamma_new / gamma;
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < n; ++i) p[i] = s[i] + beta * p[i];
    gamma = gamma_new;
    ++it;
    rel = sqrt(dot(r, r, n)) / bnorm;
    if (hist) hist[it] = rel;
    if (progress > 0 && it % progress == 0) {
      fprintf(stderr, "[oracle cgls] iteration %d  relative residual %.3e  %.1f s\n", it, rel,
              omp_get_wtime() - t0);
      fflush(stderr);
    }
  }
  free(r); free(s); free(p); free(q);
  *rel_out = rel;
  return it;
}

void ref_set_threads(int nthreads) {
  if (nthreads > 0) omp_set_num_threads(nthreads);
}

int ref_max_threads(void) { return omp_get_max_threads(); }
