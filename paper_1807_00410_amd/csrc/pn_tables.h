// Compile-time tables of the staggered real P_N operator.
//
// Transport couplings.  The appendix of the paper ("Final equation" of the
// real-valued derivation) gives, for the row of coefficient (l, m), the
// transport term as a sum  c * d/dx_d L^{l',m'}  with c built from the
// factors a..f, beta and delta.  Here those rows are written out at compile
// time for every order N <= 7.  Three corrections make the printed rows equal
// to the projection  int omega_d Y_R^{l,m} Y_R^{l',m'} d omega  of the real
// basis as the appendix defines it (no Condon-Shortley phase):
//   1. a^{l,m} has the denominator (2l+3)(2l+1);
//   2. in the m > 0 x-row, the e-factor of the L^{l-1,m-1} term is e^{l-1,-m+1};
//   3. every x and y coupling changes sign (the printed rows belong to a basis
//      that carries an extra (-1)^m; the paper notes the x/y signs depend on
//      the coordinate convention).
// The missing "+" signs of the printed m = 0 row and the missing L factor of
// the first m > 0 x-term are read in the obvious way.
//
// Staggering.  Coefficient (l, m) lives on the lattice of class (px, py, pz),
// the reflection parities of Y_R^{l,m}: px = m mod 2 (m >= 0) or
// (|m| + 1) mod 2 (m < 0), py = [m < 0], pz = (l + |m|) mod 2.  Every coupling
// joins two classes that differ in exactly the derivative axis, so each
// derivative is a two-point difference over one cell (section
// "Precomputation": staggered placement after StaRMAP).
#pragma once

namespace pn {

constexpr int kMaxOrder = 7;

constexpr double c_sqrt(double v) {
  if (!(v > 0.0)) return 0.0;
  double x = v > 1.0 ? v : 1.0;
  for (int i = 0; i < 200; ++i) {
    double nx = 0.5 * (x + v / x);
    if (nx == x) break;
    x = nx;
  }
  return x;
}

constexpr double q_sqrt(long num, long den) { return c_sqrt(double(num) / double(den)); }

constexpr double fa(int l, int m) { return q_sqrt(long(l - m + 1) * (l + m + 1), long(2 * l + 3) * (2 * l + 1)); }
constexpr double fb(int l, int m) { return q_sqrt(long(l - m) * (l + m), long(2 * l + 1) * (2 * l - 1)); }
constexpr double fc(int l, int m) { return q_sqrt(long(l + m + 1) * (l + m + 2), long(2 * l + 3) * (2 * l + 1)); }
constexpr double fd(int l, int m) { return q_sqrt(long(l - m) * (l - m - 1), long(2 * l + 1) * (2 * l - 1)); }
constexpr double fe(int l, int m) { return q_sqrt(long(l - m + 1) * (l - m + 2), long(2 * l + 3) * (2 * l + 1)); }
constexpr double ff(int l, int m) { return q_sqrt(long(l + m) * (l + m - 1), long(2 * l + 1) * (2 * l - 1)); }
constexpr double fbeta(int m) { return (m == 1 || m == -1) ? 2.0 / c_sqrt(2.0) : 1.0; }
constexpr double fdelta_ne(int a, int b) { return a != b ? 1.0 : 0.0; }

constexpr int coeff_index(int l, int m) { return l * l + l + m; }
constexpr int band_of(int k) {
  int l = 0;
  while ((l + 1) * (l + 1) <= k) ++l;
  return l;
}
constexpr int m_of(int k) { int l = band_of(k); return k - l * l - l; }
constexpr int cls_x(int k) { int m = m_of(k); return m >= 0 ? (m & 1) : ((-m + 1) & 1); }
constexpr int cls_y(int k) { return m_of(k) < 0 ? 1 : 0; }
constexpr int cls_z(int k) { int m = m_of(k); int am = m < 0 ? -m : m; return (band_of(k) + am) & 1; }
constexpr int cls_axis(int k, int d) { return d == 0 ? cls_x(k) : (d == 1 ? cls_y(k) : cls_z(k)); }
constexpr int cls_id(int k) { return cls_x(k) | (cls_y(k) << 1) | (cls_z(k) << 2); }

struct Coupling {
  int k;     // output (row) coefficient
  int d;     // derivative axis 0 = x, 1 = y, 2 = z
  int kp;    // input (column) coefficient
  double c;  // int omega_d Y^k Y^kp
  int ck;    // staggering class id of k
};

struct Term { int d, lp, mp; double c; };

// Printed terms of row (l, m), targets outside the expansion excluded.
// Returns the number of terms written to t (at most 10).
constexpr int row_terms(int N, int l, int m, Term* t) {
  int n = 0;
  auto valid = [N](int lp, int mp) { return lp >= 0 && lp <= N && mp >= -lp && mp <= lp; };
  const double r2 = 1.0 / c_sqrt(2.0);
  auto add = [&](int d, int lp, int mp, double c) {
    if (c != 0.0) { t[n].d = d; t[n].lp = lp; t[n].mp = mp; t[n].c = c; ++n; }
  };
  if (m == 0) {
    if (valid(l - 1, 1)) add(0, l - 1, 1, r2 * fc(l - 1, -1));
    if (valid(l + 1, 1)) add(0, l + 1, 1, -r2 * fd(l + 1, -1));
    if (valid(l - 1, -1)) add(1, l - 1, -1, r2 * fc(l - 1, -1));
    if (valid(l + 1, -1)) add(1, l + 1, -1, -r2 * fd(l + 1, -1));
    if (valid(l - 1, 0)) add(2, l - 1, 0, fa(l - 1, 0));
    if (valid(l + 1, 0)) add(2, l + 1, 0, fb(l + 1, 0));
  } else if (m < 0) {
    if (valid(l - 1, -m + 1)) add(1, l - 1, -m + 1, -0.5 * fc(l - 1, m - 1));
    if (valid(l + 1, -m + 1)) add(1, l + 1, -m + 1, 0.5 * fd(l + 1, m - 1));
    if (valid(l - 1, -m - 1)) add(1, l - 1, -m - 1, -0.5 * fbeta(m) * fe(l - 1, m + 1));
    if (valid(l + 1, -m - 1)) add(1, l + 1, -m - 1, 0.5 * fbeta(m) * ff(l + 1, m + 1));
    if (valid(l - 1, m - 1)) add(0, l - 1, m - 1, 0.5 * fc(l - 1, m - 1));
    if (valid(l - 1, m + 1)) add(0, l - 1, m + 1, -0.5 * fdelta_ne(m, -1) * fe(l - 1, m + 1));
    if (valid(l + 1, m + 1)) add(0, l + 1, m + 1, 0.5 * fdelta_ne(m, -1) * ff(l + 1, m + 1));
    if (valid(l + 1, m - 1)) add(0, l + 1, m - 1, -0.5 * fd(l + 1, m - 1));
    if (valid(l - 1, m)) add(2, l - 1, m, fa(l - 1, m));
    if (valid(l + 1, m)) add(2, l + 1, m, fb(l + 1, m));
  } else {
    if (valid(l - 1, m + 1)) add(0, l - 1, m + 1, 0.5 * fc(l - 1, -m - 1));
    if (valid(l + 1, m + 1)) add(0, l + 1, m + 1, -0.5 * fd(l + 1, -m - 1));
    if (valid(l - 1, m - 1)) add(0, l - 1, m - 1, -0.5 * fbeta(m) * fe(l - 1, -m + 1));  // correction 2
    if (valid(l + 1, m - 1)) add(0, l + 1, m - 1, 0.5 * fbeta(m) * ff(l + 1, -m + 1));
    if (valid(l - 1, -m - 1)) add(1, l - 1, -m - 1, 0.5 * fc(l - 1, -m - 1));
    if (valid(l + 1, -m - 1)) add(1, l + 1, -m - 1, -0.5 * fd(l + 1, -m - 1));
    if (valid(l - 1, -m + 1)) add(1, l - 1, -m + 1, 0.5 * fdelta_ne(m, 1) * fe(l - 1, -m + 1));
    if (valid(l + 1, -m + 1)) add(1, l + 1, -m + 1, -0.5 * fdelta_ne(m, 1) * ff(l + 1, -m + 1));
    if (valid(l - 1, m)) add(2, l - 1, m, fa(l - 1, -m));
    if (valid(l + 1, m)) add(2, l + 1, m, fb(l + 1, -m));
  }
  for (int i = 0; i < n; ++i)
    if (t[i].d != 2) t[i].c = -t[i].c;  // correction 3
  return n;
}

constexpr int num_couplings(int N) {
  int n = 0;
  for (int l = 0; l <= N; ++l)
    for (int m = -l; m <= l; ++m) {
      Term t[12] = {};
      n += row_terms(N, l, m, t);
    }
  return n;
}

template <int N>
struct Table {
  static constexpr int NC = (N + 1) * (N + 1);
  static constexpr int NCPL = num_couplings(N);
  struct Arr { Coupling v[NCPL]; };
  struct Need { bool v[NC][3]; };

  // Couplings sorted by (class of k, d, kp, k).  Along axis d the rows of
  // class c read only inputs of class c ^ (1 << d), so every (kp, d)
  // difference belongs to exactly one row class: a kernel can walk the row
  // classes one at a time, form each difference once, fan it out to the rows
  // of that class and retire their accumulators before the next class.
  static constexpr bool before(const Coupling& a, const Coupling& b) {
    if (a.ck != b.ck) return a.ck < b.ck;
    if (a.d != b.d) return a.d < b.d;
    if (a.kp != b.kp) return a.kp < b.kp;
    return a.k < b.k;
  }
  static constexpr Arr make() {
    Arr a{};
    int n = 0;
    for (int l = 0; l <= N; ++l)
      for (int m = -l; m <= l; ++m) {
        Term t[12] = {};
        int nt = row_terms(N, l, m, t);
        for (int i = 0; i < nt; ++i) {
          a.v[n].k = coeff_index(l, m);
          a.v[n].d = t[i].d;
          a.v[n].kp = coeff_index(t[i].lp, t[i].mp);
          a.v[n].c = t[i].c;
          a.v[n].ck = cls_id(a.v[n].k);
          ++n;
        }
      }
    for (int i = 1; i < NCPL; ++i) {  // insertion sort
      Coupling x = a.v[i];
      int j = i - 1;
      while (j >= 0 && before(x, a.v[j])) {
        a.v[j + 1] = a.v[j];
        --j;
      }
      a.v[j + 1] = x;
    }
    return a;
  }
  // first / one-past-last coupling index of row class c
  static constexpr Arr cpl = make();

  struct Ranges { int b[9]; bool rows[8]; };
  static constexpr Ranges make_ranges() {
    Ranges r{};
    for (int c = 0; c <= 8; ++c) {
      int i = 0;
      while (i < NCPL && cpl.v[i].ck < c) ++i;
      r.b[c] = i;
    }
    for (int k = 0; k < NC; ++k) r.rows[cls_id(k)] = true;
    return r;
  }
  static constexpr Ranges ranges = make_ranges();
  // first / one-past-last coupling index of row class c; does class c hold rows
  static constexpr int class_begin(int c) { return ranges.b[c]; }
  static constexpr int class_end(int c) { return ranges.b[c + 1]; }
  static constexpr bool class_has_rows(int c) { return ranges.rows[c]; }
  // coupling i is the first of its (row class, input, axis) run: the place
  // where that difference is formed
  static constexpr bool starts_difference(int i) {
    return i == 0 || cpl.v[i - 1].ck != cpl.v[i].ck || cpl.v[i - 1].kp != cpl.v[i].kp || cpl.v[i - 1].d != cpl.v[i].d;
  }

  static constexpr Need make_need() {
    Need q{};
    for (int i = 0; i < NCPL; ++i) q.v[cpl.v[i].kp][cpl.v[i].d] = true;
    return q;
  }
  static constexpr Need need = make_need();

  // Sum of the squared transport entries of row k of A in units of 1/h^2:
  // each coupling (k, kp, d, c) puts +c/h and -c/h into the row (the two
  // staggered neighbours along d), so 2 c^2 per coupling.
  static constexpr double row_c2(int k) {
    double s = 0.0;
    for (int i = 0; i < NCPL; ++i)
      if (cpl.v[i].k == k) s += 2.0 * cpl.v[i].c * cpl.v[i].c;
    return s;
  }
};

}  // namespace pn
