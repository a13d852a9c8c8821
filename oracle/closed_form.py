"""Closed-form transport couplings printed in the paper (oracle pin only;
test infrastructure).

The appendix ("Final equation" of the real-valued derivation) prints, for the
row (l, m), the transport term as a sum of c_j d/dx_d L^{l',m'} with
coefficients built from a..f, beta and delta.  This module writes those rows
out as a table  {(k, d, k'): coefficient}  so that ``tests/`` can compare them
with the quadrature couplings of ``couplings.transport_couplings``.

The printed rows do not match the integral as printed; three corrections make
all of them agree with quadrature (they are readings of the paper):

  1. a^{l,m}: the denominator (2l+1)(2l-1) is replaced by (2l+3)(2l+1)
     (as printed, a^{0,0} is the square root of a negative number);
  2. the m > 0 x-row term with e^{l-1,m-1} uses e^{l-1,-m+1};
  3. every x and y coupling changes sign.  The printed rows correspond to a
     real basis that keeps the Condon-Shortley phase (an extra (-1)^m, i.e. a
     rotation by pi about the pole axis); the basis as defined in the appendix
     has no such phase.  The paper itself notes that the signs of the x and y
     terms depend on the handedness convention.

Typographical slips that do not change the couplings are read in the obvious
way: the missing "+" signs of the m = 0 row, and the missing L^{l-1,m+1}
factor of the first m > 0 x-term.
"""
from math import sqrt

from .sh import coeff_index


def _sq(num, den, what):
    if den == 0:
        raise ZeroDivisionError(what)
    v = num / den
    if v < -1e-15:
        raise ValueError("negative radicand in %s" % what)
    return sqrt(max(v, 0.0))


def a_(l, m):  # corrected denominator (correction 1)
    return _sq((l - m + 1) * (l + m + 1), (2 * l + 3) * (2 * l + 1), "a")


def b_(l, m):
    return _sq((l - m) * (l + m), (2 * l + 1) * (2 * l - 1), "b")


def c_(l, m):
    return _sq((l + m + 1) * (l + m + 2), (2 * l + 3) * (2 * l + 1), "c")


def d_(l, m):
    return _sq((l - m) * (l - m - 1), (2 * l + 1) * (2 * l - 1), "d")


def e_(l, m):
    return _sq((l - m + 1) * (l - m + 2), (2 * l + 3) * (2 * l + 1), "e")


def f_(l, m):
    return _sq((l + m) * (l + m - 1), (2 * l + 1) * (2 * l - 1), "f")


def beta(m):
    """beta^m = 2/sqrt(2) for |m| = 1, else 1 (appendix definition)."""
    return 2.0 / sqrt(2.0) if abs(m) == 1 else 1.0


def delta_ne(x, y):
    return 1.0 if x != y else 0.0


def _valid(order, l, m):
    return 0 <= l <= order and -l <= m <= l


def row_terms(l, m):
    """Printed transport terms of row (l, m): list of (d, l', m', thunk).

    The coefficient is a thunk so that terms whose target (l', m') lies
    outside the expansion are never evaluated (their a..f may be undefined).
    Signs are the printed ones; correction 3 is applied in ``closed_form_table``.
    """
    X, Y, Z = 0, 1, 2
    r2 = 1.0 / sqrt(2.0)
    t = []
    if m == 0:
        t += [(X, l - 1, 1, lambda: r2 * c_(l - 1, -1)),
              (X, l + 1, 1, lambda: -r2 * d_(l + 1, -1)),
              (Y, l - 1, -1, lambda: r2 * c_(l - 1, -1)),
              (Y, l + 1, -1, lambda: -r2 * d_(l + 1, -1)),
              (Z, l - 1, 0, lambda: a_(l - 1, 0)),
              (Z, l + 1, 0, lambda: b_(l + 1, 0))]
    elif m < 0:
        t += [(Y, l - 1, -m + 1, lambda: -0.5 * c_(l - 1, m - 1)),
              (Y, l + 1, -m + 1, lambda: 0.5 * d_(l + 1, m - 1)),
              (Y, l - 1, -m - 1, lambda: -0.5 * beta(m) * e_(l - 1, m + 1)),
              (Y, l + 1, -m - 1, lambda: 0.5 * beta(m) * f_(l + 1, m + 1)),
              (X, l - 1, m - 1, lambda: 0.5 * c_(l - 1, m - 1)),
              (X, l - 1, m + 1, lambda: -0.5 * delta_ne(m, -1) * e_(l - 1, m + 1)),
              (X, l + 1, m + 1, lambda: 0.5 * delta_ne(m, -1) * f_(l + 1, m + 1)),
              (X, l + 1, m - 1, lambda: -0.5 * d_(l + 1, m - 1)),
              (Z, l - 1, m, lambda: a_(l - 1, m)),
              (Z, l + 1, m, lambda: b_(l + 1, m))]
    else:
        t += [(X, l - 1, m + 1, lambda: 0.5 * c_(l - 1, -m - 1)),
              (X, l + 1, m + 1, lambda: -0.5 * d_(l + 1, -m - 1)),
              # correction 2: e^{l-1,-m+1} instead of the printed e^{l-1,m-1}
              (X, l - 1, m - 1, lambda: -0.5 * beta(m) * e_(l - 1, -m + 1)),
              (X, l + 1, m - 1, lambda: 0.5 * beta(m) * f_(l + 1, -m + 1)),
              (Y, l - 1, -m - 1, lambda: 0.5 * c_(l - 1, -m - 1)),
              (Y, l + 1, -m - 1, lambda: -0.5 * d_(l + 1, -m - 1)),
              (Y, l - 1, -m + 1, lambda: 0.5 * delta_ne(m, 1) * e_(l - 1, -m + 1)),
              (Y, l + 1, -m + 1, lambda: -0.5 * delta_ne(m, 1) * f_(l + 1, -m + 1)),
              (Z, l - 1, m, lambda: a_(l - 1, -m)),
              (Z, l + 1, m, lambda: b_(l + 1, -m))]
    return t


def closed_form_table(order, printed_signs=False):
    """{(k, d, k'): coefficient} for all rows with l <= order.

    Terms that reference a coefficient outside the truncated expansion are
    dropped (truncation at order N).  Duplicate (k, d, k') entries are summed.
    With ``printed_signs=False`` correction 3 (x and y signs flipped) is applied.
    """
    out = {}
    for l in range(order + 1):
        for m in range(-l, l + 1):
            k = coeff_index(l, m)
            for (d, lp, mp, coef) in row_terms(l, m):
                if not _valid(order, lp, mp):
                    continue
                v = coef()
                if v == 0.0:
                    continue
                if d in (0, 1) and not printed_signs:
                    v = -v
                key = (k, d, coeff_index(lp, mp))
                out[key] = out.get(key, 0.0) + v
    return out
