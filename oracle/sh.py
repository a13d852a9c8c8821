"""Real spherical-harmonics basis in FP64 (oracle; test infrastructure only).

Paper, appendix "Derivation of the complex-valued P_N-equations": the complex
basis is Y_C^{l,m} = (-1)^m K_l^m e^{i m phi} P^{l,m}(cos theta) for m >= 0 and
Y_C^{l,m} = (-1)^m conj(Y_C^{l,|m|}) for m < 0, where the associated Legendre
function P^{l,m} does NOT contain the Condon-Shortley phase.

Appendix "Derivation of the real-valued P_N-equations", real basis equation:
Y_R^{l,m} is built from Y_C^{l,m} and Y_C^{l,-m}.  Composing the two
definitions gives (with mu = |m|)

    m < 0 :  Y_R = sqrt(2) K_l^mu P^{l,mu}(cos theta) sin(mu phi)
    m = 0 :  Y_R = K_l^0 P^{l,0}(cos theta)
    m > 0 :  Y_R = sqrt(2) K_l^m  P^{l,m}(cos theta)  cos(m phi)

This module evaluates Y_R by building Y_C literally from its definition and
forming the real combination of the appendix (the "+" form of the m > 0 case;
the main-text "-" form is imaginary, see ``real_basis_from_complex``), so the
composition above is checked, not assumed.

Coefficient index: k = l*l + l + m, 0 <= k < (N+1)^2.
"""
from math import factorial, pi, sqrt

import numpy as np


def coeff_index(l, m):
    """Flat coefficient index k = l^2 + l + m of (l, m)."""
    return l * l + l + m


def coeff_lm(k):
    """Inverse of ``coeff_index``: returns (l, m)."""
    l = int(np.floor(np.sqrt(k)))
    while (l + 1) * (l + 1) <= k:
        l += 1
    while l * l > k:
        l -= 1
    return l, k - l * l - l


def num_coeffs(order):
    """(N+1)^2 coefficients for truncation order N (main text, truncation)."""
    return (order + 1) * (order + 1)


def assoc_legendre(l, m, x):
    """P^{l,m}(x) for 0 <= m <= l WITHOUT the Condon-Shortley phase.

    Standard three-term recurrence in l at fixed m, started from
    P^{m,m}(x) = (2m-1)!! (1-x^2)^{m/2}.
    """
    x = np.asarray(x, dtype=np.float64)
    if m < 0 or m > l:
        raise ValueError("need 0 <= m <= l")
    s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    pmm = np.ones_like(x)
    for i in range(1, m + 1):
        pmm = pmm * (2 * i - 1) * s
    if l == m:
        return pmm
    pm1 = x * (2 * m + 1) * pmm
    if l == m + 1:
        return pm1
    p_prev, p_cur = pmm, pm1
    for ll in range(m + 2, l + 1):
        p_next = ((2 * ll - 1) * x * p_cur - (ll + m - 1) * p_prev) / (ll - m)
        p_prev, p_cur = p_cur, p_next
    return p_cur


def norm_K(l, m):
    """K_l^m = sqrt((2l+1)/(4 pi) * (l-m)!/(l+m)!) for m >= 0."""
    return sqrt((2 * l + 1) / (4.0 * pi) * factorial(l - m) / factorial(l + m))


def complex_sh(l, m, theta, phi):
    """Complex basis Y_C^{l,m}(theta, phi) of the appendix (CS phase outside P)."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    if m >= 0:
        return ((-1.0) ** m) * norm_K(l, m) * np.exp(1j * m * phi) * assoc_legendre(l, m, np.cos(theta))
    return ((-1.0) ** m) * np.conj(complex_sh(l, -m, theta, phi))


def real_basis_from_complex(l, m, theta, phi):
    """Y_R^{l,m} from Y_C by the appendix real-basis equation.

    m < 0 : (i/sqrt 2) (Y_C^{l,m} - (-1)^m Y_C^{l,-m})
    m = 0 : Y_C^{l,0}
    m > 0 : (1/sqrt 2) (Y_C^{l,-m} + (-1)^m Y_C^{l,m})

    The main-text version of the m > 0 case carries a "-" instead of the "+";
    that combination is purely imaginary for odd m, so the appendix form is the
    one used (a reading of the paper).  Returns the complex value; its imaginary
    part is zero to rounding.
    """
    if m < 0:
        return (1j / sqrt(2.0)) * (complex_sh(l, m, theta, phi) - ((-1.0) ** m) * complex_sh(l, -m, theta, phi))
    if m == 0:
        return complex_sh(l, 0, theta, phi)
    return (1.0 / sqrt(2.0)) * (complex_sh(l, -m, theta, phi) + ((-1.0) ** m) * complex_sh(l, m, theta, phi))


def real_sh(l, m, theta, phi):
    """Real basis Y_R^{l,m}(theta, phi) (real part of ``real_basis_from_complex``)."""
    return np.real(real_basis_from_complex(l, m, theta, phi))


def real_sh_all(order, theta, phi):
    """Array [(N+1)^2, ...] of Y_R^{k} at the given directions, k = l^2+l+m."""
    theta = np.asarray(theta, dtype=np.float64)
    out = np.empty((num_coeffs(order),) + theta.shape, dtype=np.float64)
    for l in range(order + 1):
        for m in range(-l, l + 1):
            out[coeff_index(l, m)] = real_sh(l, m, theta, phi)
    return out
