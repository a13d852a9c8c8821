"""Angular coupling tables by quadrature (oracle; test infrastructure only).

Transport term (paper, section "Real-valued P_N-equations" and the appendix
"Transport term"): projecting (omega . grad) L_hat onto Y_R^k gives

    P^k T(L_hat) = sum_d sum_k' A_d[k,k'] d/dx_d L^k',
    A_d[k,k'] = int_{S^2} omega_d Y_R^k(omega) Y_R^k'(omega) d omega,

with omega = (sin t cos p, sin t sin p, cos t).  The oracle takes this
integral itself as the definition and evaluates it with a product rule:
Gauss-Legendre in cos(theta) times the uniform (trapezoidal) rule in phi.  The
integrand is a polynomial in (x, y, z) of degree <= 2N+1 on the sphere, so
``nodes_mu >= N + 2`` and ``nodes_phi >= 2N + 2`` make the rule exact; the
defaults use twice that.

Scattering term (appendix "Phase function" and "Scattering term"): a phase
function symmetric about the pole axis has only m = 0 moments
p^{l,0} = int p(cos t) Y_C^{l,0} d omega; the scattering projection is
sigma_s lambda_l p^{l,0} L^{l,m} with lambda_l = sqrt(4 pi / (2l+1)).
"""
from math import pi, sqrt

import numpy as np

from .sh import num_coeffs, real_sh_all, coeff_lm, assoc_legendre, norm_K


def sphere_rule(order, nodes_mu=None, nodes_phi=None):
    """Product quadrature on S^2: returns (theta, phi, weights) flattened."""
    nmu = nodes_mu if nodes_mu is not None else 2 * order + 4
    nphi = nodes_phi if nodes_phi is not None else 4 * order + 8
    mu, wmu = np.polynomial.legendre.leggauss(nmu)
    phi = (np.arange(nphi) + 0.5) * (2.0 * pi / nphi)
    wphi = np.full(nphi, 2.0 * pi / nphi)
    MU, PHI = np.meshgrid(mu, phi, indexing="ij")
    W = np.outer(wmu, wphi)
    return np.arccos(MU).ravel(), PHI.ravel(), W.ravel()


def gram_matrix(order, **kw):
    """G[k,k'] = int Y_R^k Y_R^k' d omega (must be the identity)."""
    th, ph, w = sphere_rule(order, **kw)
    Y = real_sh_all(order, th, ph)
    return (Y * w) @ Y.T


def transport_couplings(order, **kw):
    """A[d, k, k'] = int omega_d Y_R^k Y_R^k' d omega for d = x, y, z.

    Returns an array of shape (3, (N+1)^2, (N+1)^2) in FP64.  Entries below
    1e-14 in magnitude are set to exactly 0 (they are quadrature round-off of
    integrals that vanish by symmetry).
    """
    th, ph, w = sphere_rule(order, **kw)
    Y = real_sh_all(order, th, ph)
    om = (np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th))
    A = np.empty((3, num_coeffs(order), num_coeffs(order)))
    for d in range(3):
        A[d] = (Y * (w * om[d])) @ Y.T
    A[np.abs(A) < 1e-14] = 0.0
    return A


def coupling_list(order, **kw):
    """Non-zero couplings as a list of (k, d, k', value), sorted by (k, d, k')."""
    A = transport_couplings(order, **kw)
    out = []
    n = num_coeffs(order)
    for k in range(n):
        for d in range(3):
            for kp in range(n):
                if A[d, k, kp] != 0.0:
                    out.append((k, d, kp, float(A[d, k, kp])))
    return out


def hg_phase(g, cos_t):
    """Henyey-Greenstein phase function p(cos t), normalised over the sphere."""
    return (1.0 - g * g) / (4.0 * pi * (1.0 + g * g - 2.0 * g * cos_t) ** 1.5)


def phase_moments(order, phase, nodes_mu=None):
    """p^{l,0} = int p(omega . e3) Y_C^{l,0}(omega) d omega, l = 0..N (appendix
    "Phase function").  ``phase`` is a callable of cos(theta).  The integrand
    does not depend on phi, so the phi integral is the factor 2 pi."""
    nmu = nodes_mu if nodes_mu is not None else 400
    mu, wmu = np.polynomial.legendre.leggauss(nmu)
    pv = phase(mu)
    return np.array([2.0 * pi * np.sum(wmu * pv * norm_K(l, 0) * assoc_legendre(l, 0, mu))
                     for l in range(order + 1)])


def scattering_factors(order, phase, **kw):
    """lambda_l p^{l,0} for l = 0..N, lambda_l = sqrt(4 pi / (2l+1)) (appendix,
    Funk-Hecke step of the scattering term).  For Henyey-Greenstein this is
    g^l; the solver uses that value, this function checks it."""
    p = phase_moments(order, phase, **kw)
    return np.array([sqrt(4.0 * pi / (2 * l + 1)) * p[l] for l in range(order + 1)])


def degree_of(k):
    """Band l of flat coefficient index k."""
    return coeff_lm(k)[0]
