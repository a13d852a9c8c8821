"""Pins of the rendering-side oracle (oracle/render.py): un-staggering
reproduces linear fields exactly at the voxel centres; the exact optical
depth of a segment equals the closed form in a homogeneous grid (also for
segments leaving the grid) and a fine Riemann sum in a heterogeneous one; the
projection of the Henyey-Greenstein phase function onto the real basis,
int p(w_L . w) Y^{l,m}(w) dw, equals g^l Y^{l,m}(w_L) by quadrature; and the
single-scatter source of a point light in a homogeneous medium equals its
closed form sigma_s Phi exp(-sigma_t r) / (4 pi r^2) g^l Y^{l,m}(w_L)."""
import numpy as np
import pytest

from oracle.couplings import sphere_rule
from oracle.render import segment_optical_depth, single_scatter_source, unstagger
from oracle.sh import coeff_lm, real_sh
from oracle.stagger import Layout


@pytest.mark.parametrize("order,dims", [(1, (5, 4, 3)), (3, (4, 3, 5)), (5, (3, 4, 2))])
def test_unstagger_reproduces_linear_fields(order, dims):
    lay = Layout(order, dims, 0)
    h = 0.25
    u = np.zeros(lay.n)
    coef = np.random.default_rng(order).normal(size=(lay.ncoeff, 4))
    for k in range(lay.ncoeff):
        x, y, z = lay.positions(k)
        a, b, c, d = coef[k]
        lay.view(u, k)[...] = a + b * x * h + c * y * h + d * z * h
    out = unstagger(lay, u)
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for k in range(lay.ncoeff):
        a, b, c, d = coef[k]
        ref = a + b * (x + 0.5) * h + c * (y + 0.5) * h + d * (z + 0.5) * h
        assert np.allclose(out[k], ref, rtol=0, atol=1e-13)


def test_unstagger_periodic_constant_and_face_mean():
    lay = Layout(3, (4, 3, 2), 1)
    u = np.zeros(lay.n)
    for k in range(lay.ncoeff):
        lay.view(u, k)[...] = float(k)
    out = unstagger(lay, u)
    for k in range(lay.ncoeff):
        assert np.all(out[k] == float(k))
    # a face class along x on a periodic axis: cell 3 averages faces 3 and 0
    k = next(k for k in range(lay.ncoeff) if lay.cls[k] == (1, 0, 0))
    v = lay.view(u, k)
    v[...] = 0.0
    v[0, 0, 0], v[0, 0, 3] = 2.0, 4.0
    assert unstagger(lay, u)[k][0, 0, 3] == 3.0


def test_optical_depth_homogeneous_closed_form():
    rng = np.random.default_rng(0)
    sig = np.full((5, 6, 7), 2.5)
    h = 0.2
    box = np.array([7, 6, 5]) * h
    for _ in range(20):
        p0 = rng.uniform(0, 1, 3) * box
        p1 = rng.uniform(0, 1, 3) * box
        assert abs(segment_optical_depth(sig, h, p0, p1) - 2.5 * np.linalg.norm(p1 - p0)) <= 1e-12
    # a segment leaving the grid: only the part inside counts
    p0, p1 = np.array([0.1, 0.1, 0.1]), np.array([0.1, 0.1, 3.0])
    assert abs(segment_optical_depth(sig, h, p0, p1) - 2.5 * (5 * h - 0.1)) <= 1e-12


def test_optical_depth_vs_riemann_sum():
    rng = np.random.default_rng(1)
    sig = rng.uniform(0.0, 10.0, size=(4, 5, 6))
    h = 0.3
    box = np.array([6, 5, 4]) * h
    for _ in range(5):
        p0 = rng.uniform(0, 1, 3) * box
        p1 = rng.uniform(0, 1, 3) * box
        t = (np.arange(200000) + 0.5) / 200000
        pts = p0[None, :] + t[:, None] * (p1 - p0)[None, :]
        idx = np.minimum(np.floor(pts / h).astype(int), np.array([5, 4, 3]))
        riemann = sig[idx[:, 2], idx[:, 1], idx[:, 0]].mean() * np.linalg.norm(p1 - p0)
        assert abs(segment_optical_depth(sig, h, p0, p1) - riemann) <= 1e-3 * riemann + 1e-9


@pytest.mark.parametrize("g", [0.0, 0.3, -0.4])
def test_hg_projection_is_g_power_times_basis(g):
    theta, phi, w = sphere_rule(5, nodes_mu=400, nodes_phi=400)
    mu = np.cos(theta)
    wl = np.array([0.3, -0.5, 0.81])
    wl /= np.linalg.norm(wl)
    dirs = np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), mu], axis=-1)
    c = dirs @ wl
    p = (1 - g * g) / (4 * np.pi * (1 + g * g - 2 * g * c) ** 1.5)
    tl, pl = np.arccos(wl[2]), np.arctan2(wl[1], wl[0])
    for k in range(36):
        l, m = coeff_lm(k)
        proj = float(np.sum(w * p * real_sh(l, m, theta, phi)))
        assert abs(proj - g ** l * float(real_sh(l, m, tl, pl))) <= 1e-6


def test_single_scatter_homogeneous_closed_form():
    dims = (6, 5, 4)
    st = np.full((4, 5, 6), np.float32(3.0))
    al = np.full((4, 5, 6), np.float32(0.7))
    g = np.float32(0.4)
    h = 0.25
    light = np.array([0.8, 0.55, 0.4])
    q, lay = single_scatter_source(3, dims, st, al, g, 0.0, light, 2.0, h=h)
    sts = float(np.float32(3.0))
    ss = float(np.float32(0.7)) * sts
    for k in range(lay.ncoeff):
        l, m = coeff_lm(k)
        x, y, z = lay.positions(k)
        pos = np.stack([x, y, z], axis=-1) * h
        v = pos - light
        r = np.maximum(np.linalg.norm(v, axis=-1), 0.5 * h)
        wv = v / np.linalg.norm(v, axis=-1, keepdims=True)
        ref = ss * 2.0 * np.exp(-sts * np.linalg.norm(v, axis=-1)) / (4 * np.pi * r * r) * float(g) ** l * \
            real_sh(l, m, np.arccos(np.clip(wv[..., 2], -1, 1)), np.arctan2(wv[..., 1], wv[..., 0]))
        assert np.allclose(lay.view(q, k), ref, rtol=1e-12, atol=1e-15)
