"""Pins of the oracle's quadrature, special functions, translation operator
and band-limited resampling (the mathematics the paper defers to its
references in Sec. 2, and the exact global interpolation of Sec. 3.2.2),
against library routines (numpy, scipy) and closed-form identities."""
import math

import numpy as np
import pytest
import scipy.special as sp

from oracle import mlfma as M
from oracle import sphere

K = 2.0 * math.pi


@pytest.mark.parametrize("n", [1, 2, 5, 9, 14, 58, 197])
def test_gauss_legendre_vs_numpy(n):
    x, w = sphere.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    # ours are descending in x
    assert np.all(np.diff(x) < 0)
    assert np.allclose(x[::-1], xr, atol=2e-15)
    # numpy's own weights lose ~1e-11 near the poles at high n (see the
    # mpmath pin below), so compare loosely here
    assert np.allclose(w[::-1], wr, rtol=1e-10, atol=1e-16)
    assert abs(w.sum() - 2.0) < 1e-13


@pytest.mark.parametrize("n", [9, 58, 197])
def test_gauss_legendre_vs_mpmath(n):
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    x, w = sphere.gauss_legendre(n)
    for i in (0, n // 3, n - 1):
        xs = mpmath.mpf(x[i])
        assert abs(mpmath.legendre(n, xs)) < 1e-12 * n
        dp = mpmath.diff(lambda t: mpmath.legendre(n, t), xs)
        wm = 2 / ((1 - xs ** 2) * dp ** 2)
        assert float(abs(w[i] - wm) / wm) < 1e-13


def test_legendre_p_vs_scipy():
    u = np.linspace(-1, 1, 37)
    P = sphere.legendre_p(40, u)
    for l in (0, 1, 2, 7, 40):
        assert np.allclose(P[l], sp.eval_legendre(l, u), atol=1e-13)


@pytest.mark.parametrize("m", [0, 1, 3, 10])
def test_assoc_legendre_vs_scipy(m):
    x = np.linspace(-0.99, 0.99, 23)
    lmax = 30
    P = sphere.assoc_legendre_normalised(lmax, m, x)
    for l in range(m, lmax + 1):
        norm = math.sqrt((2 * l + 1) / 2.0 * math.exp(
            math.lgamma(l - m + 1) - math.lgamma(l + m + 1)))
        ref = norm * sp.lpmv(m, l, x)
        # scipy includes the Condon-Shortley sign (-1)^m; ours drops it
        assert np.allclose(P[l - m], (-1) ** m * ref, atol=1e-11)


def test_assoc_legendre_orthonormal_high_degree():
    # Gauss-Legendre with L+1 nodes integrates degree <= 2L+1 exactly, so the
    # normalised functions of one order are orthonormal on the nodes; at
    # L = 196 (the 16-wavelength level) tiny values near the poles must
    # underflow cleanly (no NaN).
    L = 196
    x, w = sphere.gauss_legendre(L + 1)
    for m in (0, 1, 50, 150, 196):
        P = sphere.assoc_legendre_normalised(L, m, x)
        assert np.all(np.isfinite(P))
        G = (P * w) @ P.T
        assert np.allclose(G, np.eye(L - m + 1), atol=1e-11)


def test_hankel_vs_scipy():
    for x in (0.3, math.pi, 7.5, 60.0):
        h = sphere.spherical_hankel1(50, x)
        l = np.arange(51)
        ref = sp.spherical_jn(l, x) + 1j * sp.spherical_yn(l, x)
        assert np.allclose(h, ref, rtol=1e-10, atol=0)


def test_grid_quadrature_exact_for_harmonics():
    # sum_q w_q Y_lm conj(Y_l'm') = delta for l + l' <= 2L + 1 (and
    # |m| <= L so that the phi sum does not alias)
    L = 8
    g = sphere.SphereGrid(L)
    th = np.arccos(g.khat[:, 2])
    ph = np.arctan2(g.khat[:, 1], g.khat[:, 0])
    idx = [(l, m) for l in range(L + 1) for m in range(-l, l + 1)]
    Y = np.stack([sp.sph_harm_y(l, m, th, ph) for l, m in idx])
    G = (Y * g.w) @ Y.conj().T
    assert np.allclose(G, np.eye(len(idx)), atol=1e-13)
    assert abs(g.w.sum() - 4 * math.pi) < 1e-13


def test_plane_wave_identity():
    # sum_q w_q exp(ik khat.d) P_l(khat.Xhat) = 4 pi i^l j_l(k|d|) P_l(dhat.Xhat)
    L = 20
    g = sphere.SphereGrid(L)
    d = np.array([0.1, -0.05, 0.07])
    Xh = np.array([1.0, 2.0, -0.5])
    Xh /= np.linalg.norm(Xh)
    e = np.exp(1j * K * (g.khat @ d))
    P = sphere.legendre_p(6, g.khat @ Xh)
    dn = np.linalg.norm(d)
    for l in range(7):
        lhs = np.sum(g.w * e * P[l])
        rhs = 4 * math.pi * 1j ** l * sp.spherical_jn(l, K * dn) * \
            sp.eval_legendre(l, d @ Xh / dn)
        assert abs(lhs - rhs) < 1e-12


@pytest.mark.parametrize("L", [8, 13])
def test_translation_quadrature_equals_gegenbauer_series(L):
    # (ik/4pi) sum_q w_q exp(ik khat.d) T_L(khat, X) equals the truncated
    # Gegenbauer series ik sum_{l<=L} (-1)^l (2l+1) j_l(kd) h_l(kX) P_l
    g = sphere.SphereGrid(L)
    a = 0.25 if L == 8 else 0.5
    X = np.array([2 * a, a, -a])
    d = np.array([0.3, -0.2, 0.25]) * a
    T = M.translation_operator(K, L, X, g)
    quad = 1j * K / (4 * math.pi) * np.sum(g.w * np.exp(1j * K * (g.khat @ d)) * T)
    l = np.arange(L + 1)
    x, dn = np.linalg.norm(X), np.linalg.norm(d)
    cosg = (d @ X) / (dn * x)
    series = 1j * K * np.sum((-1.0) ** l * (2 * l + 1) * sp.spherical_jn(l, K * dn)
                             * (sp.spherical_jn(l, K * x) + 1j * sp.spherical_yn(l, K * x))
                             * sp.eval_legendre(l, cosg))
    # the grid integrates the plane wave's components of degree <= 2L+1-l
    # exactly; the tail beyond, ~ j_{L+2}(k|d|) h_L(k|X|), is ~1e-10 here
    assert abs(quad - series) < 1e-8 * abs(series)
    # and it approximates the kernel itself to the 3-digit design accuracy
    r = np.linalg.norm(X + d)
    exact = np.exp(1j * K * r) / r
    assert abs(quad - exact) < 2e-3 * abs(exact)


def _bandlimited(coef, grid):
    th = np.arccos(grid.khat[:, 2])
    ph = np.arctan2(grid.khat[:, 1], grid.khat[:, 0])
    f = np.zeros(grid.K, dtype=np.complex128)
    for (l, m), c in coef.items():
        f += c * sp.sph_harm_y(l, m, th, ph)
    return f.reshape(grid.ntheta, grid.nphi)


def test_interpolation_exact_on_bandlimited():
    rng = np.random.default_rng(11)
    Lc, Lp = 8, 13
    gc, gp = sphere.SphereGrid(Lc), sphere.SphereGrid(Lp)
    coef = {(l, m): rng.standard_normal() + 1j * rng.standard_normal()
            for l in range(Lc + 1) for m in range(-l, l + 1)}
    fc = _bandlimited(coef, gc)
    fp = _bandlimited(coef, gp)
    maps = M.legendre_map(Lc, gc.x, gc.wx, gp.x)
    got = M.resample(fc, Lc, gc, gp, maps)
    assert np.max(np.abs(got - fp)) < 1e-12 * np.max(np.abs(fp))


def test_anterpolation_is_band_projection():
    # parent-grid function = low band (<= Lc) + high band; anterpolation
    # keeps exactly the low band on the child grid
    rng = np.random.default_rng(12)
    Lc, Lp = 8, 13
    gc, gp = sphere.SphereGrid(Lc), sphere.SphereGrid(Lp)
    low = {(l, m): rng.standard_normal() + 1j * rng.standard_normal()
           for l in range(Lc + 1) for m in range(-l, l + 1)}
    high = {(l, m): rng.standard_normal() + 1j * rng.standard_normal()
            for l in range(Lc + 1, Lp + 1) for m in range(-l, l + 1)}
    fp = _bandlimited({**low, **high}, gp)
    maps = M.legendre_map(Lc, gp.x, gp.wx, gc.x)
    got = M.resample(fp, Lc, gp, gc, maps)
    assert np.max(np.abs(got - _bandlimited(low, gc))) < 1e-12 * np.max(np.abs(fp))


def test_anterpolation_weighted_adjoint_of_interpolation():
    # <I x, y>_{W_p} = <x, A y>_{W_c}
    rng = np.random.default_rng(13)
    Lc, Lp = 13, 20
    gc, gp = sphere.SphereGrid(Lc), sphere.SphereGrid(Lp)
    I = M.legendre_map(Lc, gc.x, gc.wx, gp.x)
    A = M.legendre_map(Lc, gp.x, gp.wx, gc.x)
    x = rng.standard_normal((gc.ntheta, gc.nphi)) + 1j * rng.standard_normal((gc.ntheta, gc.nphi))
    y = rng.standard_normal((gp.ntheta, gp.nphi)) + 1j * rng.standard_normal((gp.ntheta, gp.nphi))
    Ix = M.resample(x, Lc, gc, gp, I).ravel()
    Ay = M.resample(y, Lc, gp, gc, A).ravel()
    lhs = np.sum(gp.w * Ix * np.conj(y.ravel()))
    rhs = np.sum(gc.w * x.ravel() * np.conj(Ay))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_truncation_orders_per_level():
    # 3 digits: 0.25 -> 8, 0.5 -> 13, 1 -> 20, 2 -> 33, 4 -> 57, 8 -> 104, 16 -> 196
    got = [M.truncation_order(K, a, 3) for a in (0.25, 0.5, 1, 2, 4, 8, 16)]
    assert got == [8, 13, 20, 33, 57, 104, 196]


@pytest.mark.parametrize("L", [8, 13, 20])
def test_translation_operator_antipodal_symmetry(L):
    """T_{-X}(k) = T_X(-k): P_l(-u) = (-1)^l P_l(u) is the same sign flip
    whether the offset or the direction is negated.  On the grid, -k of
    sample (i, j) is sample (L - i, j + L + 1) (Gauss-Legendre nodes
    symmetric about the equator, 2L + 2 phi samples): the one-RHS M2L form
    that keeps one offset of each +-pair in LDS reads the other through
    that mirror."""
    g = sphere.SphereGrid(L)
    nth, nph = g.ntheta, g.nphi
    q = np.arange(g.K)
    anti = (nth - 1 - q // nph) * nph + (q % nph + nph // 2) % nph
    assert np.array_equal(anti[anti], q) and np.all(anti != q)
    assert np.allclose(g.khat[anti], -g.khat, atol=1e-15)
    a = 0.25
    for d in [(2, 0, 0), (3, -1, 2), (-2, 3, 3), (0, -2, 1)]:
        X = np.array(d, dtype=float) * a
        tp = M.translation_operator(K, L, X, g)
        tm = M.translation_operator(K, L, -X, g)
        assert np.max(np.abs(tm - tp[anti])) <= 1e-12 * np.max(np.abs(tp))
