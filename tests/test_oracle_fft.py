"""Pins of the oracle's FFT interpolation and anterpolation on uniform
sphere grids (Sec. 3.2.2 "Fine-grained Parallel Interpolation", Fig. 3;
Sec. 3.2.4).

Every check is against something the mathematics fixes, not against the
oracle's own code:

* Fejer's rule against the closed-form moments of cos(theta)^k sin(theta);
* interpolation of functions of degree <= Lband (sums of spherical
  harmonics from scipy) reproduces their values on the output grid;
* interpolation of the folded trigonometric functions
  exp(i m phi) (exp(i n theta) + (-1)^m exp(-i n theta)), |m|, |n| <= Lband
  (the closed form of what the two FFT stages represent) is exact;
* the tiny case against an interpolation written out as direct sums of
  Dirichlet kernels over the samples (no FFT, no fold helpers);
* anterpolation: the weighted-adjoint identity
  sum w_c (A y)_c g_c = sum w_p y_p (I g)_p on random data, and the
  property L2L needs: for every g of degree <= Lband the anterpolated
  samples integrate against g on the coarse grid as the fine samples do;
  a copy without the quadrature weights fails that property.  (The
  anterpolated samples are not the pointwise band projection: multiplying
  by the theta weights leaves the band, so only integrals against
  band-limited functions are preserved, which is all that L2L and L2O
  use.)
"""
import numpy as np
import pytest
import scipy.special as sp

from oracle import fft_interp as F


def _band_limited(rng, Lb, grid):
    """Random sum of spherical harmonics of degree <= Lb on a grid (and the
    coefficients, to evaluate the same function elsewhere)."""
    coef = {(l, m): rng.standard_normal() + 1j * rng.standard_normal()
            for l in range(Lb + 1) for m in range(-l, l + 1)}
    return coef, _eval(coef, grid)


def _eval(coef, grid):
    th = np.repeat(grid.theta, grid.nphi)
    ph = np.tile(grid.phi, grid.ntheta)
    f = np.zeros(th.size, dtype=np.complex128)
    for (l, m), c in coef.items():
        f += c * sp.sph_harm_y(l, m, th, ph)
    return f.reshape(grid.ntheta, grid.nphi)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("nt", [1, 2, 5, 9, 16, 35, 60])
def test_fejer_moments(nt):
    w = F.fejer_weights(nt)
    th = (np.arange(nt) + 0.5) * np.pi / nt
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(nt):
        exact = (1.0 + (-1.0) ** k) / (k + 1.0)
        assert abs(np.sum(w * np.cos(th) ** k) - exact) < 1e-13, (nt, k)
    if 2 <= nt <= 16:
        # and the degree is tight: cos^nt (nt even) or cos^(nt+1) is not
        # (for larger nt the miss falls below FP64 resolution)
        k = nt if nt % 2 == 0 else nt + 1
        exact = (1.0 + (-1.0) ** k) / (k + 1.0)
        assert abs(np.sum(w * np.cos(th) ** k) - exact) > 1e-10


CASES = [(2, 6, 10), (3, 8, 12), (8, 18, 28), (8, 18, 32), (13, 28, 42), (20, 42, 70),
         (5, 14, 12), (6, 14, 14), (0, 2, 4)]


@pytest.mark.parametrize("Lb,Pi,Po", CASES)
def test_interpolation_exact_on_spherical_harmonics(Lb, Pi, Po):
    rng = np.random.default_rng(100 + Lb + Pi + Po)
    gi, go = F.UniformGrid(Pi), F.UniformGrid(Po)
    coef, fi = _band_limited(rng, Lb, gi)
    fo = _eval(coef, go)
    got = F.interpolate(fi, Lb, gi, go)
    assert got.shape == (go.ntheta, go.nphi)
    assert _rel(got, fo) < 1e-12


@pytest.mark.parametrize("Lb,Pi,Po", [(3, 8, 12), (8, 18, 28), (5, 14, 12)])
def test_interpolation_exact_on_folded_trig_functions(Lb, Pi, Po):
    gi, go = F.UniformGrid(Pi), F.UniformGrid(Po)

    def h(g, m, n):
        th, ph = g.theta[:, None], g.phi[None, :]
        return np.exp(1j * m * ph) * (np.exp(1j * n * th) + (-1) ** m * np.exp(-1j * n * th))

    for m in range(-Lb, Lb + 1):
        for n in range(0, Lb + 1):
            if n == 0 and m % 2:
                continue                # identically zero
            got = F.interpolate(h(gi, m, n), Lb, gi, go)
            assert _rel(got, h(go, m, n)) < 1e-12, (m, n)


def test_interpolation_tiny_vs_direct_sums():
    """Lband 2, 6 -> 10 samples: the output written as direct sums.  Along
    phi, Dirichlet kernel D_P(x) = (1/P) sum_{|f|<=2} exp(i f x); the
    great circle through phi' holds the value at polar angle t of the
    function at (t, phi') for t in (0, pi) and at (2 pi - t, phi' + pi)
    for t in (pi, 2 pi)."""
    Lb, Pi, Po = 2, 6, 10
    rng = np.random.default_rng(7)
    gi, go = F.UniformGrid(Pi), F.UniformGrid(Po)
    X = rng.standard_normal((gi.ntheta, Pi)) + 1j * rng.standard_normal((gi.ntheta, Pi))

    def D(P, x):
        return sum(np.exp(1j * f * x) for f in range(-Lb, Lb + 1)) / P

    def phi_interp(i, phi):
        return sum(X[i, j] * D(Pi, phi - gi.phi[j]) for j in range(Pi))

    out = np.empty((go.ntheta, Po), dtype=np.complex128)
    for a in range(go.ntheta):
        for b in range(Po):
            t_out, p_out = go.theta[a], go.phi[b]
            total = 0.0
            for s in range(Pi):              # samples on the input circle
                t = (s + 0.5) * 2.0 * np.pi / Pi
                if t < np.pi:
                    val = phi_interp(s, p_out)
                else:
                    val = phi_interp(Pi - 1 - s, p_out + np.pi)
                total += val * D(Pi, t_out - t)
            out[a, b] = total
    got = F.interpolate(X, Lb, gi, go)
    assert _rel(got, out) < 1e-13


@pytest.mark.parametrize("Lb,Pc,Pp", [(2, 6, 10), (8, 18, 28), (13, 28, 42), (5, 12, 14)])
def test_anterpolation_weighted_adjoint(Lb, Pc, Pp):
    rng = np.random.default_rng(200 + Lb)
    gc, gp = F.UniformGrid(Pc), F.UniformGrid(Pp)
    y = rng.standard_normal((gp.ntheta, Pp)) + 1j * rng.standard_normal((gp.ntheta, Pp))
    g = rng.standard_normal((gc.ntheta, Pc)) + 1j * rng.standard_normal((gc.ntheta, Pc))
    Ay = F.anterpolate(y, Lb, gp, gc)
    Ig = F.interpolate(g, Lb, gc, gp)
    lhs = np.sum(gc.w * (Ay * g).ravel())
    rhs = np.sum(gp.w * (y * Ig).ravel())
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


def _unweighted_anterpolate(Y, Lb, g_in, g_out):
    """A planted mistake: the transposed stages without the quadrature
    weights (plain band truncation)."""
    C = F.resample_periodic(F.fold(Y), Lb, g_out.nphi, 0.5)
    return F.resample_periodic(F.unfold(C), Lb, g_out.nphi, 0.0)


@pytest.mark.parametrize("Lb,Pc,Pp", [(3, 8, 12), (8, 18, 28), (13, 28, 42)])
def test_anterpolation_preserves_integrals_against_band_limited(Lb, Pc, Pp):
    """L2L's requirement: a local expansion is only ever integrated against
    functions of degree <= Lband (plane waves truncated at the child's
    band); the anterpolated samples must give the same integrals."""
    rng = np.random.default_rng(300 + Lb)
    gc, gp = F.UniformGrid(Pc), F.UniformGrid(Pp)
    y = rng.standard_normal((gp.ntheta, Pp)) + 1j * rng.standard_normal((gp.ntheta, Pp))
    Ay = F.anterpolate(y, Lb, gp, gc)
    Ay_bad = _unweighted_anterpolate(y, Lb, gp, gc)
    worst_bad = 0.0
    for trial in range(3):
        coef, gcs = _band_limited(rng, Lb, gc)
        gps = _eval(coef, gp)
        fine = np.sum(gp.w * (y * gps).ravel())
        coarse = np.sum(gc.w * (Ay * gcs).ravel())
        assert abs(coarse - fine) < 1e-11 * np.sum(gp.w * np.abs(y * gps).ravel())
        bad = np.sum(gc.w * (Ay_bad * gcs).ravel())
        worst_bad = max(worst_bad, abs(bad - fine) / abs(fine))
    assert worst_bad > 1e-3


def test_bad_sizes_rejected():
    with pytest.raises(ValueError):
        F.UniformGrid(7)
    with pytest.raises(ValueError):
        F.interpolate(np.zeros((3, 6)), 3, F.UniformGrid(6), F.UniformGrid(10))


def _interp_with_mistake(X, Lb, gi, go, mistake):
    Y1 = F.resample_periodic(X, Lb, go.nphi, 0.0)
    if mistake == "fold_not_reversed":
        h = go.nphi // 2
        C = np.concatenate([Y1[:, :h].T, Y1[:, h:].T], axis=-1)
    else:
        C = F.fold(Y1)
    off = 0.0 if mistake == "no_half_sample_phase" else 0.5
    return F.unfold(F.resample_periodic(C, Lb, go.nphi, off))


@pytest.mark.parametrize("mistake", [None, "fold_not_reversed", "no_half_sample_phase"])
def test_planted_interpolation_mistakes_are_seen(mistake):
    Lb, Pi, Po = 8, 18, 28
    rng = np.random.default_rng(12)
    gi, go = F.UniformGrid(Pi), F.UniformGrid(Po)
    coef, fi = _band_limited(rng, Lb, gi)
    err = _rel(_interp_with_mistake(fi, Lb, gi, go, mistake), _eval(coef, go))
    if mistake is None:
        assert err < 1e-12
    else:
        assert err > 1e-2
