"""Sampled and interpolated translation operators, FP64 (oracle; test
infrastructure only: only tests, the smoke check and the bench's CPU
baseline may import it).

The paper stores precomputed translation operators and, when memory does
not suffice, samples them and interpolates (Sec. 3.2.3, paragraph
"Translation Operators").  The diagonal operator of an offset X,

    T_L(khat, X) = sum_{l=0}^{L} i^l (2l + 1) h_l(k|X|) P_l(khat . Xhat),

depends on the direction only through the angle gamma between khat and
Xhat, and P_l(cos gamma) is a cosine polynomial of degree l, so T is a
trigonometric polynomial of degree L in gamma, even and 2 pi periodic.
One table per distinct |X| holds T at gamma_m = m pi / M, m = 0..M,
M = s L (s-fold oversampling of the band); a direction's value is the
p-point Lagrange interpolant through the samples around its angle, samples
beyond 0 or pi taken from the mirror images (T(-g) = T(g),
T(pi + g) = T(pi - g)).

Error bound (Lagrange remainder with Bernstein's inequality
|f^(p)| <= L^p max|f| for a trigonometric polynomial of degree L, applied
to the real and imaginary parts):
    |error| <= sqrt(2) max|T| (L pi / M)^p omega_p / p!,
    omega_p = max over x in [0, 1] of prod_{i=1-p/2}^{p/2} |x - i|.
"""
import math

import numpy as np

from oracle import sphere
from oracle import mlfma as M

S_OVERSAMPLE = 8
P_POINTS = 10


def series(k, L, r, u):
    """T_L at cos(angle) = u for an offset of length r (the definition)."""
    h = sphere.spherical_hankel1(L, k * r)
    P = sphere.legendre_p(L, np.asarray(u, dtype=np.float64))
    coef = (1j ** np.arange(L + 1)) * (2 * np.arange(L + 1) + 1) * h
    return np.tensordot(coef, P, axes=(0, 0))


def table(k, L, r, s=S_OVERSAMPLE):
    """Samples T(gamma_m), gamma_m = m pi / M, m = 0..M, M = s L."""
    Mi = int(s * L)
    return series(k, L, r, np.cos(np.arange(Mi + 1) * np.pi / Mi)), Mi


def interpolate(tab, Mi, gamma, p=P_POINTS):
    """p-point Lagrange interpolation of the table at angles gamma in
    [0, pi]: nodes m0 .. m0 + p - 1 with m0 = floor(x) - (p/2 - 1),
    x = gamma M / pi; indices below 0 or above M reflect."""
    gamma = np.asarray(gamma, dtype=np.float64)
    x = gamma * Mi / np.pi
    m0 = np.floor(x).astype(np.int64) - (p // 2 - 1)
    out = np.zeros(gamma.shape, dtype=np.complex128)
    for j in range(p):
        w = np.ones(gamma.shape)
        for i in range(p):
            if i != j:
                w = w * (x - (m0 + i)) / (j - i)
        m = np.abs(m0 + j)
        m = np.where(m > Mi, 2 * Mi - m, m)
        out += w * tab[m]
    return out


def omega(p):
    """max over x in [0, 1] of prod_{i=1-p/2}^{p/2} |x - i| (dense scan;
    the maximum is at x = 1/2 by symmetry and log-concavity)."""
    xs = np.linspace(0.0, 1.0, 20001)
    prod = np.ones_like(xs)
    for i in range(1 - p // 2, p // 2 + 1):
        prod *= np.abs(xs - i)
    return float(prod.max())


def error_bound(L, Mi, p, tmax):
    return math.sqrt(2.0) * tmax * (L * math.pi / Mi) ** p * omega(p) / math.factorial(p)


def operator(k, L, X, grid, s=S_OVERSAMPLE, p=P_POINTS):
    """T_L(khat, X) on the grid's directions through the sampled table."""
    X = np.asarray(X, dtype=np.float64)
    r = float(np.linalg.norm(X))
    tab, Mi = table(k, L, r, s)
    u = np.clip(grid.khat @ (X / r), -1.0, 1.0)
    return interpolate(tab, Mi, np.arccos(u), p)


def sampled_operators(ops, s=S_OVERSAMPLE, p=P_POINTS):
    """The oracle's operators with every translation operator replaced by
    its sampled-and-interpolated value (everything else unchanged)."""
    out = M.Operators.__new__(M.Operators)
    out.__dict__.update(ops.__dict__)
    out.T = {}
    for lev, tab in ops.T.items():
        a = ops.tree.levels[lev].a
        new = {}
        for t in tab:
            dx, rem = divmod(int(t), 49)
            dy, dz = divmod(rem, 7)
            X = a * np.array([dx - 3, dy - 3, dz - 3], dtype=np.float64)
            new[t] = operator(ops.k, ops.L[lev], X, ops.grid[lev], s, p)
        out.T[lev] = new
    return out
