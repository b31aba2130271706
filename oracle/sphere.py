"""Quadrature on the unit sphere and special functions, FP64 (oracle; test
infrastructure only).

The paper treats a multipole or local expansion as a 2-D array of samples of
a function on the sphere over (theta, phi) (Sec. 2, related-work paragraph;
Sec. 3.2.2) and relies on exact ("global") interpolation between levels
(Sec. 2, related work).  The mathematics of the diagonal plane-wave form is
deferred by the paper to its references (Sec. 2, list of five stages).  This
module writes out the textbook pieces that form needs:

- the (L+1)-point Gauss-Legendre rule in cos(theta) and the uniform phi grid
  with 2L+2 points, which together integrate spherical harmonics of degree
  <= 2L+1 exactly;
- associated Legendre functions normalised to unit L2 norm on [-1, 1];
- Legendre polynomials;
- spherical Hankel functions of the first kind.
"""
import numpy as np


def gauss_legendre(n):
    """Nodes and weights of the n-point Gauss-Legendre rule on [-1, 1].

    Nodes are returned in DESCENDING order of x (so theta = arccos(x) is
    ascending).  Newton's method on P_n, evaluated with the three-term
    recurrence, from the classical cosine initial guesses.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    i = np.arange(1, n + 1, dtype=np.float64)
    x = np.cos(np.pi * (i - 0.25) / (n + 0.5))
    for _ in range(100):
        p_prev = np.ones_like(x)
        p = x.copy()
        for l in range(2, n + 1):
            p_prev, p = p, ((2 * l - 1) * x * p - (l - 1) * p_prev) / l
        dp = n * (x * p - p_prev) / (x * x - 1.0)
        dx = p / dp
        x = x - dx
        if np.max(np.abs(dx)) < 1e-15:
            break
    # final derivative at the converged nodes
    p_prev = np.ones_like(x)
    p = x.copy()
    for l in range(2, n + 1):
        p_prev, p = p, ((2 * l - 1) * x * p - (l - 1) * p_prev) / l
    dp = n * (x * p - p_prev) / (x * x - 1.0)
    w = 2.0 / ((1.0 - x * x) * dp * dp)
    return x, w


def legendre_p(lmax, u):
    """P_l(u) for l = 0..lmax, shape [lmax+1, *u.shape] (three-term recurrence)."""
    u = np.asarray(u, dtype=np.float64)
    out = np.empty((lmax + 1,) + u.shape)
    out[0] = 1.0
    if lmax >= 1:
        out[1] = u
    for l in range(1, lmax):
        out[l + 1] = ((2 * l + 1) * u * out[l] - l * out[l - 1]) / (l + 1)
    return out


def assoc_legendre_normalised(lmax, m, x):
    """Pbar_l^m(x) for l = m..lmax, shape [lmax-m+1, len(x)].

    Pbar_l^m is the associated Legendre function scaled so that
    int_{-1}^{1} Pbar_l^m(x)^2 dx = 1.  The Condon-Shortley sign is left
    out (every use here multiplies two functions of the same m, where the
    sign cancels).  Computed with the normalised recurrences, which stay
    finite near the poles for large m (values that would underflow become 0).
    """
    x = np.asarray(x, dtype=np.float64)
    s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    if m > lmax:
        return np.zeros((0, x.size))
    pmm = np.full(x.shape, np.sqrt(0.5))
    for mm in range(1, m + 1):
        pmm = np.sqrt((2.0 * mm + 1.0) / (2.0 * mm)) * s * pmm
    out = np.empty((lmax - m + 1, x.size))
    out[0] = pmm
    if lmax >= m + 1:
        out[1] = np.sqrt(2.0 * m + 3.0) * x * pmm
    for l in range(m + 2, lmax + 1):
        a = np.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
        b = np.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
        out[l - m] = a * (x * out[l - m - 1] - b * out[l - m - 2])
    return out


def spherical_hankel1(lmax, x):
    """h_l^(1)(x) for l = 0..lmax, x > 0 scalar; upward recurrence.

    h_0 = -i e^{ix}/x, h_1 = -e^{ix}(x+i)/x^2,
    h_{l+1} = (2l+1)/x h_l - h_{l-1}  (stable upward for h^(1)).
    """
    x = float(x)
    h = np.empty(lmax + 1, dtype=np.complex128)
    e = np.exp(1j * x)
    h[0] = -1j * e / x
    if lmax >= 1:
        h[1] = -e * (x + 1j) / (x * x)
    for l in range(1, lmax):
        h[l + 1] = (2 * l + 1) / x * h[l] - h[l - 1]
    return h


class SphereGrid:
    """Sample grid of one tree level (truncation order L).

    theta_i = arccos(x_i) with x_i the L+1 Gauss-Legendre nodes (theta
    ascending); phi_j = 2 pi j / (2L+2).  Quadrature weight of sample (i, j)
    is w_i * 2 pi / (2L+2); the weights sum to 4 pi.  Samples are stored
    row-major [theta][phi], phi fastest.
    """

    def __init__(self, L):
        self.L = int(L)
        self.ntheta = self.L + 1
        self.nphi = 2 * self.L + 2
        self.K = self.ntheta * self.nphi
        self.x, self.wx = gauss_legendre(self.ntheta)
        self.theta = np.arccos(self.x)
        self.phi = 2.0 * np.pi * np.arange(self.nphi) / self.nphi
        st = np.sin(self.theta)[:, None]
        ct = np.cos(self.theta)[:, None]
        self.khat = np.stack(
            [st * np.cos(self.phi)[None, :],
             st * np.sin(self.phi)[None, :],
             np.broadcast_to(ct, (self.ntheta, self.nphi))],
            axis=-1).reshape(self.K, 3)
        self.w = (self.wx[:, None] * (2.0 * np.pi / self.nphi)
                  * np.ones((1, self.nphi))).reshape(self.K)
