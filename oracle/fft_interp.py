"""FFT interpolation and anterpolation between uniform sphere grids, FP64
(oracle; test infrastructure only: only tests, the smoke check and the
bench's CPU baseline may import it).

The paper's M2M brings a child's samples to the parent's sampling with FFT
interpolation over equispaced samples in theta and phi (Sec. 3.2.2,
paragraph "Fine-grained Parallel Interpolation", and Fig. 3, after Sarvas):
independent FFT interpolations along phi first; then the samples are
transposed and folded so that every phi column, together with the column
half a turn away, becomes a whole circle of theta samples, and FFT
interpolation runs along those circles; the result is transposed and
unfolded back into a (theta, phi) array.  L2L runs the reverse,
anterpolation (Sec. 3.2.4: the same procedure with the sample count
reduced).  This module takes those steps in that order with numpy's FFT.

Grid (UniformGrid): P phi samples phi_j = 2 pi j / P (P even) and P / 2
theta samples theta_i = (i + 1/2) 2 pi / P.  A function on the sphere,
read along the great circle through phi_j and phi_j + pi, is periodic in
theta with period 2 pi:  f(2 pi - theta, phi) = f(theta, phi + pi).  The
circle through column j holds P equispaced samples at (s + 1/2) 2 pi / P,
s = 0..P-1: s < P/2 is theta_s in column j, s >= P/2 is theta_{P-1-s} in
column j + P/2.  A spherical harmonic of degree l is, along phi, a
trigonometric polynomial of degree <= l and, along such a circle, one of
degree <= l as well, so both FFT stages are exact for functions of degree
<= Lband when P >= 2 Lband + 2 on both grids.

Anterpolation is the weighted adjoint of interpolation,
A = W_out^-1 I^T W_in, with I the interpolation from the output grid to the
input grid and W the quadrature weights (Fejer's first rule in theta times
2 pi / P in phi): for every function g of degree <= Lband the anterpolated
samples integrate against g on the coarse grid as the original samples do
on the fine grid.  Transposing each FFT stage gives the same stages run in
reverse order (theta circles first, then phi), each resampling from the
fine grid to the coarse one, times P_in / P_out per stage.
"""
import numpy as np


def fejer_weights(nt):
    """Fejer's first rule on theta_i = (i + 1/2) pi / nt for the integral
    int_0^pi f(theta) sin(theta) d theta: exact when f is a polynomial in
    cos(theta) of degree <= nt - 1.
      w_i = (2 / nt) [1 - 2 sum_{k=1}^{floor(nt/2)} cos(2 k theta_i) / (4 k^2 - 1)]
    """
    th = (np.arange(nt) + 0.5) * np.pi / nt
    s = np.zeros(nt)
    for k in range(1, nt // 2 + 1):
        s += np.cos(2 * k * th) / (4.0 * k * k - 1.0)
    return 2.0 / nt * (1.0 - 2.0 * s)


class UniformGrid:
    """Equispaced grid of P phi samples and P / 2 theta samples (no poles);
    samples stored row-major [theta][phi], phi fastest."""

    def __init__(self, P):
        P = int(P)
        if P < 2 or P % 2:
            raise ValueError("P must be even and >= 2")
        self.nphi = P
        self.ntheta = P // 2
        self.K = self.ntheta * self.nphi
        self.theta = (np.arange(self.ntheta) + 0.5) * 2.0 * np.pi / P
        self.phi = 2.0 * np.pi * np.arange(P) / P
        self.wtheta = fejer_weights(self.ntheta)
        self.w = (self.wtheta[:, None] * (2.0 * np.pi / P)
                  * np.ones((1, P))).reshape(self.K)


def resample_periodic(X, Lband, n_out, offset):
    """Trigonometric interpolation along the last axis: X holds n_in
    equispaced samples at (s + offset) 2 pi / n_in of a periodic function;
    return its band-limited (|frequency| <= Lband) interpolant at the n_out
    points (s + offset) 2 pi / n_out.  FFT, drop the frequencies above the
    band, zero-pad to n_out, inverse FFT; the sample offset enters as a
    phase per frequency."""
    n_in = X.shape[-1]
    if n_in < 2 * Lband + 1 or n_out < 2 * Lband + 1:
        raise ValueError("grid too coarse for the band")
    c = np.fft.fft(X, axis=-1) / n_in
    f = np.arange(-Lband, Lband + 1)
    # coefficient of exp(i f x): the DFT of samples at (s + offset) h is
    # sum_s X_s exp(-i f s h), so the coefficient carries exp(-i f offset h)
    coef = c[..., f % n_in] * np.exp(-1j * f * offset * 2.0 * np.pi / n_in)
    out = np.zeros(X.shape[:-1] + (n_out,), dtype=np.complex128)
    out[..., f % n_out] = coef * np.exp(1j * f * offset * 2.0 * np.pi / n_out)
    return np.fft.ifft(out, axis=-1) * n_out


def fold(Y):
    """[..., nt, P] (theta, phi) -> [..., P/2, 2 nt] theta circles: circle j
    holds column j top to bottom, then column j + P/2 bottom to top."""
    P = Y.shape[-1]
    h = P // 2
    top = np.swapaxes(Y[..., :, :h], -1, -2)
    bottom = np.swapaxes(Y[..., ::-1, h:], -1, -2)
    return np.concatenate([top, bottom], axis=-1)


def unfold(C):
    """Inverse of fold: [..., P/2, 2 nt] circles -> [..., nt, P]."""
    nt = C.shape[-1] // 2
    left = np.swapaxes(C[..., :nt], -1, -2)
    right = np.swapaxes(C[..., nt:][..., ::-1], -1, -2)
    return np.concatenate([left, right], axis=-1)


def interpolate(X, Lband, g_in, g_out):
    """M2M interpolation (Sec. 3.2.2, Fig. 3): X [..., nt_in, P_in] ->
    [..., nt_out, P_out], keeping degrees <= Lband.
      1. FFT interpolation of every theta row along phi (P_in -> P_out);
      2. transpose and fold: the columns j and j + P_out/2 become one
         theta circle of P_in samples;
      3. FFT interpolation along every circle (P_in -> P_out samples, both
         at half-sample offsets);
      4. transpose and unfold back to (theta, phi)."""
    Y1 = resample_periodic(X, Lband, g_out.nphi, 0.0)
    C = fold(Y1)
    C2 = resample_periodic(C, Lband, g_out.nphi, 0.5)
    return unfold(C2)


def anterpolate(Y, Lband, g_in, g_out):
    """L2L anterpolation (Sec. 3.2.4), the weighted adjoint of
    interpolate(., Lband, g_out, g_in):
      A Y = (P_in / P_out) diag(1 / w_out) D(diag(w_in) Y),
    with w the Fejer theta weights of each grid and D the transposed
    stages in reverse order: fold the input, FFT-resample every theta
    circle (P_in -> P_out), unfold to [nt_out, P_in], FFT-resample every
    row along phi (P_in -> P_out)."""
    Z = Y * g_in.wtheta[:, None]
    C = resample_periodic(fold(Z), Lband, g_out.nphi, 0.5)
    Z2 = resample_periodic(unfold(C), Lband, g_out.nphi, 0.0)
    return Z2 * (g_in.nphi / g_out.nphi) / g_out.wtheta[:, None]
