"""GPU FFT interpolation and anterpolation between uniform sphere grids
(Sec. 3.2.2 "Fine-grained Parallel Interpolation", Fig. 3; Sec. 3.2.4)
through the C ABI, against the FP64 oracle (`oracle/fft_interp.py`).

Bound: largest element deviation over the largest reference value
<= 2e-6.  Each output is the sum of four FFT stages of at most 120 points
(about log2(120) = 7 rounding steps of 2^-24 each, on values of one
scale) plus two phase or weight multiplies, so FP32 carries it to a few
times 1e-7; the anterpolation's row factors (up to 1/w of the smallest
Fejer weight) scale a row's values and its error alike.
"""
import numpy as np
import pytest
import scipy.special as sp

from gpu_common import cuda_or_skip, max_rel, say

from oracle import fft_interp as F

pytestmark = pytest.mark.gpu

TOL = 2e-6



def _run(torch, G, lb, pi, po, ant, X):
    r = G.FFTResampler(lb, pi, po, anterpolate=ant)
    xd = torch.from_numpy(X.astype(np.complex64)).cuda()
    y = r(xd)
    torch.cuda.synchronize()
    return y.cpu().numpy(), r


def _oracle(lb, pi, po, ant, X):
    gi, go = F.UniformGrid(pi), F.UniformGrid(po)
    fn = F.anterpolate if ant else F.interpolate
    return np.stack([fn(x, lb, gi, go) for x in X.astype(np.complex128)])


CASES = [(0, 2, 4), (2, 6, 10), (5, 14, 12), (8, 18, 28), (13, 28, 42), (20, 42, 70),
         (33, 70, 120)]


@pytest.mark.parametrize("lb,pc,pp", CASES)
@pytest.mark.parametrize("ant", [False, True])
@pytest.mark.parametrize("nitems", [1, 37])
def test_fft_resample_vs_oracle(lb, pc, pp, ant, nitems):
    torch = cuda_or_skip()
    from paper_2006_15367_amd import mlfma as G
    pi, po = (pp, pc) if ant else (pc, pp)
    rng = np.random.default_rng(lb * 1000 + pi * 10 + po + nitems + ant)
    X = rng.standard_normal((nitems, pi // 2, pi)) + 1j * rng.standard_normal((nitems, pi // 2, pi))
    say("fft: lband %d, %d -> %d, %s, %d items" % (lb, pi, po, "anterp" if ant else "interp",
                                                   nitems))
    got, r = _run(torch, G, lb, pi, po, ant, X)
    assert got.shape == (nitems, po // 2, po)
    ref = _oracle(lb, pi, po, ant, X.astype(np.complex64))
    e = max_rel(got, ref)
    say("fft: max rel %.2e (items per workgroup %d)" % (e, r.info()["items_per_workgroup"]))
    assert e < TOL


def test_fft_interpolation_exact_on_spherical_harmonics():
    """The GPU interpolation of a degree-20 function against its values
    evaluated directly (scipy) on the output grid."""
    torch = cuda_or_skip()
    from paper_2006_15367_amd import mlfma as G
    lb, pi, po = 20, 42, 70
    rng = np.random.default_rng(5)
    gi, go = F.UniformGrid(pi), F.UniformGrid(po)

    def ev(g, coef):
        th = np.repeat(g.theta, g.nphi)
        ph = np.tile(g.phi, g.ntheta)
        f = sum(c * sp.sph_harm_y(l, m, th, ph) for (l, m), c in coef.items())
        return f.reshape(g.ntheta, g.nphi)

    coef = {(l, m): rng.standard_normal() + 1j * rng.standard_normal()
            for l in range(lb + 1) for m in range(-l, l + 1)}
    got, _ = _run(torch, G, lb, pi, po, False, ev(gi, coef)[None])
    e = max_rel(got[0], ev(go, coef))
    say("fft: spherical harmonics to degree 20, 42 -> 70: max rel %.2e" % e)
    assert e < TOL


@pytest.mark.parametrize("ant", [False, True])
def test_fft_full_size_level_pairs(ant):
    """The level pairs of the 262,144-point sphere (orders 8, 13, 20, 33, 57
    on uniform grids of 18, 28, 42, 70, 120 phi samples), one item per
    child box (17,334, 4,593, 1,160, 272): 64 sampled items and the first
    and last against the oracle."""
    torch = cuda_or_skip()
    from paper_2006_15367_amd import mlfma as G
    pairs = [(8, 18, 28, 17334), (13, 28, 42, 4593), (20, 42, 70, 1160), (33, 70, 120, 272)]
    for lb, pc, pp, n in pairs:
        pi, po = (pp, pc) if ant else (pc, pp)
        rng = np.random.default_rng(pi + po + n)
        X = (rng.standard_normal((n, pi // 2, pi)) +
             1j * rng.standard_normal((n, pi // 2, pi))).astype(np.complex64)
        say("fft full: lband %d, %d -> %d, %d items, %s" % (lb, pi, po, n,
                                                             "anterp" if ant else "interp"))
        got, _ = _run(torch, G, lb, pi, po, ant, X)
        idx = np.unique(np.concatenate([[0, n - 1], rng.choice(n, 64, replace=False)]))
        ref = _oracle(lb, pi, po, ant, X[idx])
        e = max_rel(got[idx], ref)
        say("fft full: max rel %.2e" % e)
        assert e < TOL


def test_fft_empty_batch_is_a_noop():
    torch = cuda_or_skip()
    from paper_2006_15367_amd import mlfma as G
    r = G.FFTResampler(8, 18, 28)
    x = torch.empty((0, 9, 18), dtype=torch.complex64, device="cuda")
    y = r(x)
    torch.cuda.synchronize()
    assert tuple(y.shape) == (0, 14, 28)


def test_fft_overlapping_buffers_rejected():
    torch = cuda_or_skip()
    from paper_2006_15367_amd import mlfma as G
    r = G.FFTResampler(8, 18, 18)
    x = torch.zeros((4, 9, 18), dtype=torch.complex64, device="cuda")
    with pytest.raises(G.MlfmaError) as e:
        r(x, out=x)
    assert e.value.status == G.EINVAL
    y = r(x)
    torch.cuda.synchronize()
    assert tuple(y.shape) == (4, 9, 18)
