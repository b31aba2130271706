"""The allocation-free GMRES entry point (mlfma_solve_gmres_noalloc)
against the allocating one (mlfma_solve_gmres), through the C ABI.

Both run the same kernels in the same order on the same handle, the one on
the library's fixed device scratch and the other on the handle's own
workspace, so the solutions, step counts and residuals agree exactly.  Two
calls in a row, the second on a smaller point set; then a request larger
than the scratch is refused with MLFMA_ENOMEM before any work."""
import ctypes
import math

import numpy as np
import pytest

from gpu_common import cuda_or_skip, rel_l2, say

from paper_2006_15367_amd import workloads as W

pytestmark = pytest.mark.gpu

K = W.K_WAVENUMBER
SHIFT = 1000j


def _solve(G, ops, b, name, restart=30):
    """One solve through the named C entry point; x starts at zero."""
    torch = cuda_or_skip()
    x = torch.zeros_like(b)
    it = ctypes.c_int(-1)
    rr = ctypes.c_double(-1.0)
    fn = getattr(G._load(), name)
    st = fn(ops._h, b.data_ptr(), x.data_ptr(), SHIFT.real, SHIFT.imag, restart, 300,
            1e-5, ctypes.byref(it), ctypes.byref(rr), None)
    torch.cuda.synchronize()
    return st, x.cpu().numpy(), it.value, rr.value


def _case(n, radius, seed):
    from paper_2006_15367_amd import mlfma as G
    torch = cuda_or_skip()
    rng = np.random.default_rng(seed)
    xyz = W.sphere_points(rng, n, radius)
    b = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
    tree = G.Tree(xyz, W.LEAF_SIZE)
    ops = G.Operators(tree, K, W.DIGITS, max_rhs=1)
    return G, ops, torch.from_numpy(b).cuda()


def test_noalloc_solve_equals_allocating_solve():
    for n, radius, seed in ((4096, 1.0, 71), (2048, 0.8, 72)):
        say("no-alloc GMRES: n = %d (sphere radius %.1f)" % (n, radius))
        G, ops, b = _case(n, radius, seed)
        st0, x0, it0, r0 = _solve(G, ops, b, "mlfma_solve_gmres")
        st1, x1, it1, r1 = _solve(G, ops, b, "mlfma_solve_gmres_noalloc")
        assert st0 == G.OK and st1 == G.OK
        say("  steps %d / %d, residual %.3e / %.3e, rel diff %.2e"
            % (it0, it1, r0, r1, rel_l2(x1, x0)))
        assert 0 < it0 <= 300 and r0 <= 1e-5
        assert it1 == it0 and r1 == r0
        assert np.array_equal(x1, x0)


def test_noalloc_solve_refuses_more_than_its_scratch():
    from paper_2006_15367_amd import mlfma as G
    torch = cuda_or_skip()
    xyz, q = W.make("sphere262k")
    say("no-alloc GMRES: size limit on the 262k sphere")
    tree = G.Tree(xyz, W.LEAF_SIZE)
    ops = G.Operators(tree, K, W.DIGITS, max_rhs=1, autotune=False)
    b = torch.from_numpy(q.astype(np.complex64)).cuda()
    st, x, it, rr = _solve(G, ops, b, "mlfma_solve_gmres_noalloc", restart=30)
    assert st == G.ENOMEM
    assert it == 0 and rr == 0.0
    assert np.all(x == 0)
    # restart 29 fits: (29 + 2) x 2 MiB of basis plus the partial sums
    st, x, it, rr = _solve(G, ops, b, "mlfma_solve_gmres_noalloc", restart=29)
    assert st == G.OK and it > 0
