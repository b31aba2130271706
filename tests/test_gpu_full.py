"""Full-size workloads in the launch configuration the benchmark uses,
checked on sampled outputs against the dense definition (the oracle
evaluates those targets one by one)."""
import numpy as np
import pytest

from gpu_common import cuda_or_skip, rel_l2, say

from paper_2006_15367_amd import workloads as W

pytestmark = pytest.mark.gpu

K = W.K_WAVENUMBER


def _run_full(name, ntargets, bf16x3=False):
    torch = cuda_or_skip()
    from oracle import dense
    from paper_2006_15367_amd import mlfma as G
    xyz, q = W.make(name)
    R = 1 if q.ndim == 1 else q.shape[1]
    say("full:", name, "N=%d R=%d bf16x3=%s" % (xyz.shape[0], R, bf16x3))
    tree = G.Tree(xyz, W.LEAF_SIZE)
    ops = G.Operators(tree, K, W.DIGITS, max_rhs=R, bf16x3=bf16x3)
    phi = ops.matvec(torch.from_numpy(q).cuda())
    torch.cuda.synchronize()
    phi = phi.cpu().numpy()
    assert np.all(np.isfinite(phi))
    rng = np.random.default_rng(51)
    idx = rng.choice(xyz.shape[0], ntargets, replace=False)
    ref = dense.potential(xyz, q, K, tgt=xyz[idx])
    err = rel_l2(phi[idx], ref)
    say(name, "sampled rel L2 vs dense", err, "levels", tree.info()["n_levels"])
    return err


def test_full_sphere262k():
    assert _run_full("sphere262k", 512) < 1e-3


def test_full_spheroid1m():
    assert _run_full("spheroid1m", 256) < 1e-3


def test_full_sphere262k_r64_bf16x3():
    assert _run_full("sphere262k_r64", 64, bf16x3=True) < 1e-3


def test_full_cube1m_r16():
    assert _run_full("cube1m_r16", 96) < 1e-3
