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


def test_onepass_work_splits_agree_sphere262k():
    """Every one-pass work split of the two lowest level pairs (bands 8 -> 13
    and 13 -> 20) gives the three-pass result of the 262k sphere at 4 RHS
    (FP32 reassociation only), and one of them matches the dense definition
    on sampled targets."""
    torch = cuda_or_skip()
    from oracle import dense
    from paper_2006_15367_amd import mlfma as G
    xyz, q = W.make("sphere262k", nrhs=4)
    say("full: one-pass work splits, sphere262k, 4 RHS")
    tree = G.Tree(xyz, W.LEAF_SIZE)
    ops = G.Operators(tree, K, W.DIGITS, max_rhs=4, autotune=False)
    nl = tree.info()["n_levels"]
    qd = torch.from_numpy(q.astype(np.complex64)).cuda()
    pairs = {nl - 1: 3, nl - 2: 2}  # level of the pair -> number of splits
    for k in ("interp", "anterp"):
        for l in range(3, nl):
            ops.set_variant(l, 0, kernel=k)
    ref = ops.matvec(qd).cpu().numpy()
    for v in (1, 2, 3):
        for k in ("interp", "anterp"):
            for l, nsh in pairs.items():
                ops.set_variant(l, min(v, nsh), kernel=k)
        say("one-pass variant", v)
        got = ops.matvec(qd).cpu().numpy()
        torch.cuda.synchronize()
        err = rel_l2(got, ref)
        say("variant", v, "rel L2 vs three passes", err)
        assert err < 1e-5, (v, err)
    rng = np.random.default_rng(52)
    idx = rng.choice(xyz.shape[0], 128, replace=False)
    dref = dense.potential(xyz, q[:, 1], K, tgt=xyz[idx])
    assert rel_l2(got[idx, 1], dref) < 1e-3
