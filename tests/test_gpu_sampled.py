"""GPU M2L with sampled and interpolated translation operators
(MLFMA_SAMPLED_OPERATORS; Sec. 3.2.3 "Translation Operators") through the
C ABI, against the FP64 oracle (`oracle/sampled_ops.py`, `oracle/mlfma.py`).

The interpolated operators differ from the exact ones by less than 3e-8 of
their largest value (the oracle's pinned bound) plus the FP32 evaluation in
the kernel (the angle from atan2 of the cross and dot products, error about
1e-7 rad, times |dT/dgamma| <= L max|T| by Bernstein's inequality: 6e-6 of
max|T| at L = 57; the Lagrange weights in FP32, a few 1e-7).  The M2L sums
carry that like the FP32 rounding of the exact tables, so the bounds are
those of the exact path: locals 1e-4 and the potential 1e-4 against the
FP64 oracle, 1e-3 against the dense definition.
"""
import numpy as np
import pytest

from gpu_common import cuda_or_skip, max_rel, rel_l2, say

from paper_2006_15367_amd import workloads as W

pytestmark = pytest.mark.gpu

K = W.K_WAVENUMBER
TOL = 1e-4



def _matvec(torch, ops, q):
    qd = torch.from_numpy(np.ascontiguousarray(q).astype(np.complex64)).cuda()
    phi = ops.matvec(qd)
    torch.cuda.synchronize()
    return phi.cpu().numpy()


def test_sampled_sphere4k_levels_vs_oracle(oracle_dense):
    torch = cuda_or_skip()
    from oracle import mlfma as M
    from oracle import sampled_ops as SO
    from paper_2006_15367_amd import mlfma as G
    xyz, q = W.make("sphere4k")
    q = q.astype(np.complex128)
    ot = M.Tree(xyz, W.LEAF_SIZE)
    sops = SO.sampled_operators(M.Operators(ot, K, W.DIGITS))
    ophi, inter = M.matvec(ot, sops, q, keep=True)
    gt = G.Tree(xyz, W.LEAF_SIZE)
    ops = G.Operators(gt, K, W.DIGITS, sampled=True)
    say("sampled: sphere4k M2L forms", ops.variants("m2l"))
    # (form 9, the matrix-core form, runs here at one RHS: 3 of its 4
    # right-hand-side columns idle)
    for v in (3, 4, 5, 9):
        for l in range(3, ot.n_lev + 1):
            ops.set_variant(l, v)
        phi = _matvec(torch, ops, q)
        for l in range(3, ot.n_lev + 1):
            Lg = ops.copy_spectra(l, 1).cpu().numpy()
            torch.cuda.synchronize()
            rl, ml = rel_l2(Lg, inter["L"][l]), max_rel(Lg, inter["L"][l])
            say("sampled form %d level %d: L rel %.2e max %.2e" % (v, l, rl, ml))
            assert rl < TOL and ml < TOL
        e, m = rel_l2(phi, ophi), max_rel(phi, ophi)
        say("sampled form %d: potential rel %.2e max %.2e" % (v, e, m))
        assert e < TOL and m < TOL
    ref = oracle_dense.potential(xyz, q, K)
    assert rel_l2(phi, ref) < 1e-3
    # the forms that copy from full tables are refused
    for v in (0, 1, 2, 6, 7, 8):
        with pytest.raises(G.MlfmaError) as ex:
            ops.set_variant(3, v)
        assert ex.value.status == G.EINVAL


def test_sampled_sphere262k_vs_oracle_and_exact_tables():
    """Full depth (orders 8 .. 57): the potential against the FP64 oracle
    MLFMA with exact operators, 1 and 2 right-hand sides, and the operator
    memory against the full tables."""
    torch = cuda_or_skip()
    from oracle import mlfma as M
    from paper_2006_15367_amd import mlfma as G
    xyz, q = W.make("sphere262k")
    q = q.astype(np.complex128)
    say("sampled: FP64 oracle MLFMA of the 262k sphere")
    ot = M.Tree(xyz, W.LEAF_SIZE)
    ophi = M.matvec(ot, M.Operators(ot, K, W.DIGITS), q)
    gt = G.Tree(xyz, W.LEAF_SIZE)
    ops = G.Operators(gt, K, W.DIGITS, max_rhs=2, sampled=True)
    full = G.Operators(gt, K, W.DIGITS, max_rhs=2)
    phi = _matvec(torch, ops, q)
    e, m = rel_l2(phi, ophi), max_rel(phi, ophi)
    say("sampled 262k: potential vs FP64 oracle rel %.2e max %.2e" % (e, m))
    assert e < TOL and m < TOL
    rng = np.random.default_rng(71)
    Q = np.stack([q, rng.standard_normal(q.size) + 1j * rng.standard_normal(q.size)], axis=1)
    P = _matvec(torch, ops, Q)
    assert rel_l2(P[:, 0], phi) < 1e-5
    pf = _matvec(torch, full, q)
    say("sampled 262k: vs exact tables rel %.2e" % rel_l2(phi, pf))
    assert rel_l2(phi, pf) < 2e-5
    ms, mf = ops.memory(), full.memory()
    say("sampled 262k: operator bytes %d (full tables %d)" % (ms["operator_bytes"],
                                                             mf["operator_bytes"]))
    assert ms["operator_bytes"] * 100 < mf["operator_bytes"]
    assert ms["total_bytes"] < mf["total_bytes"]


def test_sampled_spheroid_vs_exact_tables_and_dense(oracle_dense):
    """The elongated cloud (9 levels, orders up to 196, 278 MB of full
    operator tables): sampled against exact tables and the dense sum."""
    torch = cuda_or_skip()
    from paper_2006_15367_amd import mlfma as G
    xyz, q = W.make("spheroid1m")
    gt = G.Tree(xyz, W.LEAF_SIZE)
    ops = G.Operators(gt, K, W.DIGITS, sampled=True)
    phi = _matvec(torch, ops, q)
    ms = ops.memory()
    del ops
    full = G.Operators(gt, K, W.DIGITS)
    pf = _matvec(torch, full, q)
    mf = full.memory()
    e = rel_l2(phi, pf)
    say("sampled spheroid: vs exact tables rel %.2e; operator bytes %d vs %d" % (
        e, ms["operator_bytes"], mf["operator_bytes"]))
    assert e < 2e-5
    assert ms["operator_bytes"] * 100 < mf["operator_bytes"]
    rng = np.random.default_rng(72)
    idx = rng.choice(xyz.shape[0], 256, replace=False)
    ref = oracle_dense.potential(xyz, q.astype(np.complex128), K, tgt=xyz[idx])
    assert rel_l2(phi[idx], ref) < 1e-3


def test_sampled_with_bf16x3_adjoint_and_field():
    """The sampled operators with the other options on the 4k sphere: three
    right-hand sides with BF16x3 interpolation against the exact-table FP32
    handle, the adjoint through the dot-product identity, the field against
    the exact-table field.  The BF16x3 maps leave about 1.5e-5 on the
    spectra (full-depth test), which the leaf evaluation amplifies on the
    potential (its quadrature sum is much smaller than its terms): about
    2e-4 there against the FP64 oracle; bound: the method's 3-digit target,
    1e-3."""
    torch = cuda_or_skip()
    from paper_2006_15367_amd import mlfma as G
    xyz, q = W.make("sphere4k")
    rng = np.random.default_rng(73)
    n = xyz.shape[0]
    Q = (rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))).astype(np.complex64)
    gt = G.Tree(xyz, W.LEAF_SIZE)
    ops = G.Operators(gt, K, W.DIGITS, max_rhs=3, sampled=True, bf16x3=True)
    ref = G.Operators(gt, K, W.DIGITS, max_rhs=3)
    Qd = torch.from_numpy(Q).cuda()
    P, Pr = ops.matvec(Qd), ref.matvec(Qd)
    V = torch.from_numpy(np.ascontiguousarray(Q[:, ::-1])).cuda()
    A = ops.adjoint(V)
    F, Fr = ops.field(Qd[:, 0].contiguous()), ref.field(Qd[:, 0].contiguous())
    torch.cuda.synchronize()
    P, Pr, A = P.cpu().numpy(), Pr.cpu().numpy(), A.cpu().numpy()
    F, Fr = F.cpu().numpy(), Fr.cpu().numpy()
    e = rel_l2(P, Pr)
    say("sampled + bf16x3, 3 RHS: vs exact-table FP32 %.2e" % e)
    assert e < 1e-3
    # (with BF16x3 the data are split to about 16 significand bits per map,
    # so the discrete operator is linear, and its adjoint exact, only to
    # about 2^-16 per map: bound 1e-4 of |v| |A q|)
    Vn = V.cpu().numpy()
    for r in range(3):
        lhs = np.vdot(Vn[:, r], P[:, r])
        rhs = np.vdot(A[:, r], Q[:, r])
        assert abs(lhs - rhs) <= 1e-4 * np.linalg.norm(Vn[:, r]) * np.linalg.norm(P[:, r])
    ef = rel_l2(F, Fr)
    say("sampled + bf16x3: field vs exact-table FP32 %.2e" % ef)
    assert ef < 1e-3
