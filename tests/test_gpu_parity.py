"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Stage by stage on the 4,096-point sphere (leaf spectra, multipoles per
level, local expansions per level, near and far parts), then end to end
against the dense definition; adjoint, multi-RHS and dtype checks."""
import math

import numpy as np
import pytest

from gpu_common import cuda_or_skip, max_rel, rel_l2, say

from paper_2006_15367_amd import workloads as W

pytestmark = pytest.mark.gpu

K = W.K_WAVENUMBER


@pytest.fixture(scope="module")
def c1():
    torch = cuda_or_skip()
    from oracle import dense
    from oracle import mlfma as M
    from paper_2006_15367_amd import mlfma as G
    xyz, q = W.make("sphere4k")
    ot = M.Tree(xyz, W.LEAF_SIZE)
    oops = M.Operators(ot, K, W.DIGITS)
    ophi, inter = M.matvec(ot, oops, q, keep=True)
    dense_phi = dense.potential(xyz, q, K)
    say("c1: building GPU tree/operators (sphere4k, N=4096)")
    gt = G.Tree(xyz, W.LEAF_SIZE)
    gops = G.Operators(gt, K, W.DIGITS, max_rhs=4)
    return dict(torch=torch, xyz=xyz, q=q, ot=ot, oops=oops, ophi=ophi, inter=inter,
                dense=dense_phi, gt=gt, gops=gops, G=G)


def _run(c, fn, *args, **kw):
    torch = c["torch"]
    out = fn(*args, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_levels_match_oracle(c1):
    lv = c1["gops"].levels()
    ot, oops = c1["ot"], c1["oops"]
    for l in range(3, ot.n_lev + 1):
        assert lv[l - 1]["L"] == oops.L[l]
        assert lv[l - 1]["nbox"] == ot.levels[l].nbox
        assert lv[l - 1]["K"] == oops.grid[l].K


def test_stage_spectra(c1):
    torch = c1["torch"]
    say("c1: matvec for stage spectra")
    qd = torch.from_numpy(c1["q"].astype(np.complex64)).cuda()
    _run(c1, c1["gops"].matvec, qd)
    ot, inter = c1["ot"], c1["inter"]
    for l in range(3, ot.n_lev + 1):
        S = c1["gops"].copy_spectra(l, 0).cpu().numpy()
        Lg = c1["gops"].copy_spectra(l, 1).cpu().numpy()
        torch.cuda.synchronize()
        e_s = rel_l2(S, inter["S"][l])
        e_l = rel_l2(Lg, inter["L"][l])
        m_s, m_l = max_rel(S, inter["S"][l]), max_rel(Lg, inter["L"][l])
        say("level", l, "multipole rel err", e_s, "max", m_s, "local rel err", e_l, "max", m_l)
        assert e_s < 1e-5 and m_s < 1e-5
        assert e_l < 1e-4 and m_l < 1e-4


def test_near_and_far_parts(c1):
    torch = c1["torch"]
    G = c1["G"]
    qd = torch.from_numpy(c1["q"].astype(np.complex64)).cuda()
    perm = c1["ot"].perm
    say("c1: near part")
    near = _run(c1, c1["gops"].matvec_ex, qd, parts=G.NEAR)
    near_o = np.empty_like(c1["inter"]["near"][:, 0])
    near_o[perm] = c1["inter"]["near"][:, 0]
    assert rel_l2(near, near_o) < 1e-5 and max_rel(near, near_o) < 1e-5
    say("c1: far part")
    far = _run(c1, c1["gops"].matvec_ex, qd, parts=G.FAR)
    far_o = np.empty_like(near_o)
    far_o[perm] = c1["inter"]["far"][:, 0]
    assert rel_l2(far, far_o) < 1e-4 and max_rel(far, far_o) < 1e-4


def test_end_to_end_vs_dense_and_oracle(c1):
    torch = c1["torch"]
    say("c1: end to end, complex128 input")
    qd = torch.from_numpy(c1["q"]).cuda()          # complex128 at the boundary
    phi = _run(c1, c1["gops"].matvec, qd)
    assert phi.dtype == np.complex128
    e_dense = rel_l2(phi, c1["dense"])
    e_orc = rel_l2(phi, c1["ophi"])
    say("rel L2 vs dense", e_dense, "vs FP64 MLFMA", e_orc)
    assert e_dense < 1e-3
    assert e_orc < 1e-4


def test_adjoint(c1):
    torch = c1["torch"]
    rng = np.random.default_rng(31)
    n = c1["xyz"].shape[0]
    x = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
    y = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
    say("c1: adjoint")
    xd, yd = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    Ax = _run(c1, c1["gops"].matvec, xd).astype(np.complex128)
    Ahy = _run(c1, c1["gops"].adjoint, yd).astype(np.complex128)
    lhs = np.vdot(y, Ax)
    rhs = np.vdot(Ahy, x)
    # random vectors: |<y, Ax>| ~ |y||Ax|/sqrt(n), so scale by the norms
    assert abs(lhs - rhs) < 1e-5 * np.linalg.norm(y) * np.linalg.norm(Ax)
    # the adjoint is the conjugate pass: compare with the oracle's adjoint
    from oracle import mlfma as M
    ref = M.adjoint(c1["ot"], c1["oops"], y.astype(np.complex128))
    assert rel_l2(Ahy, ref) < 1e-4


def test_multi_rhs_equals_single(c1):
    torch = c1["torch"]
    rng = np.random.default_rng(32)
    n = c1["xyz"].shape[0]
    Q = (rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))).astype(np.complex64)
    say("c1: 3 right-hand sides")
    P = _run(c1, c1["gops"].matvec, torch.from_numpy(Q).cuda())
    for r in range(3):
        p = _run(c1, c1["gops"].matvec, torch.from_numpy(np.ascontiguousarray(Q[:, r])).cuda())
        assert rel_l2(P[:, r], p) < 1e-6


def test_field_vs_dense(c1):
    torch = c1["torch"]
    from oracle import dense
    say("c1: field")
    qd = torch.from_numpy(c1["q"].astype(np.complex64)).cuda()
    F = _run(c1, c1["gops"].field, qd)
    ref = dense.field(c1["xyz"], c1["q"], K)
    e = rel_l2(F, ref)
    say("field rel L2 vs dense", e)
    assert e < 1e-3


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_every_m2l_variant(c1, variant):
    torch = c1["torch"]
    say("c1: M2L variant", variant)
    qd = torch.from_numpy(c1["q"].astype(np.complex64)).cuda()
    ops = c1["gops"]
    chosen = ops.variants("m2l")
    n = c1["xyz"].shape[0]
    rng = np.random.default_rng(40 + variant)
    Q = np.empty((n, 4), np.complex64)
    Q[:, 0] = c1["q"]
    Q[:, 1:] = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
    try:
        for l in range(3, c1["ot"].n_lev + 1):
            ops.set_variant(l, variant)
        phi = _run(c1, ops.matvec, qd)
        # the locals of every level (M2L plus what L2L brought down)
        for l in range(3, c1["ot"].n_lev + 1):
            Lg = ops.copy_spectra(l, 1).cpu().numpy()
            torch.cuda.synchronize()
            assert rel_l2(Lg, c1["inter"]["L"][l]) < 1e-4, (variant, l)
            assert max_rel(Lg, c1["inter"]["L"][l]) < 1e-4, (variant, l)
        P = _run(c1, ops.matvec, torch.from_numpy(Q).cuda())
    finally:
        for l in range(3, c1["ot"].n_lev + 1):
            ops.set_variant(l, chosen[l - 1])
    assert rel_l2(phi, c1["ophi"]) < 1e-4
    # the same variant with four right-hand sides at once
    assert rel_l2(P[:, 0], phi) < 1e-5


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4])
def test_interpolation_variants(c1, variant):
    """Three-pass (0), one-pass (1 + work split) and fused pair kernel (4)
    M2M / L2L: per-level multipoles and locals against the oracle, then end
    to end."""
    torch = c1["torch"]
    say("c1: interpolation variant", variant)
    qd = torch.from_numpy(c1["q"].astype(np.complex64)).cuda()
    ops = c1["gops"]
    nl = c1["ot"].n_lev
    chosen = {k: ops.variants(k) for k in ("interp", "anterp")}
    try:
        for k in ("interp", "anterp"):
            for l in range(3, nl):
                ops.set_variant(l, variant, kernel=k)
        assert ops.variants("interp")[2:nl - 1] == [variant] * (nl - 3)
        phi = _run(c1, ops.matvec, qd)
        for l in range(3, nl + 1):
            S = ops.copy_spectra(l, 0).cpu().numpy()
            Lg = ops.copy_spectra(l, 1).cpu().numpy()
            torch.cuda.synchronize()
            e_s, e_l = rel_l2(S, c1["inter"]["S"][l]), rel_l2(Lg, c1["inter"]["L"][l])
            say("variant", variant, "level", l, "S err", e_s, "L err", e_l)
            assert e_s < 1e-5 and max_rel(S, c1["inter"]["S"][l]) < 1e-5
            assert e_l < 1e-4 and max_rel(Lg, c1["inter"]["L"][l]) < 1e-4
    finally:
        for k in ("interp", "anterp"):
            for l in range(3, nl):
                ops.set_variant(l, chosen[k][l - 1], kernel=k)
    assert rel_l2(phi, c1["ophi"]) < 1e-4


def test_bf16x3_interpolation_accuracy(c1):
    """BF16 split-precision interpolation: same accuracy class as FP32."""
    torch = c1["torch"]
    G = c1["G"]
    say("c1: bf16x3 operators")
    ops = G.Operators(c1["gt"], K, W.DIGITS, max_rhs=1, bf16x3=True)
    qd = torch.from_numpy(c1["q"].astype(np.complex64)).cuda()
    phi = _run(c1, ops.matvec, qd)
    e_orc = rel_l2(phi, c1["ophi"])
    e_dense = rel_l2(phi, c1["dense"])
    fp32 = _run(c1, c1["gops"].matvec, qd)
    say("bf16x3 rel L2 vs FP64 MLFMA", e_orc, "vs dense", e_dense, "vs FP32 path",
        rel_l2(phi, fp32))
    # the split products keep about 2^-17 of each operand; the far-field
    # sums magnify that to about 2e-4 of the potential here, inside the
    # 1e-3 accuracy target with room for rounding-order changes
    assert e_dense < 1e-3
    assert e_orc < 3e-4
    assert rel_l2(phi, fp32) < 3e-4


def test_m2l_matrix_core_form_ragged_rhs(c1):
    """M2L form 9 (matrix cores, right-hand sides in blocks of 16 per wave)
    forced on every level with 20 right-hand sides (a full block and a
    block of 4 of 16) against form 5 (the VALU record kernel) element by
    element, and the first column's locals against the FP64 oracle.  The
    two forms sum the same products in another order: FP32 rounding of the
    far-field sums, bound 1e-5 of the largest value per level."""
    torch = c1["torch"]
    from paper_2006_15367_amd import mlfma as G
    R = 20
    ops = G.Operators(c1["gt"], K, W.DIGITS, max_rhs=R)
    n = c1["xyz"].shape[0]
    rng = np.random.default_rng(91)
    Q = (rng.standard_normal((n, R)) + 1j * rng.standard_normal((n, R))).astype(np.complex64)
    Q[:, 0] = c1["q"]
    Qd = torch.from_numpy(Q).cuda()
    nl = c1["ot"].n_lev
    out = {}
    for v in (5, 9):
        for l in range(3, nl + 1):
            ops.set_variant(l, v)
        say("m2l form", v, "with", R, "rhs")
        P = _run(c1, ops.matvec, Qd)
        Ls = {l: ops.copy_spectra(l, 1, nrhs=R).cpu().numpy() for l in range(3, nl + 1)}
        torch.cuda.synchronize()
        out[v] = (P, Ls)
    for l in range(3, nl + 1):
        a, b = out[9][1][l], out[5][1][l]
        e = float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
        say("level", l, "form 9 vs 5: max rel", e)
        assert e < 1e-5, l
        L0 = a.reshape(a.shape[0], R, -1)[:, 0, :]
        assert rel_l2(L0, c1["inter"]["L"][l].reshape(L0.shape)) < 1e-4, l
    e = float(np.max(np.abs(out[9][0] - out[5][0])) / np.max(np.abs(out[5][0])))
    say("potential form 9 vs 5: max rel", e)
    assert e < 1e-5
    assert rel_l2(out[9][0][:, 0], c1["ophi"]) < 1e-4


def test_m2l_matrix_core_form_64_rhs():
    """M2L form 9 at 64 right-hand sides (four blocks of 16 per sample
    slice) on the 32,768-point sphere (6 levels), forced on every level,
    against form 5 element by element: the same products summed in another
    order, FP32 rounding, bound 1e-5 of the largest value per level."""
    torch = cuda_or_skip()
    from paper_2006_15367_amd import mlfma as G
    xyz, Q = W.make("sphere262k_r64", n=32768)
    tree = G.Tree(xyz, W.LEAF_SIZE)
    nl = tree.info()["n_levels"]
    ops = G.Operators(tree, K, W.DIGITS, max_rhs=64)
    Qd = torch.from_numpy(Q).cuda()
    out = {}
    for v in (5, 9):
        for l in range(3, nl + 1):
            ops.set_variant(l, v)
        say("m2l form", v, "at 64 rhs,", nl, "levels")
        P = ops.matvec(Qd)
        Ls = {l: ops.copy_spectra(l, 1, nrhs=64).cpu().numpy() for l in range(3, nl + 1)}
        torch.cuda.synchronize()
        out[v] = (P.cpu().numpy(), Ls)
    for l in range(3, nl + 1):
        a, b = out[9][1][l], out[5][1][l]
        e = float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
        say("level", l, "form 9 vs 5: max rel", e)
        assert e < 1e-5, l
    e = float(np.max(np.abs(out[9][0] - out[5][0])) / np.max(np.abs(out[5][0])))
    assert e < 1e-5


def test_batched_64_rhs_equals_single():
    """64 right-hand sides in one call equal 64 single-RHS calls.

    The batched call runs C2M and L2O as per-leaf MFMA products (R >= 8),
    the single-RHS calls as per-point loops: the same FP32 arithmetic summed
    in another order.  Rounding (2^-24 per operation) grows with the
    cancellation in the far-field sums, so the bound is 1e-5, two orders
    below the method's 1e-3; the dense check pins the batched values."""
    torch = cuda_or_skip()
    from paper_2006_15367_amd import mlfma as G
    xyz, Q = W.make("sphere262k_r64", n=32768)
    say("batched: 32768-point sphere, 64 RHS")
    tree = G.Tree(xyz, W.LEAF_SIZE)
    ops = G.Operators(tree, K, W.DIGITS, max_rhs=64)
    P = ops.matvec(torch.from_numpy(Q).cuda())
    A = ops.adjoint(torch.from_numpy(Q).cuda())
    torch.cuda.synchronize()
    P = P.cpu().numpy()
    A = A.cpu().numpy()
    for r in (0, 17, 63):
        p = ops.matvec(torch.from_numpy(np.ascontiguousarray(Q[:, r])).cuda())
        a = ops.adjoint(torch.from_numpy(np.ascontiguousarray(Q[:, r])).cuda())
        torch.cuda.synchronize()
        e_p = rel_l2(P[:, r], p.cpu().numpy())
        e_a = rel_l2(A[:, r], a.cpu().numpy())
        say("rhs", r, "batched vs single: matvec", e_p, "adjoint", e_a)
        assert e_p < 1e-5
        assert e_a < 1e-5
    # the batched values against the dense definition on sampled targets
    from oracle import dense
    rng = np.random.default_rng(5)
    idx = rng.choice(xyz.shape[0], 256, replace=False)
    ref = dense.potential(xyz, np.ascontiguousarray(Q[:, :4]).astype(np.complex128), K, tgt=xyz[idx])
    e_d = rel_l2(P[idx, :4], ref)
    say("batched vs dense (256 targets, 4 rhs)", e_d)
    assert e_d < 1e-3


def test_concurrent_schedule_equals_one_stream(c1):
    """The default schedule (near field and per-level M2L on library streams,
    joined by events) gives the same numbers as every kernel on one stream:
    the same kernels, each deterministic, with every dependency kept."""
    torch = c1["torch"]
    G = c1["G"]
    say("c1: concurrent schedule vs one stream")
    ops1 = G.Operators(c1["gt"], K, W.DIGITS, max_rhs=4, one_stream=True)
    ops = c1["gops"]
    # same variants on both handles
    for k in ("m2l", "interp", "anterp"):
        v = ops.variants(k)
        for l in range(3, c1["ot"].n_lev + 1):
            if v[l - 1] >= 0:
                ops1.set_variant(l, v[l - 1], kernel=k)
    rng = np.random.default_rng(77)
    n = c1["xyz"].shape[0]
    Q = (rng.standard_normal((n, 4)) + 1j * rng.standard_normal((n, 4))).astype(np.complex64)
    Qd = torch.from_numpy(Q).cuda()
    tuned, share, late, split = ops.variants("p2p")
    # (four levels: one M2M, so fork point 4 does not exist)
    assert tuned in (0, 1, 2, 3) and share in (4, 6, 7, 8) and late in (0, 1)
    assert split in (0, 1) and ops1.variants("p2p") == [-1, -1, -1, -1]
    try:
        # near field forked at the downward pass / start / after C2M /
        # after the M2M; M2L of levels > 3 on half, three quarters or all
        # of the CUs; the leaf M2L beside the upward pass or after the
        # coarser levels' M2L
        # (and the near field forked after the M2M in two halves)
        for fork, sh, lt, sp in ((0, 6, 0, 0), (1, 6, 0, 0), (2, 6, 0, 0), (1, 4, 0, 0),
                                 (2, 8, 0, 0), (3, 6, 0, 0), (3, 8, 0, 1), (1, 6, 1, 0),
                                 (0, 8, 1, 0), (3, 7, 1, 0), (3, 4, 1, 1)):
            ops.set_variant(0, fork, kernel="p2p")
            ops.set_variant(1, sh, kernel="p2p")
            ops.set_variant(2, lt, kernel="p2p")
            ops.set_variant(3, sp, kernel="p2p")
            for rep in range(3):
                a = _run(c1, ops.matvec, Qd)
                b = _run(c1, ops1.matvec, Qd)
                assert np.array_equal(a, b), (fork, sh, lt, sp, rep)
            fa = _run(c1, ops.field, Qd[:, 0].contiguous())
            fb = _run(c1, ops1.field, Qd[:, 0].contiguous())
            assert np.array_equal(fa, fb), (fork, sh, lt, sp)
    finally:
        ops.set_variant(0, tuned, kernel="p2p")
        ops.set_variant(1, share, kernel="p2p")
        ops.set_variant(2, late, kernel="p2p")
        ops.set_variant(3, split, kernel="p2p")


def test_graph_replays_match_eager(c1):
    """Captured graph of the whole matvec, replayed several times with eager
    work and synchronisations in between; every replay equals the eager
    result bit for bit (same kernels, same order)."""
    torch = c1["torch"]
    G = c1["G"]
    say("c1: graph capture and replays")
    ops_g = G.Operators(c1["gt"], K, W.DIGITS, max_rhs=1, graph=True)
    qd = torch.from_numpy(c1["q"].astype(np.complex64)).cuda()
    eager = _run(c1, c1["gops"].matvec, qd)
    st = torch.cuda.Stream()
    out = torch.empty_like(qd)
    rng = np.random.default_rng(61)
    # both orders of the leaf M2L (beside the upward pass, or after the
    # coarser levels during the downward pass: on this four-level tree the
    # M2L stream then joins the capture through the leaf's own wait)
    for lt in (0, 1, ops_g.variants("p2p")[2]):
        ops_g.set_variant(2, lt, kernel="p2p")
        for rep in range(4):
            with torch.cuda.stream(st):
                phi = ops_g.matvec(qd, stream=st)
            st.synchronize()
            got = phi.cpu().numpy()
            assert rel_l2(got, eager) < 1e-6, (lt, rep)
            # unrelated eager work between replays
            x = torch.from_numpy(rng.standard_normal(4096).astype(np.complex64)).cuda()
            c1["gops"].matvec(x)
            torch.cuda.synchronize()
    # adjoint through the graph path too
    with torch.cuda.stream(st):
        psi = ops_g.adjoint(qd, stream=st)
    st.synchronize()
    assert rel_l2(psi.cpu().numpy(), _run(c1, c1["gops"].adjoint, qd)) < 1e-6


def test_variant_and_schedule_limits(c1):
    """mlfma_ops_set_variant rejects unknown kernel forms and schedule
    settings with MLFMA_EINVAL and leaves the handle as it was."""
    G = c1["G"]
    ops = c1["gops"]
    say("c1: variant and schedule limits")
    nl = c1["ot"].n_lev
    before = (ops.variants("m2l"), ops.variants("p2p"))
    bad = [
        (3, 10, "m2l"), (3, -1, "m2l"), (2, 0, "m2l"), (nl + 1, 0, "m2l"),
        (0, 4, "p2p"), (0, 5, "p2p"), (0, -1, "p2p"), (1, 0, "p2p"), (1, 9, "p2p"),
        (2, 2, "p2p"), (2, -1, "p2p"), (3, 2, "p2p"), (3, -1, "p2p"),
        (nl, 0, "interp"),
    ]
    for level, variant, kernel in bad:
        with pytest.raises(G.MlfmaError) as e:
            ops.set_variant(level, variant, kernel=kernel)
        assert e.value.status == G.EINVAL, (level, variant, kernel)
    assert (ops.variants("m2l"), ops.variants("p2p")) == before
    ops1 = G.Operators(c1["gt"], K, W.DIGITS, max_rhs=1, one_stream=True, autotune=False)
    with pytest.raises(G.MlfmaError):
        ops1.set_variant(0, 1, kernel="p2p")  # one stream: no schedule to set
