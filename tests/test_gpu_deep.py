"""GPU stage parity at full depth: the 262,144-point sphere of diameter 16
wavelengths (7 levels, orders 8, 13, 20, 33, 57 on levels 7..3; four M2M
and four L2L level pairs), the HIP path through the C ABI against the FP64
oracle's intermediates level by level.

Each level is compared in relative L2 and element by element (largest
deviation over the level's largest value), so that a defect confined to a
few boxes is not diluted by the norm.  Every M2L kernel form and every
interpolation form the library has for a level pair is forced on every
level where it exists.

Bounds (FP32 against FP64): multipoles 1e-5 (C2M and the interpolation
maps are sums of at most a few hundred FP32 terms of one sign scale,
about 2^-24 times the square root of the term count per stage); locals
1e-4 (M2L sums operators up to about 1.6e3 in size whose result is about
1e3 times smaller at the leaf level, so FP32 rounding of the terms shows
at about 1e3 x 2^-24); far and whole potential 1e-4 against the FP64
oracle MLFMA and 1e-3 against the dense definition (the 3-digit target).
"""
import math

import numpy as np
import pytest

from gpu_common import cuda_or_skip, max_rel, rel_l2, say

from paper_2006_15367_amd import workloads as W

pytestmark = pytest.mark.gpu

K = W.K_WAVENUMBER
TOL_S = 1e-5
TOL_L = 1e-4



@pytest.fixture(scope="module")
def c2():
    torch = cuda_or_skip()
    from oracle import mlfma as M
    from paper_2006_15367_amd import mlfma as G
    xyz, q = W.make("sphere262k")
    q = q.astype(np.complex128)
    say("deep: FP64 oracle MLFMA of the 262k sphere (keeps every level)")
    ot = M.Tree(xyz, W.LEAF_SIZE)
    oops = M.Operators(ot, K, W.DIGITS)
    ophi, inter = M.matvec(ot, oops, q, keep=True)
    say("deep: GPU tree and operators (262k sphere, max_rhs 2)")
    gt = G.Tree(xyz, W.LEAF_SIZE)
    gops = G.Operators(gt, K, W.DIGITS, max_rhs=2)
    return dict(torch=torch, G=G, M=M, xyz=xyz, q=q, ot=ot, oops=oops, ophi=ophi,
                inter=inter, gt=gt, gops=gops)


def _matvec(c, qv, ops=None):
    torch = c["torch"]
    ops = c["gops"] if ops is None else ops
    qd = torch.from_numpy(np.ascontiguousarray(qv).astype(np.complex64)).cuda()
    phi = ops.matvec(qd)
    torch.cuda.synchronize()
    return phi.cpu().numpy()


def _levels_check(c, tag, ops=None):
    """Multipoles and locals of every level against the oracle's."""
    torch = c["torch"]
    ops = c["gops"] if ops is None else ops
    ot, inter = c["ot"], c["inter"]
    worst = []
    for l in range(3, ot.n_lev + 1):
        S = ops.copy_spectra(l, 0).cpu().numpy()
        Lg = ops.copy_spectra(l, 1).cpu().numpy()
        torch.cuda.synchronize()
        rs, ms = rel_l2(S, inter["S"][l]), max_rel(S, inter["S"][l])
        rl, ml = rel_l2(Lg, inter["L"][l]), max_rel(Lg, inter["L"][l])
        say(tag, "level", l, "S rel %.2e max %.2e | L rel %.2e max %.2e" % (rs, ms, rl, ml))
        worst.append((l, rs, ms, rl, ml))
    for l, rs, ms, rl, ml in worst:
        assert rs < TOL_S and ms < TOL_S, (tag, l, rs, ms)
        assert rl < TOL_L and ml < TOL_L, (tag, l, rl, ml)


def test_deep_levels_match(c2):
    lv = c2["gops"].levels()
    ot, oops = c2["ot"], c2["oops"]
    assert ot.n_lev == 7
    for l in range(3, 8):
        assert lv[l - 1]["L"] == oops.L[l]
        assert lv[l - 1]["nbox"] == ot.levels[l].nbox
        assert lv[l - 1]["K"] == oops.grid[l].K


def test_deep_stage_spectra_autotuned(c2):
    say("deep: autotuned kernels, stage spectra")
    phi = _matvec(c2, c2["q"])
    _levels_check(c2, "autotuned")
    e = rel_l2(phi, c2["ophi"])
    m = max_rel(phi, c2["ophi"])
    say("deep: potential vs FP64 MLFMA rel %.2e max %.2e" % (e, m))
    assert e < TOL_L and m < TOL_L


def test_deep_every_near_field_fork_point(c2):
    """The concurrent schedule's fork points of the near field (start, after
    C2M, after the first or second M2M, downward pass), with the leaf M2L
    beside the upward pass or during the downward pass, run the same
    kernels with every dependency kept: results identical bit for bit."""
    torch = c2["torch"]
    ops = c2["gops"]
    tuned, share, late, split = ops.variants("p2p")
    rng = np.random.default_rng(91)
    n = c2["xyz"].shape[0]
    Q = (rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2))).astype(np.complex64)
    try:
        ref = None
        for fork, lt, sp in ((1, 0, 0), (2, 0, 0), (3, 0, 0), (4, 0, 0), (0, 0, 0), (1, 1, 0),
                             (4, 1, 0), (0, 1, 0), (3, 0, 1), (4, 1, 1)):
            ops.set_variant(0, fork, kernel="p2p")
            ops.set_variant(2, lt, kernel="p2p")
            ops.set_variant(3, sp, kernel="p2p")
            say("deep: near field forked at point", fork, "leaf M2L late", lt, "halves", sp)
            for rep in range(2):
                got = _matvec(c2, Q, ops)
                if ref is None:
                    ref = got
                assert np.array_equal(got, ref), (fork, lt, sp, rep)
    finally:
        ops.set_variant(0, tuned, kernel="p2p")
        ops.set_variant(1, share, kernel="p2p")
        ops.set_variant(2, late, kernel="p2p")
        ops.set_variant(3, split, kernel="p2p")


def test_deep_near_and_far_parts(c2):
    torch, G = c2["torch"], c2["G"]
    perm = c2["ot"].perm
    qd = torch.from_numpy(c2["q"].astype(np.complex64)).cuda()
    for part, key, tol in ((G.NEAR, "near", 1e-5), (G.FAR, "far", TOL_L)):
        say("deep: part", key)
        got = c2["gops"].matvec_ex(qd, parts=part)
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        ref = np.empty_like(c2["inter"][key][:, 0])
        ref[perm] = c2["inter"][key][:, 0]
        e, m = rel_l2(got, ref), max_rel(got, ref)
        say("deep:", key, "rel %.2e max %.2e" % (e, m))
        assert e < tol and m < tol


def test_deep_vs_dense_sampled(c2, oracle_dense):
    phi = _matvec(c2, c2["q"])
    rng = np.random.default_rng(8)
    idx = rng.choice(phi.size, 2048, replace=False)
    ref = oracle_dense.potential(c2["xyz"], c2["q"], K, tgt=c2["xyz"][idx])
    e = rel_l2(phi[idx], ref)
    say("deep: vs dense on 2048 targets", e)
    assert e < 1e-3


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_deep_every_m2l_form_on_every_level(c2, variant):
    ops = c2["gops"]
    nl = c2["ot"].n_lev
    chosen = ops.variants("m2l")
    say("deep: M2L form", variant, "forced on levels 3..7")
    rng = np.random.default_rng(60 + variant)
    n = c2["xyz"].shape[0]
    Q = np.empty((n, 2), np.complex64)
    Q[:, 0] = c2["q"]
    Q[:, 1] = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    try:
        for l in range(3, nl + 1):
            ops.set_variant(l, variant)
        phi = _matvec(c2, c2["q"])
        _levels_check(c2, "m2l form %d" % variant)
        P = _matvec(c2, Q)
    finally:
        for l in range(3, nl + 1):
            ops.set_variant(l, chosen[l - 1])
    assert rel_l2(phi, c2["ophi"]) < TOL_L
    # two right-hand sides through the same form: the first column is the
    # single-RHS product up to FP32 summation order
    assert rel_l2(P[:, 0], phi) < 1e-5


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4])
def test_deep_every_interpolation_form(c2, variant):
    """Three passes (0), one pass in work split variant - 1 (1..3) or the
    fused pair kernel (4), forced on every level pair and direction that
    has that form (the one-pass kernels exist for the two finest pairs, the
    pair kernel for those and for the M2M of 20 -> 33); the others keep the
    autotuner's choice."""
    G = c2["G"]
    ops = c2["gops"]
    nl = c2["ot"].n_lev
    chosen = {k: ops.variants(k) for k in ("interp", "anterp")}
    forced = []
    try:
        for l in range(3, nl):
            for k in ("interp", "anterp"):
                try:
                    ops.set_variant(l, variant, kernel=k)
                    forced.append((l, k))
                except G.MlfmaError as e:
                    assert e.status == G.EINVAL
        say("deep: interpolation form", variant, "on (level pair, direction)", forced)
        if not forced:
            pytest.skip("no level pair has interpolation form %d" % variant)
        phi = _matvec(c2, c2["q"])
        _levels_check(c2, "interp form %d" % variant)
    finally:
        for k in ("interp", "anterp"):
            for l in range(3, nl):
                ops.set_variant(l, chosen[k][l - 1], kernel=k)
    assert rel_l2(phi, c2["ophi"]) < TOL_L
    if variant == 0:
        assert forced == [(l, k) for l in range(3, nl) for k in ("interp", "anterp")]


@pytest.mark.parametrize("form", ["autotuned", "three_pass", "pair"])
def test_deep_bf16x3_levels(c2, form):
    """BF16 split-precision interpolation at full depth, with the autotuned
    forms, three passes forced everywhere, or the BF16x3 pair kernel forced
    on every level pair and direction that has it.  A split operand hi + lo
    carries 16 significand bits and the dropped lo * lo product is 2^-16 of
    the full one, so each of the three maps of a level pair is good to
    about 2^-16 = 1.5e-5; twelve maps from the leaf to level 3, added
    coherently, give 1.8e-4: bound 2e-4 on the multipoles.  Locals: the
    FP32 M2L bound (1e-4) plus the anterpolation maps down to the level
    (at most twelve, 1.8e-4): 3e-4.  The potential within 1e-3 of the FP64
    oracle (the 3-digit target)."""
    G, torch = c2["G"], c2["torch"]
    say("deep: bf16x3 operators,", form)
    ops = G.Operators(c2["gt"], K, W.DIGITS, max_rhs=1, bf16x3=True)
    nl = c2["ot"].n_lev
    forced = []
    if form != "autotuned":
        for l in range(3, nl):
            for k in ("interp", "anterp"):
                try:
                    ops.set_variant(l, 0 if form == "three_pass" else 4, kernel=k)
                    forced.append((l, k))
                except G.MlfmaError as e:
                    assert e.status == G.EINVAL
        say("deep bf16x3: forced on", forced)
        if form == "pair":
            assert (nl - 1, "interp") in forced and (nl - 1, "anterp") in forced
    say("deep bf16x3: forms", ops.variants("interp"), ops.variants("anterp"))
    phi = _matvec(c2, c2["q"], ops=ops)
    for l in range(3, nl + 1):
        S = ops.copy_spectra(l, 0).cpu().numpy()
        Lg = ops.copy_spectra(l, 1).cpu().numpy()
        torch.cuda.synchronize()
        es, ms = rel_l2(S, c2["inter"]["S"][l]), max_rel(S, c2["inter"]["S"][l])
        el, ml = rel_l2(Lg, c2["inter"]["L"][l]), max_rel(Lg, c2["inter"]["L"][l])
        say("deep bf16x3 %s: level %d S rel %.2e max %.2e | L rel %.2e max %.2e" % (
            form, l, es, ms, el, ml))
        assert es < 2e-4 and ms < 2e-4
        assert el < 3e-4 and ml < 3e-4
    e = rel_l2(phi, c2["ophi"])
    say("deep bf16x3: potential vs FP64 MLFMA", e)
    assert e < 1e-3


def test_spheroid_every_level_and_far_part():
    """The elongated cloud at full size (1,048,576 points, 9 levels, orders
    8 .. 196 on levels 9 .. 3, K up to 77,618 samples, tip leaves of 1,566
    points): multipoles and locals of every level, the far part and the
    potential against the FP64 oracle, same bounds as the sphere."""
    torch = cuda_or_skip()
    from oracle import mlfma as M
    from paper_2006_15367_amd import mlfma as G
    xyz, q = W.make("spheroid1m")
    q = q.astype(np.complex128)
    say("spheroid: FP64 oracle MLFMA (keeps every level)")
    ot = M.Tree(xyz, W.LEAF_SIZE)
    oops = M.Operators(ot, K, W.DIGITS)
    ophi, inter = M.matvec(ot, oops, q, keep=True)
    assert ot.n_lev == 9 and oops.L[3] == 196 and oops.L[4] == 104
    say("spheroid: GPU tree and operators")
    gt = G.Tree(xyz, W.LEAF_SIZE)
    gops = G.Operators(gt, K, W.DIGITS, max_rhs=1)
    c = dict(torch=torch, ot=ot, inter=inter, gops=gops)
    phi = _matvec(c, q)
    _levels_check(c, "spheroid")
    qd = torch.from_numpy(q.astype(np.complex64)).cuda()
    far = gops.matvec_ex(qd, parts=G.FAR)
    torch.cuda.synchronize()
    far = far.cpu().numpy()
    ref = np.empty_like(inter["far"][:, 0])
    ref[ot.perm] = inter["far"][:, 0]
    ef, mf = rel_l2(far, ref), max_rel(far, ref)
    e, m = rel_l2(phi, ophi), max_rel(phi, ophi)
    say("spheroid: far rel %.2e max %.2e; potential rel %.2e max %.2e" % (ef, mf, e, m))
    assert ef < TOL_L and mf < TOL_L
    assert e < TOL_L and m < TOL_L
