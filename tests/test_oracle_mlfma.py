"""Pins of the oracle's tree and FP64 MLFMA against facts the paper prints,
combinatorial invariants, brute force and the dense definition."""
import math

import numpy as np
import pytest

from oracle import mlfma as M
from paper_2006_15367_amd import workloads as W

K = 2.0 * math.pi


def test_level_count_matches_paper_grid_example():
    # Sec. 5.1: 512 x 512 wavelength planar grid, spacing 1/4, leaf 0.25:
    # a 12-level tree with 10 levels of computation.  The level count
    # depends only on the extent, so the grid's corners suffice.
    e = 511.75
    xyz = np.array([[0, 0, 0], [e, 0, 0], [0, e, 0], [e, e, 0]], float)
    t = M.Tree(xyz, 0.25)
    assert t.n_lev == 12
    assert len(t.far) == 10            # far-field levels 3..12


def test_planar_grid_box_counts_and_list_sizes():
    # Eq. (G(l)) with d = 2: one point per leaf of a 64 x 64 wavelength grid
    # gives N_s / 4^(l-1) boxes at the l-th level counted from the leaf;
    # interior boxes of a surface have 6^2 - 3^2 = 27 far boxes (Sec. 3.2.3).
    g = np.arange(256) * 0.25
    X, Y = np.meshgrid(g, g, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)
    t = M.Tree(xyz, 0.25)
    assert t.n_lev == 9
    for up in range(0, 7):
        lev = t.n_lev - up
        assert t.levels[lev].nbox == xyz.shape[0] // 4 ** up
    obs, src, typ = t.far[t.n_lev]
    counts = np.bincount(obs, minlength=t.levels[t.n_lev].nbox)
    assert counts.max() == 27
    c = t.levels[t.n_lev].coords
    interior = np.all((c[:, :2] >= 2) & (c[:, :2] <= 253), axis=1)
    assert np.all(counts[interior] == 27)


def test_volume_grid_interior_list_size():
    # Sec. 3.2.3 / Sec. 4.2: up to 6^3 - 3^3 = 189 far boxes in a volume
    g = np.arange(16) * 0.25
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    t = M.Tree(xyz, 0.25)
    obs, src, typ = t.far[t.n_lev]
    counts = np.bincount(obs, minlength=t.levels[t.n_lev].nbox)
    c = t.levels[t.n_lev].coords
    interior = np.all((c >= 2) & (c <= 13), axis=1)
    assert counts.max() == 189
    assert np.all(counts[interior] == 189)
    assert len(np.unique(typ)) == 316   # 7^3 - 3^3 offsets in use


def test_every_pair_counted_once():
    # near (leaf level) or far at exactly one level, for every pair of leaves
    rng = np.random.default_rng(21)
    xyz = rng.uniform(-1, 1, (400, 3))
    xyz[:100] *= 0.2
    t = M.Tree(xyz, 0.25)
    nl = t.n_lev
    leaf = t.levels[nl]
    B = leaf.nbox
    cover = np.zeros((B, B), dtype=np.int64)
    for b, nb in enumerate(t.near):
        cover[b, nb] += 1
    # ancestor index of each leaf at each level
    anc = {nl: np.arange(B)}
    for lev in range(nl - 1, 0, -1):
        anc[lev] = t.levels[lev + 1].parent[anc[lev + 1]]
    for lev in range(3, nl + 1):
        obs, src, _ = t.far[lev]
        F = np.zeros((t.levels[lev].nbox,) * 2, dtype=np.int64)
        F[obs, src] = 1
        cover += F[anc[lev][:, None], anc[lev][None, :]]
    assert np.all(cover == 1)


@pytest.fixture(scope="module")
def c1():
    xyz, q = W.make("sphere4k")
    t = M.Tree(xyz, W.LEAF_SIZE)
    ops = M.Operators(t, K, W.DIGITS)
    return xyz, q, t, ops


def test_sphere4k_tree_shape(c1):
    xyz, q, t, ops = c1
    assert t.n_lev == 4 and t.D0 == 2.0
    assert [ops.L[3], ops.L[4]] == [13, 8]
    assert t.levels[4].nbox == 262 and t.levels[3].nbox == 56


def test_sphere4k_vs_dense(c1, oracle_dense):
    xyz, q, t, ops = c1
    phi = M.matvec(t, ops, q)
    ref = oracle_dense.potential(xyz, q, K)
    err = np.linalg.norm(phi - ref) / np.linalg.norm(ref)
    assert err < 1e-3


def test_error_falls_with_digits(c1, oracle_dense):
    xyz, q, t, _ = c1
    ref = oracle_dense.potential(xyz, q, K)
    errs = []
    for d in (2, 3, 4, 6):
        ops = M.Operators(t, K, d)
        phi = M.matvec(t, ops, q)
        errs.append(np.linalg.norm(phi - ref) / np.linalg.norm(ref))
    assert all(errs[i + 1] < errs[i] for i in range(3)), errs
    assert errs[-1] < 2e-5


def test_plain_and_grouped_m2l_agree(c1):
    xyz, q, t, ops = c1
    a = M.matvec(t, ops, q, fast=False)
    b = M.matvec(t, ops, q, fast=True)
    assert np.allclose(a, b, rtol=0, atol=1e-12 * np.abs(a).max())


def test_approximate_operator_is_symmetric(c1):
    # A~ = A~^T (antipodal grid + weighted-adjoint anterpolation), so the
    # conjugate pass is the exact discrete adjoint
    xyz, q, t, ops = c1
    rng = np.random.default_rng(22)
    idx = rng.choice(t.n, 6, replace=False)
    E = np.zeros((t.n, idx.size), dtype=np.complex128)
    E[idx, np.arange(idx.size)] = 1.0
    A = M.matvec(t, ops, E)[idx]
    assert np.allclose(A, A.T, rtol=0, atol=1e-12 * np.abs(A).max())


def test_adjoint_dot_product(c1):
    xyz, q, t, ops = c1
    rng = np.random.default_rng(23)
    y = rng.standard_normal(t.n) + 1j * rng.standard_normal(t.n)
    lhs = np.vdot(y, M.matvec(t, ops, q))
    rhs = np.vdot(M.adjoint(t, ops, y), q)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_linearity_and_multi_rhs(c1):
    xyz, q, t, ops = c1
    rng = np.random.default_rng(24)
    q2 = rng.standard_normal(t.n) + 1j * rng.standard_normal(t.n)
    Q = np.stack([q, q2], axis=1)
    P = M.matvec(t, ops, Q)
    a, b = M.matvec(t, ops, q), M.matvec(t, ops, q2)
    assert np.allclose(P[:, 0], a, atol=1e-12 * np.abs(a).max())
    assert np.allclose(P[:, 1], b, atol=1e-12 * np.abs(b).max())
    c = M.matvec(t, ops, 2.0 * q - 3j * q2)
    assert np.allclose(c, 2.0 * a - 3j * b, atol=1e-11 * np.abs(c).max())


def test_input_order_invariance(c1):
    xyz, q, t, ops = c1
    rng = np.random.default_rng(25)
    p = rng.permutation(t.n)
    t2 = M.Tree(xyz[p], W.LEAF_SIZE)
    ops2 = M.Operators(t2, K, W.DIGITS)
    a = M.matvec(t, ops, q)[p]
    b = M.matvec(t2, ops2, q[p])
    assert np.allclose(a, b, atol=1e-12 * np.abs(a).max())

