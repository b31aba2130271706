"""Pins of the oracle's multi-level chain (M2M up, L2L down over several
levels) on trees of 6 and 7 levels, where a chaining mistake cannot hide:
the 4,096-point sphere has one M2M and one L2L step only.

Every check is against a plain definition, not against the oracle itself:

* a multipole at level l is the plane-wave signature of its box's points
  about the box centre (Sec. 3.2.1 applied at level l); M2M (Sec. 3.2.2)
  must reproduce it, because the interpolation is exact for band-limited
  data and the shift is a phase factor;
* a local at level l, evaluated at a point of its box as in L2O (Sec.
  3.2.5), is the potential of every source whose level-l box is not a
  neighbour of the target's level-l box (the far-field lists of levels
  3..l cover exactly those pairs, Sec. 2); L2L (Sec. 3.2.4) must carry
  that to every level;
* the whole product against the dense sum (Sec. 2, Eq. for Phi(r)), its
  error falling as the number of digits rises, the symmetry of the
  approximate operator probed at pairs separated at every level, and the
  adjoint identity.

Two planted mistakes in a copy of the chain (taken from the oracle's own
stage functions) show that these pins see the kind of error they exist for.
"""
import math

import numpy as np
import pytest

from oracle import mlfma as M
from paper_2006_15367_amd import workloads as W

K = 2.0 * math.pi


@pytest.fixture(scope="module")
def deep(oracle_dense):
    """16,384 points on a sphere of radius 4: 6 levels (orders 33, 20, 13, 8
    on levels 3..6): three M2M and three L2L steps."""
    rng = np.random.default_rng(41)
    xyz = W.sphere_points(rng, 16384, 4.0)
    q = rng.standard_normal(16384) + 1j * rng.standard_normal(16384)
    t = M.Tree(xyz, W.LEAF_SIZE)
    ops = M.Operators(t, K, W.DIGITS)
    phi, inter = M.matvec(t, ops, q, keep=True)
    ref = oracle_dense.potential(xyz, q, K)
    return xyz, q, t, ops, phi, inter, ref


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_deep_tree_shape(deep):
    xyz, q, t, ops, phi, inter, ref = deep
    assert t.n_lev == 6
    assert [ops.L[l] for l in range(3, 7)] == [33, 20, 13, 8]
    for lev in range(3, 7):
        assert t.far[lev][0].size > 0


def test_deep_vs_dense(deep):
    xyz, q, t, ops, phi, inter, ref = deep
    err = _rel(phi, ref)
    assert err < 1e-3, err
    # per point, not only in norm: no point's error above 2% of the rms
    # potential (a localized mistake in a few boxes would show here)
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    assert np.max(np.abs(phi - ref)) < 2e-2 * rms


def _signature(pts, qv, centre, khat):
    """S(khat) = sum_j q_j exp(-ik khat.(r_j - c)), written out directly."""
    d = pts - centre
    return np.exp(-1j * K * (d @ khat.T)).T @ qv


def test_multipole_of_every_level_is_the_box_signature(deep):
    # M2M from the leaf up to level 3 against the signature of the box's
    # own points taken directly on that level's grid
    xyz, q, t, ops, phi, inter, ref = deep
    xs = xyz[t.perm]
    qs = q[t.perm]
    rng = np.random.default_rng(42)
    for lev in range(3, t.n_lev + 1):
        Lv = t.levels[lev]
        sh = t.n_lev - lev
        box_of_pt = np.searchsorted(Lv.keys, M._interleave(t.leafc[t.perm] >> sh))
        S = inter["S"][lev][:, 0, :]
        boxes = rng.choice(Lv.nbox, min(12, Lv.nbox), replace=False)
        for b in boxes:
            sel = box_of_pt == b
            direct = _signature(xs[sel], qs[sel], Lv.centres[b], ops.grid[lev].khat)
            err = np.max(np.abs(S[b] - direct)) / np.max(np.abs(direct))
            assert err < 1e-6, (lev, b, err)


def _far_potential_at_level(xyz_s, q_s, coords_of_pt, i, lev_coords_i, K_):
    """Dense potential at point i of every source whose level box is at
    Chebyshev distance >= 2 from the target's level box."""
    sep = np.max(np.abs(coords_of_pt - lev_coords_i), axis=1) >= 2
    d = np.linalg.norm(xyz_s[sep] - xyz_s[i], axis=1)
    return np.sum(np.exp(1j * K_ * d) / d * q_s[sep])


def test_local_of_every_level_is_the_separated_potential(deep):
    # evaluate the local at level l (after L2L) at points of its box with
    # the L2O formula; compare with the direct sum over the sources that
    # are well separated at level l
    xyz, q, t, ops, phi, inter, ref = deep
    xs = xyz[t.perm]
    qs = q[t.perm]
    rng = np.random.default_rng(43)
    for lev in range(3, t.n_lev + 1):
        Lv = t.levels[lev]
        g = ops.grid[lev]
        sh = t.n_lev - lev
        cpt = t.leafc[t.perm] >> sh
        box_of_pt = np.searchsorted(Lv.keys, M._interleave(cpt))
        Lloc = inter["L"][lev][:, 0, :]
        pts = rng.choice(t.n, 24, replace=False)
        got, want = [], []
        for i in pts:
            b = box_of_pt[i]
            e = np.exp(1j * K * (g.khat @ (xs[i] - Lv.centres[b]))) * g.w
            got.append(1j * K / (4.0 * np.pi) * np.sum(e * Lloc[b]))
            want.append(_far_potential_at_level(xs, qs, cpt, i, cpt[i], K))
        got, want = np.array(got), np.array(want)
        err = _rel(got, want)
        assert err < 1e-3, (lev, err)


def test_deep_error_falls_with_digits(deep):
    xyz, q, t, _, _, _, ref = deep
    errs = []
    for d in (2, 3, 4, 6):
        ops = M.Operators(t, K, d)
        errs.append(_rel(M.matvec(t, ops, q), ref))
    assert all(errs[i + 1] < errs[i] for i in range(3)), errs
    assert errs[1] < 1e-3 and errs[-1] < 2e-5, errs


def _pair_separated_at(t, lev, rng):
    """Indices (caller order) of two points whose leaves first become
    separated at level lev (their level-lev boxes are in each other's far
    list)."""
    obs, src, _ = t.far[lev]
    sh = t.n_lev - lev
    Lv = t.levels[lev]
    box = np.searchsorted(Lv.keys, M._interleave(t.leafc >> sh))
    k = rng.integers(obs.size)
    i = rng.choice(np.nonzero(box == obs[k])[0])
    j = rng.choice(np.nonzero(box == src[k])[0])
    return int(i), int(j)


def test_deep_operator_symmetric_at_every_level(deep):
    # A~_ij = A~_ji for pairs that interact through the far field of each
    # level 3..6 (so through 3, 2, 1 and 0 L2L steps)
    xyz, q, t, ops, _, _, _ = deep
    rng = np.random.default_rng(44)
    idx = []
    for lev in range(3, t.n_lev + 1):
        idx.extend(_pair_separated_at(t, lev, rng))
    idx = np.array(idx)
    E = np.zeros((t.n, idx.size), dtype=np.complex128)
    E[idx, np.arange(idx.size)] = 1.0
    A = M.matvec(t, ops, E)[idx]
    assert np.allclose(A, A.T, rtol=0, atol=1e-12 * np.abs(A).max())
    # and each probed far entry is the Green's function to 3 digits
    for p in range(0, idx.size, 2):
        i, j = idx[p], idx[p + 1]
        r = np.linalg.norm(xyz[i] - xyz[j])
        g = np.exp(1j * K * r) / r
        assert abs(A[p, p + 1] - g) < 1e-3 * abs(g) * 30


def test_deep_adjoint_dot_product(deep):
    xyz, q, t, ops, phi, _, _ = deep
    rng = np.random.default_rng(45)
    y = rng.standard_normal(t.n) + 1j * rng.standard_normal(t.n)
    lhs = np.vdot(y, phi)
    rhs = np.vdot(M.adjoint(t, ops, y), q)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def _chain_with_mistake(t, ops, q, mistake):
    """The oracle's chain, assembled from its stage functions, with one
    planted mistake in how the levels are joined."""
    qs = q.reshape(t.n, 1)[t.perm]
    S = {t.n_lev: M.c2m(t, ops, qs)}
    for lev in range(t.n_lev - 1, 2, -1):
        S[lev] = M.m2m(t, ops, S[lev + 1], lev)
    Lm2l = {lev: M.m2l_fast(t, ops, S[lev], lev) for lev in range(3, t.n_lev + 1)}
    Lloc = {3: Lm2l[3]}
    for lev in range(3, t.n_lev):
        if mistake == "parent_without_l2l":
            parent = Lm2l[lev]              # drops everything above lev
        else:
            parent = Lloc[lev]
        child = Lm2l[lev + 1]
        if mistake == "m2l_not_added" and lev + 1 < t.n_lev:
            child = np.zeros_like(child)    # forgets an intermediate M2L
        Lloc[lev + 1] = M.l2l(t, ops, parent, child, lev)
    far = M.l2o(t, ops, Lloc[t.n_lev])
    phi_s = M.near_field(t, qs, ops.k) + far
    phi = np.empty_like(phi_s)
    phi[t.perm] = phi_s
    return phi[:, 0]


@pytest.mark.parametrize("mistake", ["parent_without_l2l", "m2l_not_added"])
def test_planted_chain_mistakes_are_seen(deep, mistake):
    xyz, q, t, ops, phi, _, ref = deep
    # the copy without a mistake is the oracle
    ok = _chain_with_mistake(t, ops, q, None)
    assert np.allclose(ok, phi, rtol=0, atol=1e-12 * np.abs(phi).max())
    bad = _chain_with_mistake(t, ops, q, mistake)
    assert _rel(bad, ref) > 1e-2
