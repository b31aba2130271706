"""Pins of the oracle's sampled and interpolated translation operators
(Sec. 3.2.3, paragraph "Translation Operators").

* Against the defining series at 4,001 angles in [0, pi] (both ends
  included) for every order and offset length the benchmark trees use
  (orders 8 .. 57 of the 262k sphere, 104 and 196 of the elongated cloud;
  offsets of 2 to 3 sqrt(3) boxes): the error stays under the rigorous
  Lagrange-remainder bound with Bernstein's inequality, and that bound is
  below 3e-8 of the operator's largest value at s = 8, p = 10.
* The bound is not vacuous: at s = 3 the measured error exceeds the
  s = 8 bound by orders of magnitude, and it still respects its own bound.
* A planted mistake (clamping the stencil at gamma = 0 and pi instead of
  mirroring) breaks the bound near the ends.
* The MLFMA with sampled operators: each level's M2L result moves by at
  most the bound factor times sum over the far pairs of max|T| |S|,
  elementwise; the product within 3e-6 of the MLFMA with exact operators
  (4k sphere and the 16k-point 6-level tree) and within 1e-3 of the dense
  sum.
"""
import math

import numpy as np
import pytest

from oracle import mlfma as M
from oracle import sampled_ops as SO
from paper_2006_15367_amd import workloads as W

K = 2.0 * math.pi
GAMMA = np.linspace(0.0, math.pi, 4001)


@pytest.mark.parametrize("L,a", [(8, 0.25), (13, 0.5), (20, 1.0), (33, 2.0), (57, 4.0),
                                 (104, 8.0), (196, 16.0)])
def test_interpolation_within_bernstein_lagrange_bound(L, a):
    for rr in (2.0, math.sqrt(5.0), 3.0, math.sqrt(12.0), 3.0 * math.sqrt(3.0)):
        r = rr * a
        tab, Mi = SO.table(K, L, r)
        got = SO.interpolate(tab, Mi, GAMMA)
        ref = SO.series(K, L, r, np.cos(GAMMA))
        tmax = np.abs(ref).max()
        bound = SO.error_bound(L, Mi, SO.P_POINTS, tmax)
        err = np.abs(got - ref).max()
        assert err <= bound, (L, rr, err, bound)
        assert bound < 3e-8 * tmax
        # the samples themselves are reproduced
        assert np.allclose(SO.interpolate(tab, Mi, np.arange(Mi + 1) * math.pi / Mi), tab,
                           rtol=0, atol=1e-12 * tmax)


def test_bound_is_not_vacuous():
    L, r = 33, 2.0 * 2.0
    ref = SO.series(K, L, r, np.cos(GAMMA))
    tmax = np.abs(ref).max()
    tab3, M3 = SO.table(K, L, r, s=3)
    err3 = np.abs(SO.interpolate(tab3, M3, GAMMA) - ref).max()
    assert err3 <= SO.error_bound(L, M3, SO.P_POINTS, tmax)
    assert err3 > 100 * SO.error_bound(L, SO.S_OVERSAMPLE * L, SO.P_POINTS, tmax)


def test_planted_clamp_mistake_is_seen():
    L, r = 20, 2.0
    tab, Mi = SO.table(K, L, r)
    p = SO.P_POINTS
    x = GAMMA * Mi / math.pi
    m0 = np.floor(x).astype(int) - (p // 2 - 1)
    bad = np.zeros(GAMMA.shape, complex)
    for j in range(p):
        w = np.ones(GAMMA.shape)
        for i in range(p):
            if i != j:
                w = w * (x - (m0 + i)) / (j - i)
        bad += w * tab[np.clip(m0 + j, 0, Mi)]
    ref = SO.series(K, L, r, np.cos(GAMMA))
    bound = SO.error_bound(L, Mi, p, np.abs(ref).max())
    assert np.abs(bad - ref).max() > 1e3 * bound


def _far_weight(t, ops, S, lev):
    """sum over the far pairs of the level of max|T_type| |S_src| per
    (observer, sample): the operator errors (each below the bound factor
    times its operator's largest value) can move a local by at most the
    bound factor times this."""
    obs, src, typ = t.far[lev]
    tmax = {ty: np.abs(T).max() for ty, T in ops.T[lev].items()}
    acc = np.zeros((t.levels[lev].nbox, S.shape[2]))
    for i in range(obs.size):
        acc[obs[i]] += tmax[int(typ[i])] * np.abs(S[src[i], 0])
    return acc


@pytest.mark.parametrize("case", ["sphere4k", "deep16k"])
def test_mlfma_with_sampled_operators(case, oracle_dense):
    rng = np.random.default_rng(70)
    if case == "sphere4k":
        xyz, q = W.make("sphere4k")
        q = q.astype(np.complex128)
    else:
        xyz = W.sphere_points(rng, 16384, 4.0)
        q = rng.standard_normal(16384) + 1j * rng.standard_normal(16384)
    t = M.Tree(xyz, W.LEAF_SIZE)
    ops = M.Operators(t, K, W.DIGITS)
    sops = SO.sampled_operators(ops)
    phi, inter = M.matvec(t, ops, q, keep=True)
    phis, inters = M.matvec(t, sops, q, keep=True)
    # the operators differ by at most the bound of their level
    for lev in range(3, t.n_lev + 1):
        L = ops.L[lev]
        for typ, T in ops.T[lev].items():
            d = np.abs(sops.T[lev][typ] - T).max()
            assert d <= SO.error_bound(L, SO.S_OVERSAMPLE * L, SO.P_POINTS, np.abs(T).max()) \
                * 1.0001 + 1e-13 * np.abs(T).max()
    # the M2L result of each level moves by at most that, elementwise
    for lev in range(3, t.n_lev + 1):
        L = ops.L[lev]
        rel = SO.error_bound(L, SO.S_OVERSAMPLE * L, SO.P_POINTS, 1.0)
        d = np.abs(M.m2l_fast(t, sops, inter["S"][lev], lev) -
                   M.m2l_fast(t, ops, inter["S"][lev], lev))[:, 0, :]
        assert np.all(d <= rel * _far_weight(t, ops, inter["S"][lev], lev) * 1.0001)
    e = np.linalg.norm(phis - phi) / np.linalg.norm(phi)
    assert e < 3e-6, e
    if case == "sphere4k":
        ref = oracle_dense.potential(xyz, q, K)
        assert np.linalg.norm(phis - ref) / np.linalg.norm(ref) < 1e-3
