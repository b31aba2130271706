"""Pins of the FP64 dense oracle (the plain definition of the potential,
paper Sec. 2, Eq. for Phi(r), with G(r) = exp(ikr)/r) against closed forms,
symmetry and scaling laws."""
import math

import numpy as np
import pytest

K = 2.0 * math.pi


def test_single_source_closed_form(oracle_dense):
    src = np.array([[0.1, -0.2, 0.3]])
    q = np.array([0.7 - 1.3j])
    tgt = np.array([[1.0, 0.5, -0.25], [-2.0, 0.0, 4.0]])
    phi = oracle_dense.potential(src, q, K, tgt=tgt)
    r = np.linalg.norm(tgt - src, axis=1)
    expect = q[0] * np.exp(1j * K * r) / r
    assert np.allclose(phi, expect, rtol=1e-15, atol=0)


def test_two_point_system_by_hand(oracle_dense):
    # two charges 0.5 apart on the x axis: each sees only the other one
    xyz = np.array([[0.0, 0.0, 0.0], [0.5, 0.0, 0.0]])
    q = np.array([1.0 + 0j, 1j])
    phi = oracle_dense.potential(xyz, q, K)
    g = np.exp(1j * K * 0.5) / 0.5          # = exp(i pi) * 2 = -2
    assert abs(g - (-2.0)) < 1e-15
    assert np.allclose(phi, [g * 1j, g * 1.0], rtol=1e-14, atol=1e-15)


def test_reciprocity_bitwise(oracle_dense):
    rng = np.random.default_rng(3)
    xyz = rng.uniform(-1, 1, (64, 3))
    n = xyz.shape[0]
    E = np.eye(n, dtype=np.complex128)
    A = oracle_dense.potential(xyz, E, K)    # column j = response to e_j
    assert np.array_equal(A, A.T)           # |r_i - r_j| is symmetric
    assert np.all(np.diag(A) == 0)          # no self term


def test_scaling_law(oracle_dense):
    # r -> s r, k -> k / s  =>  phi -> phi / s
    rng = np.random.default_rng(4)
    xyz = rng.uniform(-1, 1, (200, 3))
    q = rng.standard_normal(200) + 1j * rng.standard_normal(200)
    s = 4.0
    a = oracle_dense.potential(xyz, q, K)
    b = oracle_dense.potential(s * xyz, q, K / s)
    assert np.allclose(b, a / s, rtol=1e-13, atol=0)


def test_coulomb_limit(oracle_dense):
    rng = np.random.default_rng(5)
    xyz = rng.uniform(-1, 1, (100, 3))
    q = rng.standard_normal(100) + 0j
    phi = oracle_dense.potential(xyz, q, 0.0)
    d = np.linalg.norm(xyz[:, None, :] - xyz[None, :, :], axis=-1)
    np.fill_diagonal(d, np.inf)
    assert np.allclose(phi, (1.0 / d) @ q, rtol=1e-13)


def test_field_closed_form_and_fd(oracle_dense):
    src = np.array([[0.0, 0.0, 0.0]])
    q = np.array([1.0 - 0.5j])
    t = np.array([[0.3, -0.4, 0.2]])
    F = oracle_dense.field(src, q, K, tgt=t)[0]
    r = np.linalg.norm(t[0])
    G = np.exp(1j * K * r) / r
    expect = q[0] * G * (1j * K - 1.0 / r) * t[0] / r
    assert np.allclose(F, expect, rtol=1e-14)
    # central differences of the potential
    rng = np.random.default_rng(6)
    xyz = rng.uniform(-1, 1, (50, 3))
    qq = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    tgt = np.array([[1.7, 0.2, -0.3]])
    Fa = oracle_dense.field(xyz, qq, K, tgt=tgt)[0]
    h = 1e-5
    for a in range(3):
        e = np.zeros((1, 3))
        e[0, a] = h
        fd = (oracle_dense.potential(xyz, qq, K, tgt=tgt + e)
              - oracle_dense.potential(xyz, qq, K, tgt=tgt - e)) / (2 * h)
        assert abs(fd[0] - Fa[a]) < 1e-7 * max(1.0, abs(Fa[a]))


def test_coincident_points_skipped(oracle_dense):
    xyz = np.array([[0.0, 0, 0], [0.0, 0, 0], [1.0, 0, 0]])
    q = np.array([1.0, 2.0, 3.0], dtype=np.complex128)
    phi = oracle_dense.potential(xyz, q, K)
    g = np.exp(1j * K) / 1.0
    assert np.allclose(phi, [3 * g, 3 * g, 3 * g])


def test_multi_rhs_matches_columns(oracle_dense):
    rng = np.random.default_rng(7)
    xyz = rng.uniform(-1, 1, (80, 3))
    q = rng.standard_normal((80, 3)) + 1j * rng.standard_normal((80, 3))
    phi = oracle_dense.potential(xyz, q, K)
    for c in range(3):
        assert np.array_equal(phi[:, c], oracle_dense.potential(xyz, q[:, c], K))
