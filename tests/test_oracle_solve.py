"""Pins of the FP64 reference solution of (shift I + A) x = b
(oracle/solve.py) against facts that do not come from it: the independent
dense potential oracle (C), the closed form of a 2 x 2 system, the residual
of the system and the symmetry of A (reciprocity)."""
import numpy as np

from oracle import dense
from oracle import solve as S

K = 2 * np.pi


def _cloud(n, seed):
    rng = np.random.default_rng(seed)
    xyz = rng.uniform(-1.0, 1.0, size=(n, 3))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return xyz, b


def test_matrix_equals_dense_potential_oracle():
    xyz, q = _cloud(200, 1)
    a = S.dense_matrix(xyz, K) @ q
    ref = dense.potential(xyz, q, K)
    assert np.linalg.norm(a - ref) / np.linalg.norm(ref) < 1e-12


def test_two_point_closed_form():
    xyz = np.array([[0.0, 0.0, 0.0], [0.3, -0.2, 0.5]])
    r = np.linalg.norm(xyz[1] - xyz[0])
    g = np.exp(1j * K * r) / r
    sigma = 1.5 - 0.7j
    b = np.array([0.4 + 1.1j, -2.0 + 0.3j])
    det = sigma * sigma - g * g
    want = np.array([(sigma * b[0] - g * b[1]) / det, (sigma * b[1] - g * b[0]) / det])
    got = S.solve_shifted(xyz, b, K, sigma)
    assert np.allclose(got, want, rtol=1e-13, atol=0)


def test_residual_and_reciprocity():
    xyz, b = _cloud(300, 2)
    _, c = _cloud(300, 3)
    sigma = 40j
    x = S.solve_shifted(xyz, b, K, sigma)
    y = S.solve_shifted(xyz, c, K, sigma)
    # residual, with the matrix applied by the independent dense oracle
    res = sigma * x + dense.potential(xyz, x, K) - b
    assert np.linalg.norm(res) / np.linalg.norm(b) < 1e-12
    # A = A^T, so c^T x = c^T M^-1 b = (M^-1 c)^T b = y^T b
    assert abs(c @ x - y @ b) < 1e-10 * abs(c @ x)


def test_coincident_points_are_skipped():
    xyz = np.array([[0.1, 0.2, 0.3], [0.1, 0.2, 0.3], [1.0, 0.0, 0.0]])
    A = S.dense_matrix(xyz, K)
    assert A[0, 1] == 0 and A[1, 0] == 0 and np.all(np.diag(A) == 0)
    assert A[0, 2] != 0
