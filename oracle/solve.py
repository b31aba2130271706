"""FP64 reference for the shifted second-kind system (test infrastructure
only: imported by the tests and the bench's CPU leg, never by the library).

The potential sum of the paper's problem statement (Sec. 2, the equation for
Phi(r)) is the operator of the integral equations solved iteratively
(Sec. 1, Sec. 2):  (A q)_i = sum_{j != i} G(r_i - r_j) q_j,
G(r) = exp(ik|r|)/|r|, pairs of bit-identical points skipped.  The solver
path solves (shift I + A) x = b; the reference solution is that system
written out as a dense matrix and solved by LU (numpy.linalg.solve), i.e.
the plain definition of the solution.
"""
import numpy as np


def dense_matrix(xyz, k):
    """A_ij = exp(ik r_ij) / r_ij for r_ij > 0, else 0 (FP64, [n, n])."""
    xyz = np.asarray(xyz, dtype=np.float64)
    d = np.sqrt(((xyz[:, None, :] - xyz[None, :, :]) ** 2).sum(-1))
    A = np.zeros(d.shape, dtype=np.complex128)
    nz = d > 0
    A[nz] = np.exp(1j * k * d[nz]) / d[nz]
    return A


def solve_shifted(xyz, b, k, shift):
    """x with (shift I + A) x = b (dense LU, FP64)."""
    A = dense_matrix(xyz, k)
    A[np.diag_indices_from(A)] += shift
    return np.linalg.solve(A, np.asarray(b, dtype=np.complex128))
