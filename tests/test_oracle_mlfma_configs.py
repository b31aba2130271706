"""The oracle's FP64 MLFMA against the dense definition (Sec. 2, Eq. for
Phi(r)) on the benchmark clouds at full size, on 4,096 seeded random
targets: the 262,144-point sphere (7 levels, orders 8..57), the
1,048,576-point cube (7 levels, about 173 far boxes per leaf) and the
1,048,576-point spheroid with its tip cluster (9 levels, orders 8..196).

Measured on this container: 8.3e-5, 5.8e-5 and 1.0e-4 relative L2 at 3
digits.  The two 1M-point clouds take about four minutes each and run only
with ``--runslow``.
"""
import math

import numpy as np
import pytest

from oracle import mlfma as M
from paper_2006_15367_amd import workloads as W

K = 2.0 * math.pi


def _check(name, oracle_dense, n_lev, orders):
    xyz, q = W.make(name, nrhs=1)
    q = q.astype(np.complex128)
    t = M.Tree(xyz, W.LEAF_SIZE)
    ops = M.Operators(t, K, W.DIGITS)
    assert t.n_lev == n_lev
    assert [ops.L[l] for l in range(3, n_lev + 1)] == orders
    phi = M.matvec(t, ops, q)
    rng = np.random.default_rng(99)
    idx = rng.choice(t.n, 4096, replace=False)
    ref = oracle_dense.potential(xyz, q, K, tgt=xyz[idx])
    err = float(np.linalg.norm(phi[idx] - ref) / np.linalg.norm(ref))
    assert err < 1e-3, err
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    assert np.max(np.abs(phi[idx] - ref)) < 2e-2 * rms


def test_sphere262k_vs_dense_on_4096_targets(oracle_dense):
    _check("sphere262k", oracle_dense, 7, [57, 33, 20, 13, 8])


@pytest.mark.slow
def test_cube1m_vs_dense_on_4096_targets(oracle_dense):
    _check("cube1m_r16", oracle_dense, 7, [57, 33, 20, 13, 8])


@pytest.mark.slow
def test_spheroid1m_vs_dense_on_4096_targets(oracle_dense):
    _check("spheroid1m", oracle_dense, 9, [196, 104, 57, 33, 20, 13, 8])
