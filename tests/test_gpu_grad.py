"""GPU differentiation: charge gradient (adjoint MLFMA) and position
gradient (field evaluations) through torch.autograd, against the dense
definition, finite differences of the FP64 oracle MLFMA with the tree
frozen, and a dense PyTorch autograd twin (convention pin)."""
import math

import numpy as np
import pytest

from gpu_common import cuda_or_skip, rel_l2, say

from paper_2006_15367_amd import workloads as W

pytestmark = pytest.mark.gpu

K = W.K_WAVENUMBER


@pytest.fixture(scope="module")
def case():
    torch = cuda_or_skip()
    from paper_2006_15367_amd import mlfma as G
    xyz, q = W.make("sphere4k", nrhs=2)
    t = W.charges(xyz.shape[0], 2, seed=9, dtype=np.complex128)
    say("grad: building GPU tree/operators (sphere4k, 2 RHS)")
    tree = G.Tree(xyz, W.LEAF_SIZE)
    ops = G.Operators(tree, K, W.DIGITS, max_rhs=2)
    return dict(torch=torch, G=G, xyz=xyz, q=q, t=t, tree=tree, ops=ops)


def _loss_and_grads(c):
    torch = c["torch"]
    from paper_2006_15367_amd.autograd import potential
    q = torch.tensor(c["q"], device="cuda", requires_grad=True)
    x = torch.tensor(c["xyz"], device="cuda", requires_grad=True)
    tt = torch.tensor(c["t"], device="cuda")
    phi = potential(q, x, c["ops"])
    L = (phi - tt).abs().pow(2).sum()
    L.backward()
    torch.cuda.synchronize()
    return (float(L.detach()), phi.detach().cpu().numpy(), q.grad.cpu().numpy(),
            x.grad.cpu().numpy())


def test_grad_q_is_adjoint_of_residual(case):
    from oracle import mlfma as M
    say("grad: charge gradient")
    L, phi, gq, gx = _loss_and_grads(case)
    ot = M.Tree(case["xyz"], W.LEAF_SIZE)
    oops = M.Operators(ot, K, W.DIGITS)
    e = M.matvec(ot, oops, case["q"]) - case["t"]
    ref = 2.0 * M.adjoint(ot, oops, e)
    assert rel_l2(gq, ref) < 1e-4


def test_grad_xyz_vs_dense_fields(case, oracle_dense):
    say("grad: position gradient vs dense")
    L, phi, gq, gx = _loss_and_grads(case)
    xyz, q, t = case["xyz"], case["q"], case["t"]
    e = oracle_dense.potential(xyz, q, K) - t
    Fq = oracle_dense.field(xyz, q, K)                 # [n, R, 3]
    Fe = oracle_dense.field(xyz, np.conj(e), K)
    ref = 2.0 * np.real(np.conj(e)[:, :, None] * Fq + q[:, :, None] * Fe).sum(axis=1)
    err = rel_l2(gx, ref)
    say("position gradient rel L2 vs dense", err)
    assert err < 1e-3


def _inner_points(xyz, leaf, count, margin, rng):
    from oracle import mlfma as M
    t = M.Tree(xyz, leaf)
    frac = (xyz - t.origin) / leaf
    dist = np.minimum(frac - np.floor(frac), np.ceil(frac) - frac) * leaf
    ok = np.nonzero(np.all(dist > margin, axis=1))[0]
    return rng.choice(ok, count, replace=False)


def test_grad_xyz_vs_oracle_finite_differences(case):
    """Central differences of the FP64 oracle MLFMA loss (tree frozen: the
    moved point stays in its leaf box) against the GPU gradient."""
    from oracle import mlfma as M
    say("grad: finite differences of the oracle MLFMA")
    L, phi, gq, gx = _loss_and_grads(case)
    xyz, q, t = case["xyz"], case["q"], case["t"]
    rng = np.random.default_rng(41)
    h = 1e-4
    pts = _inner_points(xyz, W.LEAF_SIZE, 3, 10 * h, rng)
    base = M.Tree(xyz, W.LEAF_SIZE)
    for m in pts:
        for a in range(3):
            vals = []
            for sgn in (1.0, -1.0):
                x2 = xyz.copy()
                x2[m, a] += sgn * h
                t2 = M.Tree(x2, W.LEAF_SIZE)
                assert np.array_equal(t2.leafc, base.leafc)   # frozen topology
                o2 = M.Operators(t2, K, W.DIGITS)
                phi2 = M.matvec(t2, o2, q)
                vals.append(np.sum(np.abs(phi2 - t) ** 2))
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - gx[m, a]) < 2e-3 * np.abs(gx).max(), (m, a, fd, gx[m, a])


def test_update_positions_moves_points(case, oracle_dense):
    torch = case["torch"]
    G = case["G"]
    say("grad: matvec after update_positions")
    xyz = case["xyz"]
    rng = np.random.default_rng(42)
    idx = _inner_points(xyz, W.LEAF_SIZE, 200, 2e-3, rng)
    x2 = xyz.copy()
    x2[idx] += rng.uniform(-1e-3, 1e-3, (idx.size, 3))
    tree = G.Tree(xyz, W.LEAF_SIZE)
    ops = G.Operators(tree, K, W.DIGITS, max_rhs=1)
    q = case["q"][:, 0].copy()
    tree.update_positions(x2)
    phi = ops.matvec(torch.tensor(q, device="cuda"))
    torch.cuda.synchronize()
    ref = oracle_dense.potential(x2, q, K)
    assert rel_l2(phi.cpu().numpy(), ref) < 1e-3


def test_autograd_matches_dense_torch_twin():
    """Convention pin: gradients of the GPU MLFMA equal those PyTorch's own
    autograd gives for the dense operator (complex128, CPU)."""
    torch = cuda_or_skip()
    from paper_2006_15367_amd import mlfma as G
    from paper_2006_15367_amd.autograd import potential
    rng = np.random.default_rng(43)
    n = 700
    xyz = rng.uniform(-1.0, 1.0, (n, 3))
    q = rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2))
    t = rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2))
    say("grad: dense torch twin (n=700)")
    tree = G.Tree(xyz, W.LEAF_SIZE)
    assert tree.info()["n_levels"] >= 4
    ops = G.Operators(tree, K, W.DIGITS, max_rhs=2)
    qg = torch.tensor(q, device="cuda", requires_grad=True)
    xg = torch.tensor(xyz, device="cuda", requires_grad=True)
    L = (potential(qg, xg, ops) - torch.tensor(t, device="cuda")).abs().pow(2).sum()
    L.backward()
    torch.cuda.synchronize()
    # dense twin
    qc = torch.tensor(q, requires_grad=True)
    xc = torch.tensor(xyz, requires_grad=True)
    d = xc[:, None, :] - xc[None, :, :]
    r = torch.sqrt((d * d).sum(-1) + torch.eye(n, dtype=torch.float64))
    A = torch.exp(1j * K * r) / r * (1 - torch.eye(n, dtype=torch.float64))
    Lc = (A @ qc - torch.tensor(t)).abs().pow(2).sum()
    Lc.backward()
    Lv, Lcv = float(L.detach()), float(Lc.detach())
    assert abs(Lv - Lcv) < 1e-3 * Lcv
    assert rel_l2(qg.grad.cpu().numpy(), qc.grad.numpy()) < 1e-3
    assert rel_l2(xg.grad.cpu().numpy(), xc.grad.numpy()) < 1e-3
