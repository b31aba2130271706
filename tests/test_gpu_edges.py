"""Degenerate and edge inputs through the C ABI on the GPU.

Empty and one-point sets, a pair of points against the closed form of the
potential (Sec. 2: the Green's function sum over j != i) near and far
apart, coincident points (their pair is skipped, as in the oracle), trees
too shallow for a far field (one and two levels: the near field is then
the whole sum, Sec. 3.2.1), the shallowest tree that has one (three
levels: M2L on level 3 with no M2M or L2L), a ragged random cloud with a
ragged number of right-hand sides, and the right-hand-side count limits."""
import numpy as np
import pytest

from gpu_common import cuda_or_skip, rel_l2, say

from paper_2006_15367_amd import workloads as W

pytestmark = pytest.mark.gpu

K = W.K_WAVENUMBER


@pytest.fixture(scope="module")
def env():
    torch = cuda_or_skip()
    from oracle import dense
    from oracle import mlfma as M
    from paper_2006_15367_amd import mlfma as G
    return dict(torch=torch, dense=dense, M=M, G=G)


def _gpu(env, xyz, q, max_rhs=1, adjoint=False):
    torch, G = env["torch"], env["G"]
    tree = G.Tree(xyz, W.LEAF_SIZE)
    ops = G.Operators(tree, K, W.DIGITS, max_rhs=max_rhs)
    qd = torch.from_numpy(np.ascontiguousarray(q).astype(np.complex64)).cuda()
    out = (ops.adjoint if adjoint else ops.matvec)(qd)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.complex128), tree, ops


def _oracle(env, xyz, q):
    M = env["M"]
    t = M.Tree(xyz, W.LEAF_SIZE)
    return M.matvec(t, M.Operators(t, K, W.DIGITS), q), t.n_lev


def test_empty_point_set(env):
    torch, G = env["torch"], env["G"]
    say("edges: empty point set")
    tree = G.Tree(np.zeros((0, 3)), W.LEAF_SIZE)
    ops = G.Operators(tree, K, W.DIGITS)
    q = torch.zeros(0, dtype=torch.complex64, device="cuda")
    assert ops.matvec(q).shape == (0,)
    assert ops.adjoint(q).shape == (0,)
    torch.cuda.synchronize()


def test_single_point_has_zero_potential(env):
    say("edges: one point")
    xyz = np.array([[0.1, -0.2, 0.3]])
    phi, tree, _ = _gpu(env, xyz, np.array([1.0 + 2.0j]))
    assert tree.info()["n_levels"] == 1
    assert phi.shape == (1,) and phi[0] == 0


@pytest.mark.parametrize("dist", [0.1, 3.0])
def test_point_pair_closed_form(env, dist):
    """phi_0 = q_1 e^{ikr}/r and phi_1 = q_0 e^{ikr}/r: in one leaf (near
    field only) and 3 wavelengths apart (through the far field)."""
    say("edges: point pair at distance", dist)
    xyz = np.array([[0.05, 0.07, 0.02], [0.05 + dist, 0.07, 0.02]])
    q = np.array([1.0 + 0.5j, -0.25 + 1.0j])
    g = np.exp(1j * K * dist) / dist
    exact = np.array([q[1] * g, q[0] * g])
    phi, tree, _ = _gpu(env, xyz, q)
    say("n_levels", tree.info()["n_levels"], "rel err", rel_l2(phi, exact))
    assert tree.info()["n_levels"] == (1 if dist < 0.25 else 5)
    assert rel_l2(phi, exact) < (1e-6 if dist < 0.25 else 1e-4)
    # the adjoint of the symmetric operator: conj(A conj(v))
    psi, _, _ = _gpu(env, xyz, q, adjoint=True)
    assert rel_l2(psi, np.conj(np.array([np.conj(q[1]) * g, np.conj(q[0]) * g]))) < (
        1e-6 if dist < 0.25 else 1e-4)


def test_coincident_points_are_skipped(env):
    """Exact duplicates of 64 points: every pair at distance zero is left
    out of the sum, on both sides."""
    say("edges: coincident points")
    xyz, q = W.make("sphere4k")
    xyz = np.concatenate([xyz, xyz[:64]])
    rng = np.random.default_rng(3)
    q = np.concatenate([q, rng.normal(size=64) + 1j * rng.normal(size=64)])
    phi, _, _ = _gpu(env, xyz, q)
    assert np.all(np.isfinite(phi))
    ref, _ = _oracle(env, xyz, q)
    dense_phi = env["dense"].potential(xyz, q, K)
    say("vs oracle", rel_l2(phi, ref), "vs dense", rel_l2(phi, dense_phi))
    assert rel_l2(phi, ref) < 1e-4
    assert rel_l2(phi, dense_phi) < 1e-3


@pytest.mark.parametrize("side,levels", [(0.2, 1), (0.45, 2)])
def test_shallow_trees_are_the_dense_sum(env, side, levels):
    """No level 3, no far field: the near field is the whole sum."""
    say("edges: shallow tree, side", side)
    rng = np.random.default_rng(11)
    xyz = rng.uniform(0, side, (300, 3))
    q = rng.normal(size=300) + 1j * rng.normal(size=300)
    phi, tree, _ = _gpu(env, xyz, q)
    assert tree.info()["n_levels"] == levels
    assert rel_l2(phi, env["dense"].potential(xyz, q, K)) < 1e-5


def test_three_level_tree(env):
    """The shallowest tree with a far field: M2L on level 3 between leaves,
    no interpolation in either direction."""
    say("edges: three-level tree")
    rng = np.random.default_rng(12)
    xyz = rng.uniform(0, 1.0, (2000, 3))
    q = rng.normal(size=2000) + 1j * rng.normal(size=2000)
    phi, tree, _ = _gpu(env, xyz, q)
    ref, nl = _oracle(env, xyz, q)
    assert tree.info()["n_levels"] == nl == 3
    say("vs oracle", rel_l2(phi, ref))
    assert rel_l2(phi, ref) < 1e-4
    assert rel_l2(phi, env["dense"].potential(xyz, q, K)) < 1e-3


def test_ragged_cloud_and_rhs_count(env):
    """1000 random points (leaves of 1 to a few points, lists of every
    length) with 3 right-hand sides at once against 3 single calls."""
    torch = env["torch"]
    say("edges: ragged cloud, 3 RHS")
    rng = np.random.default_rng(13)
    xyz = rng.uniform(0, 2.3, (1000, 3))
    Q = rng.normal(size=(1000, 3)) + 1j * rng.normal(size=(1000, 3))
    P, tree, ops = _gpu(env, xyz, Q, max_rhs=3)
    assert tree.info()["n_levels"] == 5
    for c in range(3):
        single = ops.matvec(torch.from_numpy(Q[:, c].astype(np.complex64)).cuda())
        torch.cuda.synchronize()
        assert rel_l2(P[:, c], single.cpu().numpy()) < 1e-5
    ref, _ = _oracle(env, xyz, Q[:, 1])
    assert rel_l2(P[:, 1], ref) < 1e-4
    assert rel_l2(P, env["dense"].potential(xyz, Q, K)) < 1e-3


def test_rhs_count_limits(env):
    torch, G = env["torch"], env["G"]
    say("edges: RHS count limits")
    xyz, q = W.make("sphere4k")
    ops = G.Operators(G.Tree(xyz, W.LEAF_SIZE), K, W.DIGITS, max_rhs=2, autotune=False)
    n = xyz.shape[0]
    with pytest.raises(G.MlfmaError) as e:
        ops.matvec(torch.zeros((n, 3), dtype=torch.complex64, device="cuda"))
    assert e.value.status == G.EINVAL
    with pytest.raises(G.MlfmaError) as e:
        ops.matvec(torch.zeros((n, 0), dtype=torch.complex64, device="cuda"))
    assert e.value.status == G.EINVAL
    with pytest.raises(ValueError):
        ops.matvec(torch.zeros(n + 1, dtype=torch.complex64, device="cuda"))
    # the largest count is accepted and equals single calls
    Q = np.stack([q, 1j * q], axis=1).astype(np.complex64)
    P = ops.matvec(torch.from_numpy(Q).cuda())
    p0 = ops.matvec(torch.from_numpy(Q[:, 0].copy()).cuda())
    torch.cuda.synchronize()
    assert rel_l2(P.cpu().numpy()[:, 1], 1j * p0.cpu().numpy()) < 1e-5
