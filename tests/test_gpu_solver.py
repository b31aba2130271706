"""GPU restarted GMRES on the MLFMA operator (mlfma_solve_gmres) against the
FP64 dense solution of (shift I + A) x = b (oracle/solve.py): the iterative
use of the potential sum that the paper's introduction names."""
import numpy as np
import pytest

from gpu_common import cuda_or_skip, rel_l2, say

from paper_2006_15367_amd import workloads as W

pytestmark = pytest.mark.gpu

K = W.K_WAVENUMBER
# a complex shift of the order of A's spectral radius for this point density
# (about 3.6e3 on the sphere4k cloud): (shift I + A) has condition number
# about 3.8 there, and GMRES(30) reaches 1e-6 in about 20 steps
SHIFT = 1000j


@pytest.fixture(scope="module")
def case():
    torch = cuda_or_skip()
    from oracle import solve as S
    from paper_2006_15367_amd import mlfma as G
    xyz, q = W.make("sphere4k")
    say("gmres: building GPU tree/operators (sphere4k)")
    tree = G.Tree(xyz, W.LEAF_SIZE)
    ops = G.Operators(tree, K, W.DIGITS)
    b = q.astype(np.complex128)
    x_ref = S.solve_shifted(xyz, b, K, SHIFT)
    return dict(torch=torch, G=G, xyz=xyz, b=b, ops=ops, x_ref=x_ref)


def _solve(c, **kw):
    torch = c["torch"]
    bd = torch.from_numpy(c["b"].astype(np.complex64)).cuda()
    x, it, rr = c["ops"].solve(bd, SHIFT, **kw)
    torch.cuda.synchronize()
    return bd, x, it, rr


def test_gmres_matches_dense_solution(case):
    say("gmres: restart 30, tol 1e-5")
    bd, x, it, rr = _solve(case, restart=30, max_iters=200, tol=1e-5)
    assert rr <= 1e-5 and 0 < it < 200, (it, rr)
    # the returned residual is the operator's own, recomputed here
    r = bd - (SHIFT * x + case["ops"].matvec(x))
    rr2 = float(case["torch"].linalg.vector_norm(r) / case["torch"].linalg.vector_norm(bd))
    assert abs(rr2 - rr) < 1e-6, (rr, rr2)
    # the dense FP64 solution: within cond (about 4) x (MLFMA error + tol)
    err = rel_l2(x.cpu().numpy(), case["x_ref"])
    assert err < 1e-3, err


def test_gmres_short_restarts_agree(case):
    say("gmres: restart 5")
    _, x5, it5, rr5 = _solve(case, restart=5, max_iters=400, tol=1e-5)
    assert rr5 <= 1e-5, (it5, rr5)
    assert rel_l2(x5.cpu().numpy(), case["x_ref"]) < 1e-3


def test_gmres_iteration_budget_and_initial_guess(case):
    torch = case["torch"]
    say("gmres: max_iters 0, then a converged initial guess")
    bd, x0, it0, rr0 = _solve(case, restart=10, max_iters=0, tol=1e-5)
    assert it0 == 0 and abs(rr0 - 1.0) < 1e-6
    assert float(torch.linalg.vector_norm(x0)) == 0.0
    _, x, it, rr = _solve(case, restart=30, max_iters=200, tol=1e-5)
    _, x2, it2, rr2 = _solve(case, restart=30, max_iters=200, tol=1e-5, x0=x)
    assert it2 == 0 and rr2 == pytest.approx(rr, abs=1e-7)
    assert torch.equal(x2, x)


def test_gmres_on_a_graph_handle_equals_eager(case):
    """A handle made with graph=True solves with eager matvecs (its basis
    rows are more operand pairs than the graph cache holds): same steps,
    same solution as the plain handle."""
    torch = case["torch"]
    G = case["G"]
    say("gmres: graph handle")
    tree = G.Tree(case["xyz"], W.LEAF_SIZE)
    gops = G.Operators(tree, K, W.DIGITS, graph=True)
    ops = case["ops"]
    nl = tree.info()["n_levels"]
    for k in ("m2l", "interp", "anterp"):  # the same kernels on both handles
        v = ops.variants(k)
        for l in range(3, nl + 1):
            if v[l - 1] >= 0:
                gops.set_variant(l, v[l - 1], kernel=k)
    for i, v in enumerate(ops.variants("p2p")):  # fork point, share, leaf order
        gops.set_variant(i, v, kernel="p2p")
    st = torch.cuda.Stream()
    bd = torch.from_numpy(case["b"].astype(np.complex64)).cuda()
    with torch.cuda.stream(st):
        xg, itg, rrg = gops.solve(bd, SHIFT, restart=30, max_iters=200, tol=1e-5, stream=st)
    st.synchronize()
    _, x, it, rr = _solve(case, restart=30, max_iters=200, tol=1e-5)
    assert abs(itg - it) <= 1 and rrg <= 1e-5
    assert rel_l2(xg.cpu().numpy(), x.cpu().numpy()) < 1e-5


def test_gmres_zero_right_hand_side(case):
    """b = 0 gives x = 0 with no operator application, whatever x0 was."""
    torch = case["torch"]
    say("gmres: b = 0")
    zb = torch.zeros(case["b"].shape[0], dtype=torch.complex64, device="cuda")
    x0 = torch.ones_like(zb)
    x, it, rr = case["ops"].solve(zb, SHIFT, restart=10, max_iters=50, tol=1e-5, x0=x0)
    torch.cuda.synchronize()
    assert it == 0 and rr == 0.0
    assert float(torch.linalg.vector_norm(x)) == 0.0
