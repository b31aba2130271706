"""The C ABI on the host (no GPU needed): the library loads and exports
every symbol the header declares, the host-built tree is bit-identical to
the oracle's tree, and the error paths return their status codes."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2006_15367_amd import mlfma as G
from paper_2006_15367_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "mlfma.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mlfma_\w+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(G.LIB_PATH)
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(G.EXPORTS), set(names) ^ set(G.EXPORTS)


@pytest.mark.parametrize("name,n", [("sphere4k", None), ("spheroid1m", 30000),
                                    ("cube1m_r16", 20000)])
def test_tree_bit_exact_vs_oracle(name, n):
    from oracle import mlfma as M
    xyz, _ = W.make(name, n=n, nrhs=1)
    t = G.Tree(xyz, W.LEAF_SIZE)
    ot = M.Tree(xyz, W.LEAF_SIZE)
    info = t.info()
    assert info["n_levels"] == ot.n_lev
    assert info["root_size"] == ot.D0
    assert np.array_equal(np.array(info["origin"]), ot.origin)
    assert np.array_equal(t.permutation(), ot.perm)
    for l in range(1, ot.n_lev + 1):
        c, p = t.level(l)
        assert np.array_equal(c, ot.levels[l].coords)
        if l > 1:
            assert np.array_equal(p, ot.levels[l].parent)
    for l in range(3, ot.n_lev + 1):
        obs, src, code = t.far_list(l)
        o2, s2, c2 = ot.far[l]
        assert np.array_equal(obs, o2) and np.array_equal(src, s2) and np.array_equal(code, c2)
    start, idx = t.near_list()
    assert np.array_equal(idx, np.concatenate(ot.near))
    sizes = ot.pt_end - ot.pt_start
    pairs = sum(sizes[b] * sum(sizes[c] for c in nb) for b, nb in enumerate(ot.near))
    assert info["n_p2p_pairs"] == pairs


def _status(fn, *a):
    return fn(*a)


def test_build_tree_errors():
    lib = G._load()
    h = ctypes.c_void_p()
    xyz = np.zeros((4, 3))
    assert lib.mlfma_build_tree(None, 4, 0.25, 21, 0, ctypes.byref(h)) == G.EINVAL
    assert lib.mlfma_build_tree(xyz.ctypes.data, -1, 0.25, 21, 0, ctypes.byref(h)) == G.EINVAL
    assert lib.mlfma_build_tree(xyz.ctypes.data, 4, 0.0, 21, 0, ctypes.byref(h)) == G.EINVAL
    assert lib.mlfma_build_tree(xyz.ctypes.data, 4, float("nan"), 21, 0,
                                ctypes.byref(h)) == G.EINVAL
    assert lib.mlfma_build_tree(xyz.ctypes.data, 4, 0.25, 0, 0, ctypes.byref(h)) == G.EINVAL
    bad = xyz.copy()
    bad[2, 1] = np.inf
    assert lib.mlfma_build_tree(bad.ctypes.data, 4, 0.25, 21, 0, ctypes.byref(h)) == G.EINVAL
    assert b"non-finite" in lib.mlfma_last_error()
    wide = np.array([[0, 0, 0], [100.0, 0, 0]])
    assert lib.mlfma_build_tree(wide.ctypes.data, 2, 0.25, 5, 0, ctypes.byref(h)) == G.EDEPTH
    assert lib.mlfma_build_tree(xyz.ctypes.data, 4, 0.25, 21, 0, None) == G.EINVAL


def test_empty_tree_and_null_destroy():
    t = G.Tree(np.zeros((0, 3)), 0.25)
    assert t.info()["n_points"] == 0
    lib = G._load()
    lib.mlfma_destroy_tree(None)
    lib.mlfma_destroy_ops(None)


def test_update_positions_keeps_boxes():
    xyz, _ = W.make("sphere4k")
    t = G.Tree(xyz, W.LEAF_SIZE)
    t.update_positions(xyz + 1e-9)          # stays in every box
    with pytest.raises(G.MlfmaError) as e:
        t.update_positions(xyz + 0.3)       # leaves its boxes
    assert e.value.status == G.ERANGE


def test_update_positions_refuses_leaving_the_root_cube():
    # a point of a boundary leaf moved outward stays in the clamped leaf
    # index but leaves the cube and its box: refused, nothing changes
    xyz, _ = W.make("sphere4k")
    t = G.Tree(xyz, W.LEAF_SIZE)
    i = int(np.argmax(xyz[:, 0]))
    for shift in (5.0, 0.3, 0.26):
        moved = xyz.copy()
        moved[i, 0] += shift
        with pytest.raises(G.MlfmaError) as e:
            t.update_positions(moved)
        assert e.value.status == G.ERANGE, shift
    moved = xyz.copy()
    moved[i, 0] -= 1e-6          # inward, same box
    t.update_positions(moved)


def test_precompute_refuses_leaves_beyond_the_phase_range():
    # near pairs up to 2 sqrt(3) leaf apart must stay within 250 turns of
    # the hardware sine: leaves of 80 wavelengths are refused before the
    # device is touched, 60 wavelengths pass that check
    lib = G._load()
    rng = np.random.default_rng(3)
    h = ctypes.c_void_p()
    xyz = rng.uniform(-10, 10, (64, 3))
    t = G.Tree(xyz, 80.0)
    assert lib.mlfma_precompute_operators(t.handle, W.K_WAVENUMBER, 3, 1, 0,
                                          ctypes.byref(h)) == G.EINVAL
    assert "phase range" in lib.mlfma_last_error().decode()


def test_precompute_argument_errors_and_memory_cap():
    lib = G._load()
    xyz, _ = W.make("sphere4k")
    t = G.Tree(xyz, W.LEAF_SIZE)
    h = ctypes.c_void_p()
    k = W.K_WAVENUMBER
    assert lib.mlfma_precompute_operators(t.handle, -1.0, 3, 1, 0, ctypes.byref(h)) == G.EINVAL
    assert lib.mlfma_precompute_operators(t.handle, k, 0, 1, 0, ctypes.byref(h)) == G.EINVAL
    assert lib.mlfma_precompute_operators(t.handle, k, 3, 0, 0, ctypes.byref(h)) == G.EINVAL
    assert lib.mlfma_precompute_operators(t.handle, k, 3, 1, 32, ctypes.byref(h)) == G.EINVAL
    # leaves too small for the diagonal form: k sqrt(3) a < 1
    small = G.Tree(xyz, 0.05)
    assert lib.mlfma_precompute_operators(small.handle, k, 3, 1, 0, ctypes.byref(h)) == G.EINVAL
    # the device-memory cap is checked before any device call
    G.set_device_memory_limit(1 << 20)
    try:
        assert lib.mlfma_precompute_operators(t.handle, k, 3, 64, 0,
                                              ctypes.byref(h)) == G.ENOMEM
        assert b"limit" in lib.mlfma_last_error()
    finally:
        G.set_device_memory_limit(0)


def test_no_device_reports_edevice():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    xyz, _ = W.make("sphere4k")
    t = G.Tree(xyz, W.LEAF_SIZE)
    with pytest.raises(G.MlfmaError) as e:
        G.Operators(t, W.K_WAVENUMBER, 3)
    assert e.value.status == G.EDEVICE


def test_status_strings():
    lib = G._load()
    for s in range(6):
        assert lib.mlfma_status_string(s).startswith(b"MLFMA_")


def test_solve_gmres_argument_errors():
    """mlfma_solve_gmres rejects bad arguments before it touches a device,
    with the outputs cleared."""
    lib = G._load()
    it = ctypes.c_int(7)
    rr = ctypes.c_double(3.0)
    bad = [
        (1j, 0, 10, 1e-5),           # restart < 1
        (1j, 501, 10, 1e-5),         # restart > 500
        (1j, 30, -1, 1e-5),          # max_iters < 0
        (1j, 30, 10, 0.0),           # tol <= 0
        (1j, 30, 10, float("nan")),  # tol not finite
        (complex(float("inf"), 0), 30, 10, 1e-5),  # shift not finite
        (1j, 30, 10, 1e-5),          # null handle
    ]
    for fn in (lib.mlfma_solve_gmres, lib.mlfma_solve_gmres_noalloc):
        for sh, restart, maxit, tol in bad:
            it.value, rr.value = 7, 3.0
            st = fn(None, None, None, sh.real, sh.imag, restart, maxit, tol,
                    ctypes.byref(it), ctypes.byref(rr), None)
            assert st == G.EINVAL, (fn, sh, restart, maxit, tol)
            assert it.value == 0 and rr.value == 0.0


def test_fft_plan_argument_errors():
    """mlfma_fft_plan validates the sizes before it touches a device; the
    execute/info calls reject a null plan."""
    lib = G._load()
    h = ctypes.c_void_p(123)
    bad = [
        (-1, 18, 28),    # negative band
        (8, 17, 28),     # odd phi count
        (8, 16, 28),     # below 2 lband + 2
        (8, 18, 26),     # output below 2 lband + 2
        (8, 18, 34),     # prime factor 17
        (8, 22, 28),     # prime factor 11
        (8, 18, 1026),   # above 1024
        (60, 122, 126),  # 7-smooth? 122 = 2 x 61: no
        (100, 210, 210),  # one item's LDS above 160 KiB
    ]
    for lb, pi, po in bad:
        for ant in (0, 1):
            h.value = 123
            assert lib.mlfma_fft_plan(lb, pi, po, ant, 0, ctypes.byref(h)) == G.EINVAL, \
                (lb, pi, po)
            assert not h.value
    assert lib.mlfma_fft_plan(8, 18, 28, 0, 0, None) == G.EINVAL
    assert lib.mlfma_fft_execute(None, None, None, 1, None) == G.EINVAL
    assert lib.mlfma_fft_info(None, None, None) == G.EINVAL
    lib.mlfma_fft_destroy(None)
