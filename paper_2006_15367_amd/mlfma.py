"""Python binding of the MLFMA C ABI (``include/mlfma.h``): argument
marshalling only.  Every step of the matvec runs in the HIP kernels of
``libmlfma.so``; PyTorch provides device memory and the current stream.

There is no fallback: if the library is missing or fails to load, every
call raises.
"""
import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmlfma.so")

OK, EINVAL, EDEPTH, ENOMEM, EDEVICE, ERANGE = range(6)
C64, C128 = 0, 1
NEAR, FAR, CONJ = 1, 2, 4
FP32, BF16X3_INTERP, NO_AUTOTUNE, USE_GRAPH, ONE_STREAM, SAMPLED_OPERATORS = 0, 1, 2, 4, 8, 16
PROFILE_SERIAL = 0x80000000
KERNELS = ["gather", "p2p", "c2m", "interp_s1", "interp_s2", "interp_s3", "m2l",
           "anterp_s1", "anterp_s2", "anterp_s3", "l2o", "interp", "anterp"]

_lib = None


class MlfmaError(RuntimeError):
    def __init__(self, status, where):
        lib = _load()
        msg = lib.mlfma_last_error().decode(errors="replace")
        name = lib.mlfma_status_string(status).decode(errors="replace")
        super().__init__("%s failed: %s (%s)" % (where, name, msg))
        self.status = status


class TreeInfo(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("n_levels", ctypes.c_int32),
                ("device", ctypes.c_int32), ("leaf_size", ctypes.c_double),
                ("root_size", ctypes.c_double), ("origin", ctypes.c_double * 3),
                ("n_leaf_boxes", ctypes.c_int64), ("n_near_pairs", ctypes.c_int64),
                ("n_p2p_pairs", ctypes.c_int64)]


class LevelInfo(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("L", ctypes.c_int32),
                ("ntheta", ctypes.c_int32), ("nphi", ctypes.c_int32),
                ("K", ctypes.c_int64), ("nbox", ctypes.c_int64),
                ("n_far", ctypes.c_int64), ("n_types", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


EXPORTS = {
    "mlfma_build_tree": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int,
                          ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "mlfma_update_positions": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "mlfma_precompute_operators": ([ctypes.c_void_p, ctypes.c_double, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_uint32,
                                    ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "mlfma_matvec": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                      ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "mlfma_matvec_adjoint": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                              ctypes.c_int64, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "mlfma_matvec_ex": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                         ctypes.c_int, ctypes.c_uint32, ctypes.c_void_p], ctypes.c_int),
    "mlfma_field": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                     ctypes.c_int, ctypes.c_uint32, ctypes.c_void_p], ctypes.c_int),
    "mlfma_position_gradient": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p],
                                ctypes.c_int),
    "mlfma_solve_gmres": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                           ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "mlfma_solve_gmres_noalloc": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p], ctypes.c_int),
    "mlfma_destroy_ops": ([ctypes.c_void_p], None),
    "mlfma_destroy_tree": ([ctypes.c_void_p], None),
    "mlfma_tree_info_get": ([ctypes.c_void_p, ctypes.POINTER(TreeInfo)], ctypes.c_int),
    "mlfma_tree_permutation": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "mlfma_tree_level": ([ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                          ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "mlfma_tree_far_list": ([ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "mlfma_tree_near_list": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
                             ctypes.c_int),
    "mlfma_ops_info": ([ctypes.c_void_p, ctypes.POINTER(LevelInfo), ctypes.c_int],
                       ctypes.c_int),
    "mlfma_copy_spectra": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                            ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "mlfma_set_device_memory_limit": ([ctypes.c_int64], None),
    "mlfma_profile_begin": ([ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int64], ctypes.c_int),
    "mlfma_profile_end": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "mlfma_ops_variants": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int],
                           ctypes.c_int),
    "mlfma_ops_set_variant": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int],
                              ctypes.c_int),
    "mlfma_ops_memory": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                          ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "mlfma_fft_plan": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                        ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "mlfma_fft_execute": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                           ctypes.c_void_p], ctypes.c_int),
    "mlfma_fft_info": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
                        ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "mlfma_fft_destroy": ([ctypes.c_void_p], None),
    "mlfma_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "mlfma_last_error": ([], ctypes.c_char_p),
}


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libmlfma.so is not built (python -m paper_2006_15367_amd.build)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _check(status, where):
    if status != OK:
        raise MlfmaError(status, where)


def set_device_memory_limit(nbytes):
    _load().mlfma_set_device_memory_limit(int(nbytes))


def _as_xyz(xyz):
    if hasattr(xyz, "detach"):
        xyz = xyz.detach().cpu().numpy()
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    if xyz.ndim != 2 or xyz.shape[1] != 3:
        raise ValueError("xyz must have shape [n, 3]")
    return xyz


class Tree:
    """Octree over the points (host side; see mlfma_build_tree)."""

    def __init__(self, xyz, leaf_size=0.25, max_levels=21, device=0):
        lib = _load()
        xyz = _as_xyz(xyz)
        h = ctypes.c_void_p()
        _check(lib.mlfma_build_tree(xyz.ctypes.data if xyz.size else None, xyz.shape[0],
                                    float(leaf_size), int(max_levels), int(device),
                                    ctypes.byref(h)), "mlfma_build_tree")
        self._h = h
        self.n = xyz.shape[0]
        self.device = int(device)

    @property
    def handle(self):
        return self._h

    def info(self):
        inf = TreeInfo()
        _check(_load().mlfma_tree_info_get(self._h, ctypes.byref(inf)), "mlfma_tree_info_get")
        return {"n_points": inf.n_points, "n_levels": inf.n_levels, "device": inf.device,
                "leaf_size": inf.leaf_size, "root_size": inf.root_size,
                "origin": tuple(inf.origin), "n_leaf_boxes": inf.n_leaf_boxes,
                "n_near_pairs": inf.n_near_pairs, "n_p2p_pairs": inf.n_p2p_pairs}

    def permutation(self):
        p = np.empty(self.n, dtype=np.int64)
        _check(_load().mlfma_tree_permutation(self._h, p.ctypes.data if self.n else None),
               "mlfma_tree_permutation")
        return p

    def level(self, level):
        """Integer box coordinates [nbox, 3] and parent indices [nbox]."""
        lib = _load()
        nb = ctypes.c_int64()
        _check(lib.mlfma_tree_level(self._h, int(level), ctypes.byref(nb), None, None),
               "mlfma_tree_level")
        c = np.empty((nb.value, 3), dtype=np.int32)
        p = np.empty(nb.value, dtype=np.int32)
        _check(lib.mlfma_tree_level(self._h, int(level), ctypes.byref(nb), c.ctypes.data,
                                    p.ctypes.data), "mlfma_tree_level")
        return c, p

    def far_list(self, level):
        lib = _load()
        cnt = ctypes.c_int64()
        _check(lib.mlfma_tree_far_list(self._h, int(level), ctypes.byref(cnt), None, None, None),
               "mlfma_tree_far_list")
        n = cnt.value
        obs = np.empty(n, np.int32)
        src = np.empty(n, np.int32)
        code = np.empty(n, np.int32)
        _check(lib.mlfma_tree_far_list(self._h, int(level), ctypes.byref(cnt), obs.ctypes.data,
                                       src.ctypes.data, code.ctypes.data), "mlfma_tree_far_list")
        return obs, src, code

    def near_list(self):
        inf = self.info()
        start = np.empty(inf["n_leaf_boxes"] + 1, np.int64)
        idx = np.empty(inf["n_near_pairs"], np.int32)
        _check(_load().mlfma_tree_near_list(self._h, start.ctypes.data, idx.ctypes.data),
               "mlfma_tree_near_list")
        return start, idx

    def update_positions(self, xyz):
        xyz = _as_xyz(xyz)
        if xyz.shape[0] != self.n:
            raise ValueError("point count changed")
        _check(_load().mlfma_update_positions(self._h, xyz.ctypes.data if self.n else None),
               "mlfma_update_positions")

    def close(self):
        if getattr(self, "_h", None):
            _load().mlfma_destroy_tree(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dtype_code(t):
    import torch
    if t.dtype == torch.complex64:
        return C64
    if t.dtype == torch.complex128:
        return C128
    raise TypeError("charges must be complex64 or complex128, got %s" % t.dtype)


class Operators:
    """Precomputed operators + device workspace (see
    mlfma_precompute_operators)."""

    def __init__(self, tree, k, digits=3, max_rhs=1, bf16x3=False, autotune=True, graph=False,
                 one_stream=False, sampled=False):
        lib = _load()
        h = ctypes.c_void_p()
        flags = ((BF16X3_INTERP if bf16x3 else FP32) | (0 if autotune else NO_AUTOTUNE)
                 | (USE_GRAPH if graph else 0) | (ONE_STREAM if one_stream else 0)
                 | (SAMPLED_OPERATORS if sampled else 0))
        _check(lib.mlfma_precompute_operators(tree.handle, float(k), int(digits),
                                              int(max_rhs), flags, ctypes.byref(h)),
               "mlfma_precompute_operators")
        self._h = h
        self.tree = tree
        self.n = tree.n
        self.k = float(k)
        self.max_rhs = int(max_rhs)
        self.device = tree.device

    def memory(self):
        """{"operator_bytes": translation operator tables, "total_bytes":
        planned device bytes of the handle} (mlfma_ops_memory)."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(_load().mlfma_ops_memory(self._h, ctypes.byref(a), ctypes.byref(b)),
               "mlfma_ops_memory")
        return {"operator_bytes": a.value, "total_bytes": b.value}

    def levels(self):
        nl = self.tree.info()["n_levels"]
        arr = (LevelInfo * nl)()
        _check(_load().mlfma_ops_info(self._h, arr, nl), "mlfma_ops_info")
        return [{f: getattr(a, f) for f, _ in LevelInfo._fields_ if f != "pad"} for a in arr]

    def _prep(self, q, comps=1):
        import torch
        if not (isinstance(q, torch.Tensor) and q.is_cuda):
            raise TypeError("expected a CUDA (HIP) tensor")
        if q.shape[0] != self.n or q.dim() not in (1, 2):
            raise ValueError("expected shape [n] or [n, nrhs] with n = %d" % self.n)
        q = q.contiguous()
        nrhs = 1 if q.dim() == 1 else q.shape[1]
        shape = tuple(q.shape) + ((comps,) if comps > 1 else ())
        out = torch.empty(shape, dtype=q.dtype, device=q.device)
        return q, out, nrhs

    def matvec_ex(self, q, parts=NEAR | FAR, stream=None):
        q, out, nrhs = self._prep(q)
        _check(_load().mlfma_matvec_ex(self._h, q.data_ptr(), out.data_ptr(), nrhs,
                                       _dtype_code(q), parts, _stream_ptr(stream)),
               "mlfma_matvec_ex")
        return out

    def matvec(self, q, stream=None):
        q, out, nrhs = self._prep(q)
        _check(_load().mlfma_matvec(self._h, q.data_ptr(), out.data_ptr(), nrhs,
                                    _dtype_code(q), _stream_ptr(stream)), "mlfma_matvec")
        return out

    def adjoint(self, v, stream=None):
        v, out, nrhs = self._prep(v)
        _check(_load().mlfma_matvec_adjoint(self._h, v.data_ptr(), out.data_ptr(), nrhs,
                                            _dtype_code(v), _stream_ptr(stream)),
               "mlfma_matvec_adjoint")
        return out

    def solve(self, b, shift, restart=30, max_iters=300, tol=1e-5, x0=None, stream=None,
              noalloc=False):
        """Solve (shift I + A) x = b by restarted GMRES on the device
        (mlfma_solve_gmres; with noalloc=True mlfma_solve_gmres_noalloc,
        whose Krylov basis sits in the library's fixed device scratch); b is
        a complex64 CUDA tensor [n] in caller order.  Returns (x, operator
        applications, relative residual)."""
        import torch
        if not (isinstance(b, torch.Tensor) and b.is_cuda and b.dtype == torch.complex64):
            raise TypeError("expected a complex64 CUDA (HIP) tensor")
        if b.dim() != 1 or b.shape[0] != self.n:
            raise ValueError("expected shape [n] with n = %d" % self.n)
        b = b.contiguous()
        x = torch.zeros_like(b) if x0 is None else x0.to(torch.complex64).contiguous().clone()
        it = ctypes.c_int(0)
        rr = ctypes.c_double(0.0)
        sh = complex(shift)
        name = "mlfma_solve_gmres_noalloc" if noalloc else "mlfma_solve_gmres"
        _check(getattr(_load(), name)(self._h, b.data_ptr(), x.data_ptr(), sh.real, sh.imag,
                                      int(restart), int(max_iters), float(tol),
                                      ctypes.byref(it), ctypes.byref(rr), _stream_ptr(stream)),
               name)
        return x, it.value, rr.value

    def field(self, q, parts=0, stream=None):
        q, out, nrhs = self._prep(q, comps=3)
        _check(_load().mlfma_field(self._h, q.data_ptr(), out.data_ptr(), nrhs,
                                   _dtype_code(q), parts, _stream_ptr(stream)), "mlfma_field")
        return out

    def position_gradient(self, q, g, stream=None):
        """out[i, a] = sum_c Re[conj(g) F_q + q F_conj(g)] (see the C ABI)."""
        import torch
        q, _, nrhs = self._prep(q)
        g = g.contiguous()
        if g.shape != q.shape or g.dtype != q.dtype:
            raise ValueError("g must match q in shape and dtype")
        rdt = torch.float32 if q.dtype == torch.complex64 else torch.float64
        out = torch.empty((self.n, 3), dtype=rdt, device=q.device)
        _check(_load().mlfma_position_gradient(self._h, q.data_ptr(), g.data_ptr(),
                                               out.data_ptr(), nrhs, _dtype_code(q),
                                               _stream_ptr(stream)), "mlfma_position_gradient")
        return out

    def copy_spectra(self, level, which, nrhs=1, stream=None):
        import torch
        lv = self.levels()[level - 1]
        out = torch.empty((lv["nbox"], nrhs, lv["K"]), dtype=torch.complex64,
                          device="cuda:%d" % self.device)
        _check(_load().mlfma_copy_spectra(self._h, int(level), int(which), int(nrhs),
                                          out.data_ptr(), _stream_ptr(stream)),
               "mlfma_copy_spectra")
        return out

    def variants(self, kernel="m2l"):
        """Per-level kernel variant chosen by the autotuner (-1: no kernel).
        kernel="p2p": the concurrent schedule, [where it forks the near field
        (1 at the start, 2 after C2M, 3 / 4 after the first / second M2M, 0 at
        the downward pass), eighths of the CUs the M2L workgroups of levels
        > 3 may hold, 1 if the leaf M2L runs late (during the downward pass),
        1 if the near field forked after an M2M runs in two halves];
        [-1, -1, -1, -1] on one stream.  set_variant(level, v, "p2p") sets
        the share (level 1), the leaf M2L order (level 2), the near-field
        split (level 3) or the fork point (level 0)."""
        nl = self.tree.info()["n_levels"]
        out = np.full(4 if kernel == "p2p" else max(nl, 1), -1, np.int32)
        _check(_load().mlfma_ops_variants(self._h, KERNELS.index(kernel), out.ctypes.data,
                                          out.size), "mlfma_ops_variants")
        return out.tolist() if kernel == "p2p" else out[:nl].tolist()

    def set_variant(self, level, variant, kernel="m2l"):
        _check(_load().mlfma_ops_set_variant(self._h, KERNELS.index(kernel), int(level),
                                             int(variant)), "mlfma_ops_set_variant")

    def profile_begin(self, kernels=None, max_launches=4096, serial=False):
        """Start HIP-event timing of the named kernels (default: all).  With
        serial=True the timed calls run every kernel on the caller's stream,
        so each kernel is timed alone."""
        names = KERNELS if kernels is None else kernels
        mask = PROFILE_SERIAL if serial else 0
        for nme in names:
            mask |= 1 << KERNELS.index(nme)
        _check(_load().mlfma_profile_begin(self._h, mask, int(max_launches)),
               "mlfma_profile_begin")

    def profile_end(self):
        """{kernel: (total ms, launches)} for the timed launches."""
        ms = np.zeros(len(KERNELS), np.float64)
        cnt = np.zeros(len(KERNELS), np.int64)
        _check(_load().mlfma_profile_end(self._h, ms.ctypes.data, cnt.ctypes.data),
               "mlfma_profile_end")
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNELS) if cnt[i]}

    def close(self):
        if getattr(self, "_h", None):
            _load().mlfma_destroy_ops(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FFTResampler:
    """FFT interpolation (or, with anterpolate=True, its weighted adjoint)
    between uniform sphere grids of nphi_in and nphi_out phi samples
    (see mlfma_fft_plan).  Call with a complex64 device tensor
    [n, nphi_in // 2, nphi_in]; returns [n, nphi_out // 2, nphi_out]."""

    def __init__(self, lband, nphi_in, nphi_out, anterpolate=False, device=0):
        h = ctypes.c_void_p()
        _check(_load().mlfma_fft_plan(int(lband), int(nphi_in), int(nphi_out),
                                      1 if anterpolate else 0, int(device), ctypes.byref(h)),
               "mlfma_fft_plan")
        self._h = h
        self.lband, self.nphi_in, self.nphi_out = int(lband), int(nphi_in), int(nphi_out)
        self.anterpolate = bool(anterpolate)

    def info(self):
        ipw = ctypes.c_int()
        lds = ctypes.c_int64()
        _check(_load().mlfma_fft_info(self._h, ctypes.byref(ipw), ctypes.byref(lds)),
               "mlfma_fft_info")
        return {"items_per_workgroup": ipw.value, "lds_bytes": lds.value}

    def __call__(self, x, out=None, stream=None):
        import torch
        pi, po = self.nphi_in, self.nphi_out
        if x.dtype != torch.complex64 or not x.is_cuda or not x.is_contiguous():
            raise TypeError("input must be a contiguous complex64 device tensor")
        if x.dim() != 3 or x.shape[1] != pi // 2 or x.shape[2] != pi:
            raise ValueError("input must have shape [n, %d, %d]" % (pi // 2, pi))
        if out is None:
            out = torch.empty((x.shape[0], po // 2, po), dtype=torch.complex64, device=x.device)
        _check(_load().mlfma_fft_execute(self._h, x.data_ptr(), out.data_ptr(), x.shape[0],
                                         _stream_ptr(stream)), "mlfma_fft_execute")
        return out

    def close(self):
        if getattr(self, "_h", None):
            _load().mlfma_fft_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
