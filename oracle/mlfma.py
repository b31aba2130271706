r"""Plain FP64 MLFMA for phi_i = sum_{j != i} q_j exp(ik|r_i - r_j|)/|r_i - r_j|
(oracle; test infrastructure only -- the product path never imports this).

Follows the paper's rubric step by step (Sec. 2, the five-stage list; Sec.
3.2.1-3.2.5 for C2M, M2M, M2L, L2L, L2O): octree with near/far
classification (Sec. 2, FMM paragraph; Sec. 3.1 for the level count and the
Morton-Z order), leaf plane-wave signatures (C2M), interpolate-shift-
aggregate up the tree (M2M, Sec. 3.2.2 and its algorithm), diagonal
translation over far-field lists (M2L, Sec. 3.2.3), shift-anterpolate-
aggregate down the tree (L2L, Sec. 3.2.4), evaluation at the leaf points
(L2O, Sec. 3.2.5), and the direct near-field sum at the leaf level (Sec. 2).

Where the paper is silent (truncation order, sampling, the plane-wave
mathematics it defers to its references) the readings are:
  * kernel exp(+ikr)/r (conjugate of the paper's exp(-jkr)/(4 pi r) times
    4 pi for real k);
  * G(X+d) = (ik/4pi) \int exp(ik khat.d) T_L(khat, X) d khat with
    T_L(khat, X) = sum_{l<=L} i^l (2l+1) h_l^(1)(k|X|) P_l(khat.Xhat)
    (Gegenbauer addition theorem plus the plane-wave expansion);
  * L = ceil(k d + 1.8 digits^(2/3) (k d)^(1/3)), d = sqrt(3) a (box
    diagonal);
  * Gauss-Legendre theta x uniform phi grids and the exact band-limited
    ("global") interpolation written as three maps: a phi-Fourier
    transform, a per-order Legendre map in theta, an inverse phi-Fourier
    transform; anterpolation is the weighted adjoint of interpolation;
  * far-field lists at levels >= 3 (levels 1-2 have none).
"""
import math

import numpy as np

from . import dense, sphere


# --------------------------------------------------------------------------
# Tree (Sec. 2 FMM paragraph; Sec. 3.1)
# --------------------------------------------------------------------------

def _interleave(c):
    """Morton-Z key of integer box coordinates c [n, 3] (x bit above y above z)."""
    key = np.zeros(c.shape[0], dtype=np.int64)
    for b in range(21):
        for axis, shift in ((0, 2), (1, 1), (2, 0)):
            bit = (c[:, axis] >> b) & 1
            key |= bit << (3 * b + shift)
    return key


def offset_type(delta):
    """Index of an offset (dx, dy, dz) with |d| <= 3 per axis: (dx+3)*49+(dy+3)*7+(dz+3)."""
    delta = np.asarray(delta)
    return (delta[..., 0] + 3) * 49 + (delta[..., 1] + 3) * 7 + (delta[..., 2] + 3)


class Level:
    """Boxes of one level: integer coordinates, Morton keys, centres, parents."""


class Tree:
    """Octree over the points (Sec. 2, FMM paragraph; Sec. 3.1).

    * n_lev is the smallest integer with leaf_size * 2^(n_lev-1) >= E, where
      E is the largest side of the points' bounding box (the paper's rule
      L >= log2(D0/D(L)) + 1); the root cube has side
      D0 = leaf_size * 2^(n_lev-1) and is centred on the bounding box.
    * A point's leaf box is floor((r - origin)/leaf_size) per axis, clamped
      into the cube; its box at level l is that index shifted right by
      n_lev - l.  Only non-empty boxes are kept, in Morton-Z order.
    * Near field (leaf level only): boxes sharing a face, edge or vertex,
      i.e. Chebyshev distance <= 1, the box itself included.
    * Far field at level l: boxes that are not near but whose parents are
      near; kept for levels >= 3.
    """

    def __init__(self, xyz, leaf_size):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        self.xyz = xyz
        self.n = xyz.shape[0]
        self.leaf_size = float(leaf_size)
        lo = xyz.min(axis=0)
        hi = xyz.max(axis=0)
        extent = float(np.max(hi - lo))
        n_lev = 1
        while self.leaf_size * 2.0 ** (n_lev - 1) < extent:
            n_lev += 1
        self.n_lev = n_lev
        self.D0 = self.leaf_size * 2.0 ** (n_lev - 1)
        centre = 0.5 * (lo + hi)
        self.origin = centre - 0.5 * self.D0
        nside = 1 << (n_lev - 1)
        leafc = np.floor((xyz - self.origin) / self.leaf_size).astype(np.int64)
        leafc = np.clip(leafc, 0, nside - 1)
        key = _interleave(leafc)
        # Morton-Z order of the points, ties by original index (stable sort)
        self.perm = np.argsort(key, kind="stable")
        self.leafc = leafc
        self.levels = {}
        sorted_key = key[self.perm]
        for lev in range(1, n_lev + 1):
            sh = 3 * (n_lev - lev)
            lk = sorted_key >> sh
            keys, first = np.unique(lk, return_index=True)
            L = Level()
            L.keys = keys
            L.coords = leafc[self.perm[first]] >> (n_lev - lev)
            L.a = self.D0 / 2.0 ** (lev - 1)
            L.centres = self.origin + (L.coords + 0.5) * L.a
            L.nbox = keys.size
            if lev > 1:
                L.parent = np.searchsorted(self.levels[lev - 1].keys, keys >> 3)
            self.levels[lev] = L
        leaf = self.levels[n_lev]
        # points of each leaf box (ranges into the sorted order)
        lk = sorted_key
        self.pt_start = np.searchsorted(lk, leaf.keys, side="left")
        self.pt_end = np.searchsorted(lk, leaf.keys, side="right")
        self.box_of_sorted = np.repeat(np.arange(leaf.nbox),
                                       self.pt_end - self.pt_start)
        self.near = self._near_lists()
        self.far = {lev: self._far_list(lev) for lev in range(3, n_lev + 1)}

    def _lookup(self, lev, coords):
        """Index of the box with these integer coords at lev, or -1."""
        L = self.levels[lev]
        nside = 1 << (lev - 1)
        ok = np.all((coords >= 0) & (coords < nside), axis=1)
        idx = np.full(coords.shape[0], -1, dtype=np.int64)
        if np.any(ok):
            k = _interleave(coords[ok])
            pos = np.searchsorted(L.keys, k)
            pos = np.minimum(pos, L.nbox - 1)
            hit = L.keys[pos] == k
            sub = np.full(k.size, -1, dtype=np.int64)
            sub[hit] = pos[hit]
            idx[ok] = sub
        return idx

    def _near_lists(self):
        lev = self.n_lev
        L = self.levels[lev]
        lists = [[] for _ in range(L.nbox)]
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    nb = self._lookup(lev, L.coords + np.array([dx, dy, dz]))
                    for b in np.nonzero(nb >= 0)[0]:
                        lists[b].append(int(nb[b]))
        return [sorted(x) for x in lists]

    def _far_list(self, lev):
        """Pairs (observer, source, offset type) of the far-field list at lev.

        delta = c_obs - c_src; kept when max|delta| >= 2 and the parents are
        at Chebyshev distance <= 1 (so |delta| <= 3 per axis).
        """
        L = self.levels[lev]
        obs_all, src_all, typ_all = [], [], []
        rng = range(-3, 4)
        for dx in rng:
            for dy in rng:
                for dz in rng:
                    d = np.array([dx, dy, dz])
                    if np.max(np.abs(d)) < 2:
                        continue
                    src = self._lookup(lev, L.coords - d)
                    ok = src >= 0
                    obs = np.nonzero(ok)[0]
                    src = src[ok]
                    pc = np.max(np.abs((L.coords[obs] >> 1)
                                       - (L.coords[src] >> 1)), axis=1)
                    keep = pc <= 1
                    obs_all.append(obs[keep])
                    src_all.append(src[keep])
                    typ_all.append(np.full(int(keep.sum()), offset_type(d)))
        obs = np.concatenate(obs_all) if obs_all else np.zeros(0, np.int64)
        src = np.concatenate(src_all) if src_all else np.zeros(0, np.int64)
        typ = np.concatenate(typ_all) if typ_all else np.zeros(0, np.int64)
        order = np.lexsort((src, obs))
        return obs[order], src[order], typ[order]


# --------------------------------------------------------------------------
# Operators (Sec. 3.2.3 translation operators; Sec. 3.2.2 interpolation)
# --------------------------------------------------------------------------

def truncation_order(k, a, digits):
    """L = ceil(k d + 1.8 digits^(2/3) (k d)^(1/3)), d = sqrt(3) a."""
    kd = k * math.sqrt(3.0) * a
    return int(math.ceil(kd + 1.8 * digits ** (2.0 / 3.0) * kd ** (1.0 / 3.0)))


def translation_operator(k, L, X, grid):
    """T_L(khat, X) = sum_{l=0}^{L} i^l (2l+1) h_l^(1)(k|X|) P_l(khat . Xhat)
    on the samples of ``grid`` (diagonal translation, Sec. 3.2.3)."""
    X = np.asarray(X, dtype=np.float64)
    r = float(np.linalg.norm(X))
    h = sphere.spherical_hankel1(L, k * r)
    u = grid.khat @ (X / r)
    P = sphere.legendre_p(L, u)
    coef = (1j ** np.arange(L + 1)) * (2 * np.arange(L + 1) + 1) * h
    return coef @ P


def legendre_map(Lband, x_from, w_from, x_to):
    """Per-order theta maps M_m[i_to, i_from] = sum_{l=m}^{Lband}
    Pbar_l^m(x_to) Pbar_l^m(x_from) w_from, m = 0..Lband."""
    maps = []
    for m in range(Lband + 1):
        Pt = sphere.assoc_legendre_normalised(Lband, m, x_to)
        Pf = sphere.assoc_legendre_normalised(Lband, m, x_from)
        maps.append(Pt.T @ (Pf * w_from[None, :]))
    return maps


def resample(X, Lband, g_from, g_to, maps):
    """Band-limited resampling of X [..., ntheta_from, nphi_from] onto g_to,
    keeping degrees <= Lband, in three stages:
      s1  Xhat[i, m] = (1/Nphi) sum_j X[i, j] exp(-i m phi_j), |m| <= Lband
      s2  Yhat[i', m] = sum_i M_|m|[i', i] Xhat[i, m]
      s3  Y[i', j'] = sum_m Yhat[i', m] exp(i m phi'_j')
    """
    m = np.arange(-Lband, Lband + 1)
    E1 = np.exp(-1j * np.outer(g_from.phi, m)) / g_from.nphi
    Xhat = X @ E1
    Yhat = np.empty(X.shape[:-2] + (g_to.ntheta, m.size), dtype=np.complex128)
    for col, mm in enumerate(m):
        Yhat[..., col] = Xhat[..., col] @ maps[abs(mm)].T
    E3 = np.exp(1j * np.outer(m, g_to.phi))
    return Yhat @ E3


class Operators:
    """Per-level truncation orders, grids, translation operators, shift
    phases and interpolation/anterpolation maps for a tree and wavenumber."""

    def __init__(self, tree, k, digits=3, orders=None):
        self.tree = tree
        self.k = float(k)
        self.digits = digits
        self.L = {}
        self.grid = {}
        self.T = {}
        top = 3
        for lev in range(top, tree.n_lev + 1):
            a = tree.levels[lev].a
            L = orders[lev] if orders is not None else \
                truncation_order(self.k, a, digits)
            self.L[lev] = L
            self.grid[lev] = sphere.SphereGrid(L)
        for lev in range(top, tree.n_lev + 1):
            obs, src, typ = tree.far[lev]
            a = tree.levels[lev].a
            tab = {}
            for t in np.unique(typ):
                dx, rem = divmod(int(t), 49)
                dy, dz = divmod(rem, 7)
                X = a * np.array([dx - 3, dy - 3, dz - 3], dtype=np.float64)
                tab[int(t)] = translation_operator(self.k, self.L[lev], X,
                                                   self.grid[lev])
            self.T[lev] = tab
        # interpolation (child lev+1 -> parent lev) and anterpolation maps
        self.interp = {}
        self.anterp = {}
        for lev in range(top, tree.n_lev):
            gc, gp = self.grid[lev + 1], self.grid[lev]
            Lc = self.L[lev + 1]
            self.interp[lev] = legendre_map(Lc, gc.x, gc.wx, gp.x)
            self.anterp[lev] = legendre_map(Lc, gp.x, gp.wx, gc.x)


# --------------------------------------------------------------------------
# The five stages and the near field
# --------------------------------------------------------------------------

def c2m(tree, ops, q_sorted):
    """C2M (Sec. 3.2.1): S_b(khat) = sum_{j in b} q_j exp(-ik khat.(r_j - c_b))."""
    lev = tree.n_lev
    g = ops.grid[lev]
    L = tree.levels[lev]
    R = q_sorted.shape[1]
    S = np.zeros((L.nbox, R, g.K), dtype=np.complex128)
    xyz = tree.xyz[tree.perm]
    for b in range(L.nbox):
        s, e = tree.pt_start[b], tree.pt_end[b]
        d = xyz[s:e] - L.centres[b]
        E = np.exp(-1j * ops.k * (d @ g.khat.T))       # [n_b, K]
        S[b] = q_sorted[s:e].T @ E
    return S


def m2m(tree, ops, S_child, lev):
    """M2M (Sec. 3.2.2, its algorithm): interpolate each child of level
    lev+1 onto the parent grid, shift it to the parent centre with
    exp(-ik khat.(c_c - c_p)), and aggregate into the parent."""
    gc, gp = ops.grid[lev + 1], ops.grid[lev]
    Lc = ops.L[lev + 1]
    C = tree.levels[lev + 1]
    P = tree.levels[lev]
    B, R, _ = S_child.shape
    X = S_child.reshape(B, R, gc.ntheta, gc.nphi)
    Y = resample(X, Lc, gc, gp, ops.interp[lev]).reshape(B, R, gp.K)
    d = C.centres - P.centres[C.parent]                 # [B, 3]
    shift = np.exp(-1j * ops.k * (d @ gp.khat.T))       # [B, Kp]
    S_parent = np.zeros((P.nbox, R, gp.K), dtype=np.complex128)
    np.add.at(S_parent, C.parent, shift[:, None, :] * Y)
    return S_parent


def m2l(tree, ops, S, lev):
    """M2L (Sec. 3.2.3): L_b = sum over the far-field list of b of
    T_{lev, type(b, b')} * S_{b'} (elementwise over samples)."""
    obs, src, typ = tree.far[lev]
    nbox = tree.levels[lev].nbox
    R, K = S.shape[1], S.shape[2]
    Lloc = np.zeros((nbox, R, K), dtype=np.complex128)
    tab = ops.T[lev]
    for i in range(obs.size):
        Lloc[obs[i]] += tab[int(typ[i])][None, :] * S[src[i]]
    return Lloc


def m2l_fast(tree, ops, S, lev, chunk=4096):
    """Same sum as ``m2l``, grouped by observer in chunks (numpy speed)."""
    obs, src, typ = tree.far[lev]
    nbox = tree.levels[lev].nbox
    R, K = S.shape[1], S.shape[2]
    Lloc = np.zeros((nbox, R, K), dtype=np.complex128)
    if obs.size == 0:
        return Lloc
    tlist = sorted(ops.T[lev])
    tidx = np.searchsorted(np.array(tlist), typ)
    Ttab = np.stack([ops.T[lev][t] for t in tlist])     # [ntypes, K]
    starts = np.searchsorted(obs, np.arange(nbox), side="left")
    ends = np.searchsorted(obs, np.arange(nbox), side="right")
    b0 = 0
    while b0 < nbox:
        b1 = b0
        while b1 < nbox and ends[b1] - starts[b0] <= chunk:
            b1 += 1
        b1 = max(b1, b0 + 1)
        p0, p1 = starts[b0], ends[b1 - 1]
        if p1 > p0:
            prod = Ttab[tidx[p0:p1]][:, None, :] * S[src[p0:p1]]
            seg = starts[b0:b1] - p0
            nonempty = ends[b0:b1] > starts[b0:b1]
            sums = np.add.reduceat(prod, seg[nonempty], axis=0)
            Lloc[np.arange(b0, b1)[nonempty]] = sums
        b0 = b1
    return Lloc


def l2l(tree, ops, L_parent, L_child_m2l, lev):
    """L2L (Sec. 3.2.4): shift the parent local (level lev) to each child
    centre with exp(+ik khat.(c_c - c_p)) on the parent grid, anterpolate
    to the child grid (band L_child), and add to the child's M2L result."""
    gc, gp = ops.grid[lev + 1], ops.grid[lev]
    Lc = ops.L[lev + 1]
    C = tree.levels[lev + 1]
    P = tree.levels[lev]
    R = L_parent.shape[1]
    d = C.centres - P.centres[C.parent]
    shift = np.exp(1j * ops.k * (d @ gp.khat.T))        # [B, Kp]
    X = (shift[:, None, :] * L_parent[C.parent]).reshape(
        C.nbox, R, gp.ntheta, gp.nphi)
    Y = resample(X, Lc, gp, gc, ops.anterp[lev]).reshape(C.nbox, R, gc.K)
    return L_child_m2l + Y


def l2o(tree, ops, Lleaf):
    """L2O (Sec. 3.2.5): phi_i = (ik/4pi) sum_q w_q exp(ik khat_q.(r_i-c_b)) L_b(khat_q)."""
    lev = tree.n_lev
    g = ops.grid[lev]
    L = tree.levels[lev]
    R = Lleaf.shape[1]
    xyz = tree.xyz[tree.perm]
    out = np.zeros((tree.n, R), dtype=np.complex128)
    for b in range(L.nbox):
        s, e = tree.pt_start[b], tree.pt_end[b]
        d = xyz[s:e] - L.centres[b]
        E = np.exp(1j * ops.k * (d @ g.khat.T)) * g.w[None, :]
        out[s:e] = E @ Lleaf[b].T
    return out * (1j * ops.k / (4.0 * np.pi))


def near_field(tree, q_sorted, k):
    """Direct sum over the near-field leaves (Sec. 2: only at the leaf level)."""
    xyz = tree.xyz[tree.perm]
    R = q_sorted.shape[1]
    out = np.zeros((tree.n, R), dtype=np.complex128)
    for b, nb in enumerate(tree.near):
        s, e = tree.pt_start[b], tree.pt_end[b]
        idx = np.concatenate([np.arange(tree.pt_start[c], tree.pt_end[c])
                              for c in nb])
        out[s:e] = dense.potential(xyz[idx], q_sorted[idx], k, tgt=xyz[s:e])
    return out


def matvec(tree, ops, q, keep=False, fast=True):
    """phi = near + far for charges q [N] or [N, R] in the caller's order.

    With keep=True also returns the intermediates: leaf spectra, multipoles
    per level, locals after M2L and after L2L per level, near and far parts
    (sorted order)."""
    q = np.asarray(q)
    squeeze = q.ndim == 1
    q = q.reshape(tree.n, -1).astype(np.complex128)
    qs = q[tree.perm]
    inter = {}
    phi_s = near_field(tree, qs, ops.k)
    inter["near"] = phi_s.copy()
    if tree.n_lev >= 3:
        S = {tree.n_lev: c2m(tree, ops, qs)}
        for lev in range(tree.n_lev - 1, 2, -1):
            S[lev] = m2m(tree, ops, S[lev + 1], lev)
        f = m2l_fast if fast else m2l
        Lm2l = {lev: f(tree, ops, S[lev], lev)
                for lev in range(3, tree.n_lev + 1)}
        Lloc = {3: Lm2l[3]}
        for lev in range(3, tree.n_lev):
            Lloc[lev + 1] = l2l(tree, ops, Lloc[lev], Lm2l[lev + 1], lev)
        far = l2o(tree, ops, Lloc[tree.n_lev])
        inter.update(S=S, L_m2l=Lm2l, L=Lloc, far=far)
        phi_s = phi_s + far
    else:
        inter["far"] = np.zeros_like(phi_s)
    phi = np.empty_like(phi_s)
    phi[tree.perm] = phi_s
    if squeeze:
        phi = phi[:, 0]
    return (phi, inter) if keep else phi


def adjoint(tree, ops, v, **kw):
    """psi = conj(A~ conj(v)); A~ is symmetric, so this is A~^H v."""
    return np.conj(matvec(tree, ops, np.conj(v), **kw))
