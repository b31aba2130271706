// Octree construction on the host (Sec. 2 FMM paragraph; Sec. 3.1).
//
// Level count: smallest n_lev with leaf * 2^(n_lev-1) >= E (E = largest
// bounding-box side), i.e. the paper's L >= log2(D0/D(L)) + 1.  The root cube
// of side leaf * 2^(n_lev-1) is centred on the bounding box; points get leaf
// integer coordinates floor((r - origin)/leaf), clamped into the cube, and
// Morton-Z keys (Sec. 3.1); boxes at coarser levels are the keys shifted by 3
// bits per level.  Near lists (leaf level) hold boxes at Chebyshev distance
// <= 1; far lists (levels >= 3) hold boxes at distance >= 2 whose parents
// are at distance <= 1 (Sec. 2).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <numeric>
#include <thread>

#include "internal.h"

namespace mlfma {

static thread_local char g_err[512];

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

const char *last_error_text() { return g_err; }

static inline uint64_t spread3(uint32_t v)
{
    uint64_t x = v & 0x1fffff;  // 21 bits
    x = (x | (x << 32)) & 0x1f00000000ffffULL;
    x = (x | (x << 16)) & 0x1f0000ff0000ffULL;
    x = (x | (x << 8)) & 0x100f00f00f00f00fULL;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ULL;
    x = (x | (x << 2)) & 0x1249249249249249ULL;
    return x;
}

static inline uint32_t compact3(uint64_t x)
{
    x &= 0x1249249249249249ULL;
    x = (x | (x >> 2)) & 0x10c30c30c30c30c3ULL;
    x = (x | (x >> 4)) & 0x100f00f00f00f00fULL;
    x = (x | (x >> 8)) & 0x1f0000ff0000ffULL;
    x = (x | (x >> 16)) & 0x1f00000000ffffULL;
    x = (x | (x >> 32)) & 0x1fffffULL;
    return (uint32_t)x;
}

uint64_t morton_key(uint32_t x, uint32_t y, uint32_t z)
{
    return (spread3(x) << 2) | (spread3(y) << 1) | spread3(z);
}

void morton_decode(uint64_t key, int32_t *c)
{
    c[0] = (int32_t)compact3(key >> 2);
    c[1] = (int32_t)compact3(key >> 1);
    c[2] = (int32_t)compact3(key);
}

// index of `key` in the sorted level keys, or -1
static inline int64_t find_box(const HostLevel &L, uint64_t key)
{
    auto it = std::lower_bound(L.key.begin(), L.key.end(), key);
    if (it == L.key.end() || *it != key) return -1;
    return it - L.key.begin();
}

static void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)> &fn)
{
    unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    int64_t nth = std::min<int64_t>(hw, std::max<int64_t>(1, n / 256));
    if (nth <= 1) { fn(0, n); return; }
    std::vector<std::thread> th;
    int64_t chunk = (n + nth - 1) / nth;
    for (int64_t t = 0; t < nth; ++t) {
        int64_t b = t * chunk, e = std::min(n, b + chunk);
        if (b >= e) break;
        th.emplace_back(fn, b, e);
    }
    for (auto &x : th) x.join();
}

static void build_far_lists(Tree &t, int l)
{
    HostLevel &L = t.lev[l];
    const HostLevel &P = t.lev[l - 1];
    const HostLevel &Lc = t.lev[l];
    std::vector<std::vector<std::pair<int32_t, int16_t>>> per(L.nbox);
    parallel_for(L.nbox, [&](int64_t b0, int64_t b1) {
        for (int64_t b = b0; b < b1; ++b) {
            const int32_t *cb = &L.coord[3 * b];
            int32_t p = L.parent[b];
            const int32_t *cp = &P.coord[3 * p];
            int32_t pside = 1 << (l - 2);
            auto &out = per[b];
            for (int dx = -1; dx <= 1; ++dx)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dz = -1; dz <= 1; ++dz) {
                        int32_t nx = cp[0] + dx, ny = cp[1] + dy, nz = cp[2] + dz;
                        if (nx < 0 || ny < 0 || nz < 0 || nx >= pside ||
                            ny >= pside || nz >= pside)
                            continue;
                        int64_t q = find_box(P, morton_key(nx, ny, nz));
                        if (q < 0) continue;
                        for (int32_t c = P.child_start[q]; c < P.child_start[q + 1]; ++c) {
                            const int32_t *cc = &Lc.coord[3 * c];
                            int ex = cb[0] - cc[0], ey = cb[1] - cc[1], ez = cb[2] - cc[2];
                            int cheb = std::max(std::abs(ex), std::max(std::abs(ey), std::abs(ez)));
                            if (cheb < 2) continue;
                            out.emplace_back(c, (int16_t)((ex + 3) * 49 + (ey + 3) * 7 + (ez + 3)));
                        }
                    }
            std::sort(out.begin(), out.end());
        }
    });
    L.far_start.assign(L.nbox + 1, 0);
    for (int64_t b = 0; b < L.nbox; ++b) L.far_start[b + 1] = L.far_start[b] + (int32_t)per[b].size();
    L.far_src.resize(L.far_start[L.nbox]);
    L.far_code.resize(L.far_start[L.nbox]);
    for (int64_t b = 0; b < L.nbox; ++b) {
        int32_t o = L.far_start[b];
        for (size_t i = 0; i < per[b].size(); ++i) {
            L.far_src[o + i] = per[b][i].first;
            L.far_code[o + i] = per[b][i].second;
        }
    }
}

int build_tree(const double *xyz, int64_t n, double leaf, int max_levels,
               int device, Tree **out)
{
    if (!out) return fail(MLFMA_EINVAL, "build_tree: out is NULL");
    *out = nullptr;
    if (n < 0) return fail(MLFMA_EINVAL, "build_tree: n < 0");
    if (n > 0 && !xyz) return fail(MLFMA_EINVAL, "build_tree: xyz is NULL");
    if (n > (int64_t)INT32_MAX) return fail(MLFMA_EINVAL, "build_tree: n too large");
    if (!(leaf > 0.0) || !std::isfinite(leaf))
        return fail(MLFMA_EINVAL, "build_tree: leaf_size must be positive and finite");
    if (max_levels < 1 || max_levels > 21)
        return fail(MLFMA_EINVAL, "build_tree: max_levels must be in 1..21");
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!std::isfinite(xyz[i]))
            return fail(MLFMA_EINVAL, "build_tree: non-finite coordinate at point %lld",
                        (long long)(i / 3));

    Tree *t = new (std::nothrow) Tree();
    if (!t) return fail(MLFMA_ENOMEM, "build_tree: out of host memory");
    t->n = n;
    t->leaf = leaf;
    t->device = device;
    try {
        t->xyz.assign(xyz, xyz + 3 * n);
        double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        if (n > 0) {
            for (int a = 0; a < 3; ++a) lo[a] = hi[a] = xyz[a];
            for (int64_t i = 1; i < n; ++i)
                for (int a = 0; a < 3; ++a) {
                    lo[a] = std::min(lo[a], xyz[3 * i + a]);
                    hi[a] = std::max(hi[a], xyz[3 * i + a]);
                }
        }
        double extent = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
        int n_lev = 1;
        while (std::ldexp(leaf, n_lev - 1) < extent) {
            ++n_lev;
            if (n_lev > max_levels || n_lev > 21) {
                delete t;
                return fail(MLFMA_EDEPTH, "build_tree: needs more than %d levels",
                            std::min(max_levels, 21));
            }
        }
        t->n_lev = n_lev;
        t->D0 = std::ldexp(leaf, n_lev - 1);
        for (int a = 0; a < 3; ++a) t->origin[a] = 0.5 * (lo[a] + hi[a]) - 0.5 * t->D0;

        const int64_t nside = (int64_t)1 << (n_lev - 1);
        std::vector<uint64_t> key(n);
        for (int64_t i = 0; i < n; ++i) {
            int64_t c[3];
            for (int a = 0; a < 3; ++a) {
                double f = std::floor((xyz[3 * i + a] - t->origin[a]) / leaf);
                int64_t v = (int64_t)f;
                c[a] = std::min<int64_t>(std::max<int64_t>(v, 0), nside - 1);
            }
            key[i] = morton_key((uint32_t)c[0], (uint32_t)c[1], (uint32_t)c[2]);
        }
        t->perm.resize(n);
        std::iota(t->perm.begin(), t->perm.end(), 0);
        std::stable_sort(t->perm.begin(), t->perm.end(),
                         [&](int64_t a, int64_t b) { return key[a] < key[b]; });
        std::vector<uint64_t> skey(n);
        for (int64_t s = 0; s < n; ++s) skey[s] = key[t->perm[s]];

        t->lev.resize(n_lev + 1);
        for (int l = 1; l <= n_lev; ++l) {
            HostLevel &L = t->lev[l];
            L.level = l;
            L.a = std::ldexp(t->D0, -(l - 1));
            int sh = 3 * (n_lev - l);
            for (int64_t s = 0; s < n; ++s) {
                uint64_t k = skey[s] >> sh;
                if (L.key.empty() || L.key.back() != k) L.key.push_back(k);
            }
            L.nbox = (int64_t)L.key.size();
            L.coord.resize(3 * L.nbox);
            for (int64_t b = 0; b < L.nbox; ++b) morton_decode(L.key[b], &L.coord[3 * b]);
            L.parent.assign(L.nbox, -1);
            if (l > 1) {
                const HostLevel &P = t->lev[l - 1];
                for (int64_t b = 0; b < L.nbox; ++b)
                    L.parent[b] = (int32_t)find_box(P, L.key[b] >> 3);
            }
        }
        for (int l = 1; l < n_lev; ++l) {
            HostLevel &L = t->lev[l];
            const HostLevel &C = t->lev[l + 1];
            L.child_start.assign(L.nbox + 1, 0);
            for (int64_t b = 0; b < L.nbox; ++b)
                L.child_start[b] = (int32_t)(std::lower_bound(C.key.begin(), C.key.end(),
                                                              L.key[b] << 3) - C.key.begin());
            L.child_start[L.nbox] = (int32_t)C.nbox;
        }
        // points of each leaf
        HostLevel &leafL = t->lev[n_lev];
        t->pt_start.assign(leafL.nbox + 1, 0);
        t->pt_leaf.resize(n);
        {
            int64_t b = -1;
            for (int64_t s = 0; s < n; ++s) {
                if (s == 0 || skey[s] != skey[s - 1]) t->pt_start[++b] = s;
                t->pt_leaf[s] = (int32_t)b;
            }
            t->pt_start[leafL.nbox] = n;
        }
        // near lists
        t->near_start.assign(leafL.nbox + 1, 0);
        {
            std::vector<std::vector<int32_t>> per(leafL.nbox);
            for (int64_t b = 0; b < leafL.nbox; ++b) {
                const int32_t *c = &leafL.coord[3 * b];
                for (int dx = -1; dx <= 1; ++dx)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dz = -1; dz <= 1; ++dz) {
                            int64_t x = c[0] + dx, y = c[1] + dy, z = c[2] + dz;
                            if (x < 0 || y < 0 || z < 0 || x >= nside || y >= nside || z >= nside)
                                continue;
                            int64_t q = find_box(leafL, morton_key((uint32_t)x, (uint32_t)y, (uint32_t)z));
                            if (q >= 0) per[b].push_back((int32_t)q);
                        }
                std::sort(per[b].begin(), per[b].end());
                t->near_start[b + 1] = t->near_start[b] + (int64_t)per[b].size();
            }
            t->near_idx.resize(t->near_start[leafL.nbox]);
            for (int64_t b = 0; b < leafL.nbox; ++b) {
                std::copy(per[b].begin(), per[b].end(), t->near_idx.begin() + t->near_start[b]);
                int64_t src = 0;
                for (int32_t q : per[b]) src += t->pt_start[q + 1] - t->pt_start[q];
                t->n_p2p_pairs += (t->pt_start[b + 1] - t->pt_start[b]) * src;
            }
        }
        for (int l = 3; l <= n_lev; ++l) build_far_lists(*t, l);
    } catch (const std::bad_alloc &) {
        delete t;
        return fail(MLFMA_ENOMEM, "build_tree: out of host memory");
    }
    *out = t;
    return MLFMA_OK;
}

void neighbour_lists(const Tree &t, int l, std::vector<int32_t> &start, std::vector<int32_t> &idx)
{
    const HostLevel &L = t.lev[l];
    const int64_t side = (int64_t)1 << (l - 1);
    start.assign(L.nbox + 1, 0);
    idx.clear();
    for (int64_t b = 0; b < L.nbox; ++b) {
        const int32_t *c = &L.coord[3 * b];
        for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dz = -1; dz <= 1; ++dz) {
                    if (!dx && !dy && !dz) continue;
                    const int64_t x = c[0] + dx, y = c[1] + dy, z = c[2] + dz;
                    if (x < 0 || y < 0 || z < 0 || x >= side || y >= side || z >= side) continue;
                    const int64_t q = find_box(L, morton_key((uint32_t)x, (uint32_t)y, (uint32_t)z));
                    if (q >= 0) idx.push_back((int32_t)q);
                }
        start[b + 1] = (int32_t)idx.size();
    }
}

int update_positions(Tree *t, const double *xyz)
{
    if (!t) return fail(MLFMA_EINVAL, "update_positions: tree is NULL");
    if (t->n > 0 && !xyz) return fail(MLFMA_EINVAL, "update_positions: xyz is NULL");
    const int64_t nside = (int64_t)1 << (t->n_lev - 1);
    const HostLevel &leafL = t->lev[t->n_lev];
    for (int64_t s = 0; s < t->n; ++s) {
        int64_t i = t->perm[s];
        const int32_t *c = &leafL.coord[3 * t->pt_leaf[s]];
        for (int a = 0; a < 3; ++a) {
            double v = xyz[3 * i + a];
            if (!std::isfinite(v))
                return fail(MLFMA_EINVAL, "update_positions: non-finite coordinate");
            // the point must stay inside the root cube (up to the rounding
            // of a point on its faces, which build_tree clamps) and in its
            // leaf box: the leaf expansions and the near/far split assume it
            const double u = (v - t->origin[a]) / t->leaf;
            const double tol = 1e-9 * (double)nside;
            if (!(u >= -tol && u <= (double)nside + tol))
                return fail(MLFMA_ERANGE, "update_positions: point %lld left the root cube",
                            (long long)i);
            int64_t f = (int64_t)std::floor(u);
            f = std::min<int64_t>(std::max<int64_t>(f, 0), nside - 1);
            if (f != c[a])
                return fail(MLFMA_ERANGE, "update_positions: point %lld left its leaf box",
                            (long long)i);
        }
    }
    std::copy(xyz, xyz + 3 * t->n, t->xyz.begin());
    ++t->pos_version;
    return MLFMA_OK;
}

void release_tree(Tree *t)
{
    if (t && --t->refcount == 0) delete t;
}

}  // namespace mlfma
