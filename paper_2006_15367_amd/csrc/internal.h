// Internal structures of the MLFMA library (host side).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "mlfma.h"

namespace mlfma {

// Thread-local error text; returns `code` so callers can `return fail(...)`.
int fail(int code, const char *fmt, ...);

// Morton-Z key of integer box coordinates: bit b of x goes to key bit 3b+2,
// of y to 3b+1, of z to 3b.
uint64_t morton_key(uint32_t x, uint32_t y, uint32_t z);
void morton_decode(uint64_t key, int32_t *c);

// One level of the octree, boxes in Morton order.
struct HostLevel {
    int level = 0;
    double a = 0.0;                    // box side
    int64_t nbox = 0;
    std::vector<uint64_t> key;         // sorted Morton keys at this level
    std::vector<int32_t> coord;        // [nbox][3] integer box coordinates
    std::vector<int32_t> parent;       // index into level-1 (-1 at level 1)
    std::vector<int32_t> child_start;  // [nbox+1] into level+1 (not at leaf)
    std::vector<int32_t> far_start;    // [nbox+1] CSR of the far-field list
    std::vector<int32_t> far_src;      // source box index
    std::vector<int16_t> far_code;     // (dx+3)*49+(dy+3)*7+(dz+3), d = c_obs - c_src
};

struct Tree {
    int64_t n = 0;
    int n_lev = 0;
    int device = 0;
    double leaf = 0.0, D0 = 0.0, origin[3] = {0, 0, 0};
    std::vector<int64_t> perm;       // sorted position -> caller index
    std::vector<double> xyz;         // caller order [n][3]
    std::vector<int32_t> pt_leaf;    // sorted position -> leaf box
    std::vector<int64_t> pt_start;   // [nleaf+1] point ranges of the leaves
    std::vector<int64_t> near_start; // [nleaf+1]
    std::vector<int32_t> near_idx;   // near leaves (incl. self), ascending
    int64_t n_p2p_pairs = 0;         // sum over leaves of n_b * (near points)
    std::vector<HostLevel> lev;      // lev[1..n_lev]
    uint64_t pos_version = 0;        // bumped by mlfma_update_positions
    int refcount = 1;
};

int build_tree(const double *xyz, int64_t n, double leaf, int max_levels,
               int device, Tree **out);
int update_positions(Tree *t, const double *xyz);
void release_tree(Tree *t);
// boxes of level l at Chebyshev distance 1 (the box itself excluded), CSR
void neighbour_lists(const Tree &t, int l, std::vector<int32_t> &start,
                     std::vector<int32_t> &idx);

// Host (FP64) tables of one level l >= 3, stored in FP32 for the device.
struct LevelTables {
    int L = 0, nth = 0, nph = 0;
    int64_t K = 0;
    std::vector<double> x, wx;       // Gauss-Legendre nodes (descending), weights
    std::vector<float> khat_w;       // [K][4] (kx, ky, kz, quadrature weight)
    std::vector<int16_t> code_to_type; // [343] -> compact operator index or -1
    int ntypes = 0;
    std::vector<float> T;            // [ntypes][K][2] translation operators
    // sampled operators (instead of T): per distinct offset length a table
    // of T at gamma_m = m pi / Msamp, m = 0..Msamp, against the angle gamma
    // between the direction and the offset; per operator its integer
    // offset and table row
    int Msamp = 0, nrad = 0;
    std::vector<float> Tsamp;        // [nrad][Msamp + 1][2]
    std::vector<float> xr;           // [ntypes][4]: integer offset (dx, dy, dz), row
    std::vector<double> trig64;      // (cos, sin) of each theta node, then of each phi
    std::vector<int16_t> far_type;   // far list in compact operator indices
    // level pair (this level = parent p, level+1 = child c); empty at the leaf
    int Lc = 0, Mc = 0;              // child order, 2 Lc + 1 real-DFT columns
    std::vector<float> shift;        // [8][K][2] exp(-i k khat.(c_c - c_p))
    std::vector<float> shift_axis;   // [2K + nth][2]: exp(-i k (a/4) khat_x) over the grid,
                                     // the same for khat_y, then for khat_z per theta node
    std::vector<float> iF;           // [nph_c][Mc]   child-grid real DFT
    std::vector<float> iA;           // [Lc+1][nth_c][nth] theta maps (input index first)
    std::vector<float> iG;           // [Mc][nph]     parent-grid synthesis
    std::vector<float> aF;           // [nph][Mc]     parent-grid real DFT
    std::vector<float> aB;           // [Lc+1][nth][nth_c] theta maps (input index first)
    std::vector<float> aG;           // [Mc][nph_c]   child-grid synthesis
};

int truncation_order(double k, double a, int digits);
// oversampling of the sampled operators' tables and their stencil width
constexpr int kSampledOversample = 8;
constexpr int kSampledPoints = 10;
// sampled = true: the translation operators as sampled tables (Tsamp, xr)
// instead of their values on the grid (T)
int build_level_tables(const Tree &t, double k, int digits,
                       std::vector<LevelTables> &out, bool sampled = false);

}  // namespace mlfma
