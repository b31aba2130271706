// Launchers of the MLFMA HIP kernels (gfx950).  All pointers are device
// pointers; every launcher enqueues on `s` and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

namespace mlfma {
namespace dev {

// qs[s][r] = (conj?) q[perm[s]][r], converted to complex64
hipError_t gather(const void *q, int dtype, const int32_t *perm, int64_t n,
                  int R, int conj, float2 *qs, hipStream_t s);

// out[s][r] = 0
hipError_t zero(float2 *p, int64_t count, hipStream_t s);

// near-field potential (field = 0) or gradient (field = 1) in sorted order:
// out [n][R] or [n][R][3]; items[w] = (leaf, first target offset) covers up
// to 64 targets of that leaf; the first nheavy items (dense leaves) run with
// four waves per item
hipError_t p2p(const int2 *items, int64_t nitems, int64_t nheavy, const float4 *pts,
               const int32_t *pt_start, const int32_t *near_start, const int32_t *near_idx,
               const int32_t *leaf_coord, float leaf, float kw, const float2 *qs, int R,
               int field, float2 *out, hipStream_t s);

// C2M: S[b][r][k] = sum_{j in b} q_j exp(-i kw khat_k . d_j)
hipError_t c2m(const float4 *pts, const int32_t *pt_start, int64_t nleaf,
               const float4 *khat_w, int64_t K, float kw, const float2 *qs,
               int R, float2 *S, hipStream_t s);

// Interpolation stages (interp.hip).  T1 layout [col][(box, rhs)][theta_in],
// T2 layout [(box, rhs)][col][theta_out].
// M2M s1: T1 = child spectra x F (phi DFT on the child grid)
// (bf16x3: the BF16 split-precision MFMA path; FP32 MFMA otherwise)
hipError_t interp_s1(const float2 *Sc, int64_t BR, int nthc, int nphc, const float *F,
                     int M, float2 *T1, hipStream_t s, bool bf16x3);

// L2L s1 with the shift fused: rows (child c, r, theta_p) of the parent's
// local shifted by conj(shift[oct(c)])
hipError_t anterp_s1(const float2 *Lp, const int32_t *parent, const uint8_t *oct,
                     int64_t nchild, int R, int nthp, int nphp,
                     const float2 *shift, const float *F, int M, float2 *out,
                     hipStream_t s, bool bf16x3);

// s2: T2[br][col][i'] = sum_i mapsT[m(col)][i][i'] T1[col][br][i]
hipError_t theta_map(const float2 *T1, int64_t BR, int nin, int M,
                     const float *mapsT, int nout, float2 *T2, hipStream_t s, bool bf16x3);

// M2M s3 + shift + aggregation (parent-centric, no atomics)
hipError_t interp_s3(int64_t nboxp, int R, int nthp, int nphp, int M,
                     const int32_t *child_start, const uint8_t *child_oct,
                     const float2 *Yh, const float *G, const float2 *shift,
                     float2 *Sp, hipStream_t s);

// L2L s3 + add into the child's local expansion
hipError_t anterp_s3(int64_t nboxc, int R, int nthc, int nphc, int M,
                     const float2 *Yh, const float *G, float2 *Lc, hipStream_t s, bool bf16x3);

// One-pass M2M / L2L of a level pair (fused.hip): the three maps run back to
// back in LDS per parent box and right-hand side.  Lc, Lp: bands of the
// child and parent levels (only instantiated pairs, see pair_onepass_fits).
// M2M: Sp[p][r] = sum_{c in p} shift[oct c] (.) interp(Sc[c][r])
// L2L: Lch[c][r] += anterp(conj(shift[oct c]) (.) Lpar[parent c][r])
// F [nphi_in][M], A [(M+1)/2][ntheta_in][ntheta_out], G [M][nphi_out];
// E3: the axis factors of the shift on the parent grid.
// shape: the work split, 0 .. pair_onepass_shapes(Lc, Lp) - 1.
// Fused level-pair map (pair.hip): the three maps, the shift and the
// sibling sum (M2M, written to the parent) or the add into the child's
// local (L2L) in one launch over tiles of whole parents.  Instantiated
// pairs and directions only (pair_kernel_fits).  pair_tables builds the operator
// fragment tables on the host from the pair's maps (M2M: iF, iA, iG; L2L:
// aF, aB, aG) and states the tile limit (children per tile, whole parents);
// desc[2g], desc[2g + 1] describe group g: (first parent, first child,
// children, parents) and (octant of child slot i at bits 3i, first slot of
// parent j = 1..7 at bits 4(j - 1), parent of slot i at bits 3i, 0).
struct PairTables {
    std::vector<float> fr1, fr2, fr3;
    int max_children = 0, max_parents = 0;
};
bool pair_kernel_fits(int Lc, int Lp, bool down);
int pair_tables(int Lc, int Lp, bool down, const float *F, const float *A, const float *G,
                PairTables *t, bool bf16x3 = false);
hipError_t pair_map(int Lc, int Lp, bool down, const float2 *In, float2 *Out, const int4 *desc,
                    int64_t ngroups, int R, const float *fr1, const float *fr2, const float *fr3,
                    const float2 *shift_axis, const float2 *shift, hipStream_t st,
                    bool bf16x3 = false);

bool pair_onepass_fits(int Lc, int Lp);
int pair_onepass_shapes(int Lc, int Lp);
hipError_t interp_fused(int64_t nboxp, int R, int Lc, int Lp, int shape,
                        const int32_t *child_start, const uint8_t *child_oct, const float2 *Sc,
                        const float *F, const float *A, const float *G, const float2 *E3,
                        float2 *Sp, hipStream_t s);
hipError_t anterp_fused(int64_t nboxp, int R, int Lc, int Lp, int shape,
                        const int32_t *child_start, const uint8_t *child_oct, const float2 *Lpar,
                        const float *F, const float *B, const float *G, const float2 *E3,
                        float2 *Lch, hipStream_t s);

// out[i][a] = sum_r Re[conj(g[i][r]) Fq[i][r][a] + q[i][r] Fg[i][r][a]]
// (q, g caller order, dtype 0 = complex64 / 1 = complex128; out float/double)
hipError_t position_grad_combine(const void *q, const void *g, int dtype, const float2 *Fq,
                                 const float2 *Fg, int64_t n, int R, void *out, hipStream_t s);

// M2L: Lout[b][r][k] = sum_{e in far(b)} T[type_e][k] S[src_e][r][k]
hipError_t m2l(int64_t nbox, int64_t K, const int32_t *far_start,
               const int32_t *far_src, const int16_t *far_type, const float2 *T,
               const float2 *S, int R, float2 *Lout, hipStream_t s);

// M2L by sibling groups with per-source records: rec_src[e] source box,
// rec_off[8e + i] byte offset of the operator row of (child i of the parent,
// source) in the LDS slice of 64 samples (row ntypes = zeros: no interaction);
// each parent's records are padded to a multiple of 4 with zero records
// compute units of the current device
// Timing of the next M2L launch: when start is set, the M2L launchers
// launch with hipExtLaunchKernelGGL and these events, which the dispatch
// itself records at its start and end (no marker packets in the stream
// between kernels), and set used.  The caller arms and disarms it.
struct LaunchTiming {
    hipEvent_t start = nullptr, stop = nullptr;
    bool used = false;
};
extern thread_local LaunchTiming launch_timing;

int cu_count();

// schedule: 0 contiguous parent ranges, 1 the slice-major sweep for many
// right-hand sides, 2 ranges balanced by record count with dynamic parents,
// 3 the same with a 32-sample slice and half-waves on record pairs (one RHS;
// several RHS take 2);
// max_wg caps the resident workgroups (0: the CU count)
// One RHS, antipodal slices (operators of one offset of each +-pair,
// mirrored lanes for the other): Tp [ntp][Kp] operators in slice-lane
// order, aperm [Kp] slice lane -> sample (-1 past the end), record slots
// pair * 512 | (negated ? 504 : 0); max_wg as for m2l_rec
hipError_t m2l_anti(int64_t nparent, int64_t K, int ntp, const int32_t *child_start,
                    const int32_t *rec_start, const int32_t *rec_src, const int32_t *rec_off,
                    const float2 *Tp, const int32_t *aperm, int64_t Kp, const float2 *S,
                    float2 *Lout, hipStream_t s, int max_wg = 0, int waves = 16);

// Sampled translation operators (Sec. 3.2.3 "Translation Operators"): per
// distinct offset length a table of T at gamma_m = m pi / M (m = 0..M)
// against the angle gamma between the direction and the offset, and per
// operator its integer offset with the table row in w; the M2L record
// kernel interpolates its LDS slice of operators from them (10-point
// Lagrange, mirrored at 0 and pi) instead of copying it from a full table.
struct SampledT {
    const float2 *tab = nullptr;    // [nrad][M + 1]
    const float4 *xr = nullptr;     // [ntypes]: integer offset (dx, dy, dz), table row
    // grid directions in FP64: (cos, sin) of theta_i at [2 i], of phi_j at
    // [2 nth + 2 j]; sample k = i nph + j
    const double *trig = nullptr;
    int nth = 0, nph = 0;
    int M = 0;
};

hipError_t m2l_rec(int64_t nparent, int64_t K, int ntypes, const int32_t *child_start,
                   const int32_t *rec_start, const int32_t *rec_src, const int32_t *rec_off,
                   const float2 *T, const float2 *S, int R, float2 *Lout, hipStream_t s,
                   int schedule, int max_wg = 0, SampledT sampled = SampledT());

// M2L on the matrix cores for several right-hand sides (variant 9): the
// records and operator slices of m2l_rec; per sample, the parent's children
// (in pairs) x the right-hand sides (in fours) accumulate operator x source
// over the records on v_mfma_f32_4x4x1f32
hipError_t m2l_mfma(int64_t nparent, int64_t K, int ntypes, const int32_t *child_start,
                    const int32_t *rec_start, const int32_t *rec_src, const int32_t *rec_off,
                    const float2 *T, const float2 *S, int R, float2 *Lout, hipStream_t s,
                    int max_wg = 0, SampledT sampled = SampledT());

// M2L per observer with the operator slice in LDS
hipError_t m2l_lds(int64_t nbox, int64_t K, int ntypes, const int32_t *far_start,
                   const int32_t *far_src, const int16_t *far_type, const float2 *T,
                   const float2 *S, int R, float2 *Lout, hipStream_t s);

// M2L by sibling groups: parents at level l-1 (child ranges child_start),
// their neighbour parents (CSR nbr_start/nbr_idx, Chebyshev 1, self
// excluded), base = 49 cx + 7 cy + cz of the level-l boxes, typemap[343]
// = operator index of an offset code or -1 (near / unused)
hipError_t m2l_sg(int64_t nparent, int64_t K, int ntypes, const int32_t *child_start,
                  const int32_t *nbr_start, const int32_t *nbr_idx, const int32_t *base,
                  const int16_t *typemap, const float2 *T, const float2 *S, int R,
                  float2 *Lout, hipStream_t s);

// L2O + near + scatter to caller order:
// out[perm[s]][r] = near[s][r] + (i kw / 4 pi) sum_k w_k e^{i kw khat.d_s} L[b][r][k]
// (field = 1: gradient, extra factor i kw khat, out [n][R][3]).  With
// far = 0 only the near part is scattered (L, khat_w unused).
hipError_t l2o_scatter(const float4 *pts, const int32_t *pt_leaf,
                       const int32_t *perm, const float4 *khat_w, int64_t K,
                       float kw, const float2 *L, const float2 *near, int64_t n,
                       int R, int field, int far, int conj_out, int dtype,
                       void *out, hipStream_t s);

// L2O + near + scatter for R >= 8 potentials: per leaf box an MFMA product of
// the phase matrix [points x K] and the locals [K x R] (pt_start: leaf CSR).
hipError_t l2o_leaf_mfma(const float4 *pts, const int32_t *pt_start, int64_t nleaf,
                         const int32_t *perm, const float4 *khat_w, int64_t K, float kw,
                         const float2 *L, const float2 *near, int R, int conj_out, int dtype,
                         void *out, hipStream_t s);

// GMRES vector kernels (complex64 vectors, FP64 coefficients):
// partial[i * nb + blk] = block partial of sum_j conj(V[i][j]) w[j], i < m
// (nb = gm_dot_blocks(n) blocks; the host adds the partials);
// w += sign * sum_{i < m} V[i] c[i] (c in device memory); y = a x + b y
int gm_dot_blocks(int64_t n);
hipError_t gm_dots(const float2 *V, int64_t ldv, int m, const float2 *w, int64_t n, int nb,
                   double2 *partial, hipStream_t s);
hipError_t gm_combine(float2 *w, const float2 *V, int64_t ldv, int m, const double2 *c,
                      double sign, int64_t n, hipStream_t s);
hipError_t gm_axpby(float2 *y, double2 a, const float2 *x, double2 b, int64_t n, hipStream_t s);

}  // namespace dev
}  // namespace mlfma
