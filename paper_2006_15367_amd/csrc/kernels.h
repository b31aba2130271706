// Launchers of the MLFMA HIP kernels (gfx950).  All pointers are device
// pointers; every launcher enqueues on `s` and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mlfma {
namespace dev {

// qs[s][r] = (conj?) q[perm[s]][r], converted to complex64
hipError_t gather(const void *q, int dtype, const int32_t *perm, int64_t n,
                  int R, int conj, float2 *qs, hipStream_t s);

// out[s][r] = 0
hipError_t zero(float2 *p, int64_t count, hipStream_t s);

// near-field potential (field = 0) or gradient (field = 1) in sorted order:
// out [n][R] or [n][R][3]
hipError_t p2p(const float4 *pts, const int32_t *pt_leaf, const int32_t *pt_start,
               const int32_t *near_start, const int32_t *near_idx,
               const int32_t *leaf_coord, float leaf, float kw, const float2 *qs,
               int64_t n, int R, int field, float2 *out, hipStream_t s);

// C2M: S[b][r][k] = sum_{j in b} q_j exp(-i kw khat_k . d_j)
hipError_t c2m(const float4 *pts, const int32_t *pt_start, int64_t nleaf,
               const float4 *khat_w, int64_t K, float kw, const float2 *qs,
               int R, float2 *S, hipStream_t s);

// s1: out[row][col] = sum_j X[row][j] F[j][col]  (rows of length nin)
hipError_t dft_rows(const float2 *X, int64_t rows, int nin, const float *F,
                    int M, float2 *out, hipStream_t s);

// L2L s1 with the shift fused: rows (child c, r, theta_p) of the parent's
// local shifted by conj(shift[oct(c)])
hipError_t anterp_s1(const float2 *Lp, const int32_t *parent, const uint8_t *oct,
                     int64_t nchild, int R, int nthp, int nphp,
                     const float2 *shift, const float *F, int M, float2 *out,
                     hipStream_t s);

// s2: Yh[br][i'][col] = sum_i maps[m(col)][i'][i] Xh[br][i][col]
hipError_t theta_map(const float2 *Xh, int64_t BR, int nin, int M,
                     const float *maps, int nout, float2 *Yh, hipStream_t s);

// M2M s3 + shift + aggregation (parent-centric, no atomics)
hipError_t interp_s3(int64_t nboxp, int R, int nthp, int nphp, int M,
                     const int32_t *child_start, const uint8_t *child_oct,
                     const float2 *Yh, const float *G, const float2 *shift,
                     float2 *Sp, hipStream_t s);

// L2L s3 + add into the child's local expansion
hipError_t anterp_s3(int64_t nboxc, int R, int nthc, int nphc, int M,
                     const float2 *Yh, const float *G, float2 *Lc, hipStream_t s);

// M2L: Lout[b][r][k] = sum_{e in far(b)} T[type_e][k] S[src_e][r][k]
hipError_t m2l(int64_t nbox, int64_t K, const int32_t *far_start,
               const int32_t *far_src, const int16_t *far_type, const float2 *T,
               const float2 *S, int R, float2 *Lout, hipStream_t s);

// L2O + near + scatter to caller order:
// out[perm[s]][r] = near[s][r] + (i kw / 4 pi) sum_k w_k e^{i kw khat.d_s} L[b][r][k]
// (field = 1: gradient, extra factor i kw khat, out [n][R][3]).  With
// far = 0 only the near part is scattered (L, khat_w unused).
hipError_t l2o_scatter(const float4 *pts, const int32_t *pt_leaf,
                       const int32_t *perm, const float4 *khat_w, int64_t K,
                       float kw, const float2 *L, const float2 *near, int64_t n,
                       int R, int field, int far, int conj_out, int dtype,
                       void *out, hipStream_t s);

}  // namespace dev
}  // namespace mlfma
