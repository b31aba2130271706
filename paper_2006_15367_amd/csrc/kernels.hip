// HIP kernels of the MLFMA matvec for gfx950.
//
// Layouts (all in HBM, sorted = Morton order of the points):
//   pts      [n] float4 (x, y, z offsets from the point's leaf-box centre, 0)
//   qs, near [n][R] complex64
//   spectra  [nbox][R][K] complex64, samples [theta][phi] (phi fastest)
//   tables   FP32 copies of the FP64 host precompute
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace mlfma {
namespace dev {

static constexpr float kInv4Pi = 0.0795774715459476679f;  // 1/(4 pi)

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 c)
{
    c.x = fmaf(a.x, b.x, c.x);
    c.x = fmaf(-a.y, b.y, c.x);
    c.y = fmaf(a.x, b.y, c.y);
    c.y = fmaf(a.y, b.x, c.y);
    return c;
}
// conj(a) * b + c
__device__ __forceinline__ float2 cfma_conj(float2 a, float2 b, float2 c)
{
    c.x = fmaf(a.x, b.x, c.x);
    c.x = fmaf(a.y, b.y, c.x);
    c.y = fmaf(a.x, b.y, c.y);
    c.y = fmaf(-a.y, b.x, c.y);
    return c;
}

static inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// ---------------------------------------------------------------- gather --
template <typename Tin>
__global__ void k_gather(const Tin *__restrict__ q, const int32_t *__restrict__ perm,
                         int64_t n, int R, int conj, float2 *__restrict__ qs)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * R) return;
    int64_t s = idx / R;
    int r = (int)(idx - s * R);
    Tin v = q[(int64_t)perm[s] * R + r];
    float im = (float)v.y;
    qs[idx] = make_float2((float)v.x, conj ? -im : im);
}

hipError_t gather(const void *q, int dtype, const int32_t *perm, int64_t n, int R,
                  int conj, float2 *qs, hipStream_t s)
{
    if (n * R == 0) return hipSuccess;
    if (dtype == 0)
        hipLaunchKernelGGL(k_gather<float2>, dim3(nblocks(n * R, 256)), dim3(256), 0, s,
                           (const float2 *)q, perm, n, R, conj, qs);
    else
        hipLaunchKernelGGL(k_gather<double2>, dim3(nblocks(n * R, 256)), dim3(256), 0, s,
                           (const double2 *)q, perm, n, R, conj, qs);
    return hipGetLastError();
}

__global__ void k_zero(float2 *__restrict__ p, int64_t count)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < count) p[idx] = make_float2(0.f, 0.f);
}

hipError_t zero(float2 *p, int64_t count, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3(nblocks(count, 256)), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

// ------------------------------------------------------------------- P2P --
// One thread per (target point, chunk of RC right-hand sides).  Sources are
// the points of the target leaf's near leaves; the pair vector is formed
// from leaf-local offsets plus the (exact) integer leaf offset times the
// leaf side, so it keeps FP32 accuracy for close pairs far from the origin.
template <int RC, bool FIELD>
__global__ void k_p2p(const float4 *__restrict__ pts, const int32_t *__restrict__ pt_leaf,
                      const int32_t *__restrict__ pt_start,
                      const int32_t *__restrict__ near_start,
                      const int32_t *__restrict__ near_idx,
                      const int32_t *__restrict__ coord, float leaf, float kw,
                      const float2 *__restrict__ qs, int64_t n, int R,
                      float2 *__restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int r0 = blockIdx.y * RC;
    const int rc = min(RC, R - r0);
    const float4 pi = pts[i];
    const int b = pt_leaf[i];
    const int cbx = coord[3 * b], cby = coord[3 * b + 1], cbz = coord[3 * b + 2];
    float2 acc[RC][FIELD ? 3 : 1];
#pragma unroll
    for (int c = 0; c < RC; ++c)
#pragma unroll
        for (int a = 0; a < (FIELD ? 3 : 1); ++a) acc[c][a] = make_float2(0.f, 0.f);
    for (int e = near_start[b]; e < near_start[b + 1]; ++e) {
        const int nb = near_idx[e];
        const float ox = (float)(coord[3 * nb] - cbx) * leaf;
        const float oy = (float)(coord[3 * nb + 1] - cby) * leaf;
        const float oz = (float)(coord[3 * nb + 2] - cbz) * leaf;
        const int j1 = pt_start[nb + 1];
        for (int j = pt_start[nb]; j < j1; ++j) {
            const float4 pj = pts[j];
            const float dx = (pi.x - pj.x) - ox;
            const float dy = (pi.y - pj.y) - oy;
            const float dz = (pi.z - pj.z) - oz;
            const float r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.f) continue;  // coincident point (self)
            const float rinv = rsqrtf(r2);
            const float r = r2 * rinv;
            float sn, cs;
            __sincosf(kw * r, &sn, &cs);
            float2 g = make_float2(cs * rinv, sn * rinv);
            if (FIELD) {
                // grad G = G (ik - 1/r) rhat / ... ; f = G (ik - 1/r) / r
                float2 f = cmul(g, make_float2(-rinv, kw));
                g = make_float2(f.x * rinv, f.y * rinv);
            }
#pragma unroll
            for (int c = 0; c < RC; ++c) {
                if (c < rc) {
                    const float2 qj = qs[(int64_t)j * R + r0 + c];
                    if (FIELD) {
                        const float2 p = cmul(g, qj);
                        acc[c][0].x = fmaf(p.x, dx, acc[c][0].x);
                        acc[c][0].y = fmaf(p.y, dx, acc[c][0].y);
                        acc[c][FIELD ? 1 : 0].x = fmaf(p.x, dy, acc[c][FIELD ? 1 : 0].x);
                        acc[c][FIELD ? 1 : 0].y = fmaf(p.y, dy, acc[c][FIELD ? 1 : 0].y);
                        acc[c][FIELD ? 2 : 0].x = fmaf(p.x, dz, acc[c][FIELD ? 2 : 0].x);
                        acc[c][FIELD ? 2 : 0].y = fmaf(p.y, dz, acc[c][FIELD ? 2 : 0].y);
                    } else {
                        acc[c][0] = cfma(g, qj, acc[c][0]);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < RC; ++c) {
        if (c < rc) {
            if (FIELD) {
                float2 *o = out + ((int64_t)i * R + r0 + c) * 3;
                o[0] = acc[c][0];
                o[1] = acc[c][FIELD ? 1 : 0];
                o[2] = acc[c][FIELD ? 2 : 0];
            } else {
                out[(int64_t)i * R + r0 + c] = acc[c][0];
            }
        }
    }
}

template <int RC>
static hipError_t p2p_rc(const float4 *pts, const int32_t *pt_leaf, const int32_t *pt_start,
                         const int32_t *near_start, const int32_t *near_idx,
                         const int32_t *coord, float leaf, float kw, const float2 *qs,
                         int64_t n, int R, int field, float2 *out, hipStream_t s)
{
    dim3 grid(nblocks(n, 128), (R + RC - 1) / RC);
    if (field)
        hipLaunchKernelGGL((k_p2p<RC, true>), grid, dim3(128), 0, s, pts, pt_leaf, pt_start,
                           near_start, near_idx, coord, leaf, kw, qs, n, R, out);
    else
        hipLaunchKernelGGL((k_p2p<RC, false>), grid, dim3(128), 0, s, pts, pt_leaf, pt_start,
                           near_start, near_idx, coord, leaf, kw, qs, n, R, out);
    return hipGetLastError();
}

hipError_t p2p(const float4 *pts, const int32_t *pt_leaf, const int32_t *pt_start,
               const int32_t *near_start, const int32_t *near_idx, const int32_t *coord,
               float leaf, float kw, const float2 *qs, int64_t n, int R, int field,
               float2 *out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    if (R == 1)
        return p2p_rc<1>(pts, pt_leaf, pt_start, near_start, near_idx, coord, leaf, kw, qs,
                         n, R, field, out, s);
    if (R == 2)
        return p2p_rc<2>(pts, pt_leaf, pt_start, near_start, near_idx, coord, leaf, kw, qs,
                         n, R, field, out, s);
    return p2p_rc<4>(pts, pt_leaf, pt_start, near_start, near_idx, coord, leaf, kw, qs, n,
                     R, field, out, s);
}

// ------------------------------------------------------------------- C2M --
// One workgroup per leaf box; threads over samples; the box's points and
// charges are staged in LDS in chunks.
template <int RC>
__global__ void __launch_bounds__(256)
k_c2m(const float4 *__restrict__ pts, const int32_t *__restrict__ pt_start,
      const float4 *__restrict__ khat_w, int64_t K, float kw,
      const float2 *__restrict__ qs, int R, float2 *__restrict__ S)
{
    __shared__ float4 sp[256];
    __shared__ float2 sq[256 * RC];
    const int64_t b = blockIdx.x;
    const int r0 = blockIdx.y * RC;
    const int rc = min(RC, R - r0);
    const int p0 = pt_start[b], p1 = pt_start[b + 1];
    for (int64_t kb = 0; kb < K; kb += blockDim.x) {
        const int64_t k = kb + threadIdx.x;
        const bool valid = k < K;
        const float4 kh = valid ? khat_w[k] : make_float4(0.f, 0.f, 0.f, 0.f);
        float2 acc[RC];
#pragma unroll
        for (int c = 0; c < RC; ++c) acc[c] = make_float2(0.f, 0.f);
        for (int j0 = p0; j0 < p1; j0 += 256) {
            const int nj = min(256, p1 - j0);
            __syncthreads();
            if ((int)threadIdx.x < nj) {
                sp[threadIdx.x] = pts[j0 + threadIdx.x];
#pragma unroll
                for (int c = 0; c < RC; ++c)
                    sq[threadIdx.x * RC + c] =
                        c < rc ? qs[(int64_t)(j0 + threadIdx.x) * R + r0 + c] : make_float2(0.f, 0.f);
            }
            __syncthreads();
            for (int j = 0; j < nj; ++j) {
                const float4 d = sp[j];
                const float ph = -kw * (kh.x * d.x + kh.y * d.y + kh.z * d.z);
                float sn, cs;
                __sincosf(ph, &sn, &cs);
                const float2 e = make_float2(cs, sn);
#pragma unroll
                for (int c = 0; c < RC; ++c) acc[c] = cfma(sq[j * RC + c], e, acc[c]);
            }
        }
        if (valid) {
#pragma unroll
            for (int c = 0; c < RC; ++c)
                if (c < rc) S[(b * R + r0 + c) * K + k] = acc[c];
        }
    }
}

hipError_t c2m(const float4 *pts, const int32_t *pt_start, int64_t nleaf,
               const float4 *khat_w, int64_t K, float kw, const float2 *qs, int R,
               float2 *S, hipStream_t s)
{
    if (nleaf == 0) return hipSuccess;
    if (R == 1) {
        hipLaunchKernelGGL(k_c2m<1>, dim3((unsigned)nleaf, 1), dim3(256), 0, s, pts, pt_start,
                           khat_w, K, kw, qs, R, S);
    } else {
        hipLaunchKernelGGL(k_c2m<4>, dim3((unsigned)nleaf, (R + 3) / 4), dim3(256), 0, s, pts,
                           pt_start, khat_w, K, kw, qs, R, S);
    }
    return hipGetLastError();
}

// ------------------------------------------------- interpolation stages --
__global__ void k_dft_rows(const float2 *__restrict__ X, int64_t rows, int nin,
                           const float *__restrict__ F, int M, float2 *__restrict__ out)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows * M) return;
    const int64_t row = idx / M;
    const int col = (int)(idx - row * M);
    const float2 *x = X + row * nin;
    float2 acc = make_float2(0.f, 0.f);
    for (int j = 0; j < nin; ++j) {
        const float f = F[j * M + col];
        const float2 v = x[j];
        acc.x = fmaf(v.x, f, acc.x);
        acc.y = fmaf(v.y, f, acc.y);
    }
    out[idx] = acc;
}

hipError_t dft_rows(const float2 *X, int64_t rows, int nin, const float *F, int M,
                    float2 *out, hipStream_t s)
{
    if (rows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dft_rows, dim3(nblocks(rows * M, 256)), dim3(256), 0, s, X, rows,
                       nin, F, M, out);
    return hipGetLastError();
}

__global__ void k_anterp_s1(const float2 *__restrict__ Lp, const int32_t *__restrict__ parent,
                            const uint8_t *__restrict__ oct, int64_t nchild, int R, int nthp,
                            int nphp, const float2 *__restrict__ shift,
                            const float *__restrict__ F, int M, float2 *__restrict__ out)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t rows = nchild * R * nthp;
    if (idx >= rows * M) return;
    const int64_t row = idx / M;
    const int col = (int)(idx - row * M);
    const int it = (int)(row % nthp);
    const int64_t cr = row / nthp;
    const int r = (int)(cr % R);
    const int64_t c = cr / R;
    const int64_t Kp = (int64_t)nthp * nphp;
    const float2 *x = Lp + ((int64_t)parent[c] * R + r) * Kp + (int64_t)it * nphp;
    const float2 *sh = shift + (int64_t)oct[c] * Kp + (int64_t)it * nphp;
    float2 acc = make_float2(0.f, 0.f);
    for (int j = 0; j < nphp; ++j) {
        // exp(+ik khat.(c_c - c_p)) = conj(shift)
        const float2 v = cfma_conj(sh[j], x[j], make_float2(0.f, 0.f));
        const float f = F[j * M + col];
        acc.x = fmaf(v.x, f, acc.x);
        acc.y = fmaf(v.y, f, acc.y);
    }
    out[idx] = acc;
}

hipError_t anterp_s1(const float2 *Lp, const int32_t *parent, const uint8_t *oct,
                     int64_t nchild, int R, int nthp, int nphp, const float2 *shift,
                     const float *F, int M, float2 *out, hipStream_t s)
{
    const int64_t total = nchild * R * nthp * M;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_anterp_s1, dim3(nblocks(total, 256)), dim3(256), 0, s, Lp, parent,
                       oct, nchild, R, nthp, nphp, shift, F, M, out);
    return hipGetLastError();
}

__global__ void k_theta_map(const float2 *__restrict__ Xh, int64_t BR, int nin, int M,
                            const float *__restrict__ maps, int nout,
                            float2 *__restrict__ Yh)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= BR * nout * M) return;
    const int col = (int)(idx % M);
    const int io = (int)((idx / M) % nout);
    const int64_t br = idx / ((int64_t)M * nout);
    const int m = (col + 1) >> 1;
    const float *a = maps + ((int64_t)m * nout + io) * nin;
    const float2 *x = Xh + br * nin * M + col;
    float2 acc = make_float2(0.f, 0.f);
    for (int i = 0; i < nin; ++i) {
        const float f = a[i];
        const float2 v = x[(int64_t)i * M];
        acc.x = fmaf(v.x, f, acc.x);
        acc.y = fmaf(v.y, f, acc.y);
    }
    Yh[idx] = acc;
}

hipError_t theta_map(const float2 *Xh, int64_t BR, int nin, int M, const float *maps,
                     int nout, float2 *Yh, hipStream_t s)
{
    const int64_t total = BR * nout * M;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_theta_map, dim3(nblocks(total, 256)), dim3(256), 0, s, Xh, BR, nin,
                       M, maps, nout, Yh);
    return hipGetLastError();
}

__global__ void k_interp_s3(int64_t nboxp, int R, int nthp, int nphp, int M,
                            const int32_t *__restrict__ child_start,
                            const uint8_t *__restrict__ child_oct,
                            const float2 *__restrict__ Yh, const float *__restrict__ G,
                            const float2 *__restrict__ shift, float2 *__restrict__ Sp)
{
    const int64_t Kp = (int64_t)nthp * nphp;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nboxp * R * Kp) return;
    const int64_t kp = idx % Kp;
    const int64_t br = idx / Kp;
    const int r = (int)(br % R);
    const int64_t p = br / R;
    const int it = (int)(kp / nphp);
    const int jp = (int)(kp - (int64_t)it * nphp);
    float2 acc = make_float2(0.f, 0.f);
    for (int c = child_start[p]; c < child_start[p + 1]; ++c) {
        const float2 *y = Yh + (((int64_t)c * R + r) * nthp + it) * M;
        float2 v = make_float2(0.f, 0.f);
        for (int col = 0; col < M; ++col) {
            const float g = G[col * nphp + jp];
            v.x = fmaf(y[col].x, g, v.x);
            v.y = fmaf(y[col].y, g, v.y);
        }
        acc = cfma(shift[(int64_t)child_oct[c] * Kp + kp], v, acc);
    }
    Sp[idx] = acc;
}

hipError_t interp_s3(int64_t nboxp, int R, int nthp, int nphp, int M,
                     const int32_t *child_start, const uint8_t *child_oct, const float2 *Yh,
                     const float *G, const float2 *shift, float2 *Sp, hipStream_t s)
{
    const int64_t total = nboxp * R * nthp * nphp;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_interp_s3, dim3(nblocks(total, 256)), dim3(256), 0, s, nboxp, R,
                       nthp, nphp, M, child_start, child_oct, Yh, G, shift, Sp);
    return hipGetLastError();
}

__global__ void k_anterp_s3(int64_t nboxc, int R, int nthc, int nphc, int M,
                            const float2 *__restrict__ Yh, const float *__restrict__ G,
                            float2 *__restrict__ Lc)
{
    const int64_t Kc = (int64_t)nthc * nphc;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nboxc * R * Kc) return;
    const int64_t kc = idx % Kc;
    const int64_t br = idx / Kc;
    const int it = (int)(kc / nphc);
    const int jc = (int)(kc - (int64_t)it * nphc);
    const float2 *y = Yh + (br * nthc + it) * M;
    float2 v = Lc[idx];
    for (int col = 0; col < M; ++col) {
        const float g = G[col * nphc + jc];
        v.x = fmaf(y[col].x, g, v.x);
        v.y = fmaf(y[col].y, g, v.y);
    }
    Lc[idx] = v;
}

hipError_t anterp_s3(int64_t nboxc, int R, int nthc, int nphc, int M, const float2 *Yh,
                     const float *G, float2 *Lc, hipStream_t s)
{
    const int64_t total = nboxc * R * nthc * nphc;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_anterp_s3, dim3(nblocks(total, 256)), dim3(256), 0, s, nboxc, R,
                       nthc, nphc, M, Yh, G, Lc);
    return hipGetLastError();
}

// ------------------------------------------------------------------- M2L --
template <int RC>
__global__ void k_m2l(int64_t nbox, int64_t K, const int32_t *__restrict__ far_start,
                      const int32_t *__restrict__ far_src,
                      const int16_t *__restrict__ far_type, const float2 *__restrict__ T,
                      const float2 *__restrict__ S, int R, float2 *__restrict__ Lout)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nbox * K) return;
    const int64_t b = idx / K;
    const int64_t k = idx - b * K;
    const int r0 = blockIdx.y * RC;
    const int rc = min(RC, R - r0);
    float2 acc[RC];
#pragma unroll
    for (int c = 0; c < RC; ++c) acc[c] = make_float2(0.f, 0.f);
    for (int e = far_start[b]; e < far_start[b + 1]; ++e) {
        const int64_t src = far_src[e];
        const float2 t = T[(int64_t)far_type[e] * K + k];
#pragma unroll
        for (int c = 0; c < RC; ++c)
            if (c < rc) acc[c] = cfma(t, S[(src * R + r0 + c) * K + k], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < RC; ++c)
        if (c < rc) Lout[(b * R + r0 + c) * K + k] = acc[c];
}

hipError_t m2l(int64_t nbox, int64_t K, const int32_t *far_start, const int32_t *far_src,
               const int16_t *far_type, const float2 *T, const float2 *S, int R,
               float2 *Lout, hipStream_t s)
{
    if (nbox * K == 0) return hipSuccess;
    if (R == 1)
        hipLaunchKernelGGL(k_m2l<1>, dim3(nblocks(nbox * K, 256), 1), dim3(256), 0, s, nbox, K,
                           far_start, far_src, far_type, T, S, R, Lout);
    else
        hipLaunchKernelGGL(k_m2l<4>, dim3(nblocks(nbox * K, 256), (R + 3) / 4), dim3(256), 0,
                           s, nbox, K, far_start, far_src, far_type, T, S, R, Lout);
    return hipGetLastError();
}

// ------------------------------------------------------ L2O + scatter --
template <typename Tout, bool FIELD>
__global__ void k_l2o_scatter(const float4 *__restrict__ pts,
                              const int32_t *__restrict__ pt_leaf,
                              const int32_t *__restrict__ perm,
                              const float4 *__restrict__ khat_w, int64_t K, float kw,
                              const float2 *__restrict__ L, const float2 *__restrict__ near,
                              int64_t n, int R, int far, int conj_out, Tout *__restrict__ out)
{
    constexpr int NA = FIELD ? 3 : 1;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * R) return;
    const int64_t s = idx / R;
    const int r = (int)(idx - s * R);
    float2 acc[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) acc[a] = make_float2(0.f, 0.f);
    if (far) {
        const float4 d = pts[s];
        const float2 *Lb = L + ((int64_t)pt_leaf[s] * R + r) * K;
        for (int64_t k = 0; k < K; ++k) {
            const float4 kh = khat_w[k];
            float sn, cs;
            __sincosf(kw * (kh.x * d.x + kh.y * d.y + kh.z * d.z), &sn, &cs);
            const float2 e = make_float2(cs * kh.w, sn * kh.w);
            const float2 v = cmul(e, Lb[k]);
            if (FIELD) {
                acc[0].x = fmaf(v.x, kh.x, acc[0].x);
                acc[0].y = fmaf(v.y, kh.x, acc[0].y);
                acc[FIELD ? 1 : 0].x = fmaf(v.x, kh.y, acc[FIELD ? 1 : 0].x);
                acc[FIELD ? 1 : 0].y = fmaf(v.y, kh.y, acc[FIELD ? 1 : 0].y);
                acc[FIELD ? 2 : 0].x = fmaf(v.x, kh.z, acc[FIELD ? 2 : 0].x);
                acc[FIELD ? 2 : 0].y = fmaf(v.y, kh.z, acc[FIELD ? 2 : 0].y);
            } else {
                acc[0].x += v.x;
                acc[0].y += v.y;
            }
        }
        // potential: (i kw / 4pi) acc;  gradient: (i kw)^2 / 4pi = -kw^2/4pi
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            if (FIELD) {
                const float sc = -kw * kw * kInv4Pi;
                acc[a] = make_float2(sc * acc[a].x, sc * acc[a].y);
            } else {
                const float sc = kw * kInv4Pi;
                acc[a] = make_float2(-sc * acc[a].y, sc * acc[a].x);
            }
        }
    }
    const int64_t o = (int64_t)perm[s] * R + r;
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        float2 v = near[idx * NA + a];
        v.x += acc[a].x;
        v.y += acc[a].y;
        if (conj_out) v.y = -v.y;
        out[o * NA + a].x = v.x;
        out[o * NA + a].y = v.y;
    }
}

hipError_t l2o_scatter(const float4 *pts, const int32_t *pt_leaf, const int32_t *perm,
                       const float4 *khat_w, int64_t K, float kw, const float2 *L,
                       const float2 *near, int64_t n, int R, int field, int far, int conj_out,
                       int dtype, void *out, hipStream_t s)
{
    if (n * R == 0) return hipSuccess;
    dim3 grid(nblocks(n * R, 256)), block(256);
#define L2O_LAUNCH(T, F)                                                                 \
    hipLaunchKernelGGL((k_l2o_scatter<T, F>), grid, block, 0, s, pts, pt_leaf, perm, khat_w, \
                       K, kw, L, near, n, R, far, conj_out, (T *)out)
    if (dtype == 0) {
        if (field) L2O_LAUNCH(float2, true); else L2O_LAUNCH(float2, false);
    } else {
        if (field) L2O_LAUNCH(double2, true); else L2O_LAUNCH(double2, false);
    }
#undef L2O_LAUNCH
    return hipGetLastError();
}

}  // namespace dev
}  // namespace mlfma
