// HIP kernels of the MLFMA matvec for gfx950.
//
// Layouts (all in HBM, sorted = Morton order of the points):
//   pts      [n] float4 (x, y, z offsets from the point's leaf-box centre, 0)
//   qs, near [n][R] complex64
//   spectra  [nbox][R][K] complex64, samples [theta][phi] (phi fastest)
//   tables   FP32 copies of the FP64 host precompute
#include <hip/hip_runtime.h>

#include <algorithm>

#include "devmath.h"
#include "kernels.h"

namespace mlfma {
namespace dev {

static constexpr float kInv4Pi = 0.0795774715459476679f;  // 1/(4 pi)

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
// One single-wave workgroup per work item (a target leaf, or a chunk of 64
// of its points).  The near sources are staged in LDS in batches of 256,
// their positions moved into the target leaf's frame (leaf-local offset +
// exact integer leaf offset x leaf side, which keeps FP32 accuracy for close
// pairs far from the origin).  With nt targets the lanes form G = 64/T groups
// (T = nt rounded up to a power of two): lane (g, t) takes target t and every
// G-th staged source; the G partial sums are added with cross-lane shuffles.
template <int RC, bool FIELD>
__global__ void __launch_bounds__(64)
k_p2p(const int2 *__restrict__ items, const float4 *__restrict__ pts,
      const int32_t *__restrict__ pt_start, const int32_t *__restrict__ near_start,
      const int32_t *__restrict__ near_idx, const int32_t *__restrict__ coord, float leaf,
      float kw, const float2 *__restrict__ qs, int R, float2 *__restrict__ out)
{
    constexpr int NA = FIELD ? 3 : 1;
    constexpr int CH = 256;
    __shared__ float4 sp[CH];
    __shared__ float2 sq[CH * RC];
    const int lane = threadIdx.x;
    const int2 it = items[blockIdx.x];
    const int b = it.x;
    const int p0 = pt_start[b];
    const int nt = min(64, pt_start[b + 1] - p0 - it.y);
    int Tp = 1;
    while (Tp < nt) Tp <<= 1;
    const int G = 64 / Tp;
    const int t = lane & (Tp - 1), g = lane / Tp;
    const bool tv = t < nt;
    const int i = p0 + it.y + (tv ? t : 0);
    const int r0 = blockIdx.y * RC;
    const int rc = min(RC, R - r0);
    const float4 pi = pts[i];
    const int cbx = coord[3 * b], cby = coord[3 * b + 1], cbz = coord[3 * b + 2];
    float2 acc[RC][NA];
#pragma unroll
    for (int c = 0; c < RC; ++c)
#pragma unroll
        for (int a = 0; a < NA; ++a) acc[c][a] = make_float2(0.f, 0.f);

    auto process = [&](int n) {
        __syncthreads();
        for (int x = g; x < n; x += G) {
            const float4 sj = sp[x];
            const float dx = pi.x - sj.x, dy = pi.y - sj.y, dz = pi.z - sj.z;
            const float r2 = dx * dx + dy * dy + dz * dz;
            // coincident point (self): r2 == 0 contributes nothing
            const float rinv = r2 > 0.f ? rsqrtf(r2) : 0.f;
            float sn, cs;
            __sincosf(kw * (r2 * rinv), &sn, &cs);
            float2 gk = make_float2(cs * rinv, sn * rinv);
            if (FIELD) {
                // grad G = G (ik - 1/r) r_vec / r
                const float2 f = cmul(gk, make_float2(-rinv, kw));
                gk = make_float2(f.x * rinv, f.y * rinv);
            }
#pragma unroll
            for (int c = 0; c < RC; ++c) {
                const float2 qj = sq[x * RC + c];
                if (FIELD) {
                    const float2 pq = cmul(gk, qj);
                    const float d3[3] = {dx, dy, dz};
#pragma unroll
                    for (int a = 0; a < NA; ++a) {
                        acc[c][a].x = fmaf(pq.x, d3[a], acc[c][a].x);
                        acc[c][a].y = fmaf(pq.y, d3[a], acc[c][a].y);
                    }
                } else {
                    acc[c][0] = cfma(gk, qj, acc[c][0]);
                }
            }
        }
        __syncthreads();
    };

    int fill = 0;
    const int e1 = near_start[b + 1];
    for (int e = near_start[b]; e < e1; ++e) {
        const int nb = near_idx[e];
        const float ox = (float)(coord[3 * nb] - cbx) * leaf;
        const float oy = (float)(coord[3 * nb + 1] - cby) * leaf;
        const float oz = (float)(coord[3 * nb + 2] - cbz) * leaf;
        const int j1 = pt_start[nb + 1];
        for (int j = pt_start[nb]; j < j1; j += 64) {
            const int cnt = min(64, j1 - j);
            if (fill + cnt > CH) {
                process(fill);
                fill = 0;
            }
            if (lane < cnt) {
                const float4 pj = pts[j + lane];
                sp[fill + lane] = make_float4(pj.x + ox, pj.y + oy, pj.z + oz, 0.f);
#pragma unroll
                for (int c = 0; c < RC; ++c)
                    sq[(fill + lane) * RC + c] =
                        c < rc ? qs[(int64_t)(j + lane) * R + r0 + c] : make_float2(0.f, 0.f);
            }
            fill += cnt;
        }
    }
    process(fill);
    // add the G partial sums of each target (lanes t, t+T, t+2T, ...)
    for (int sft = Tp; sft < 64; sft <<= 1) {
#pragma unroll
        for (int c = 0; c < RC; ++c)
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                acc[c][a].x += __shfl_xor(acc[c][a].x, sft, 64);
                acc[c][a].y += __shfl_xor(acc[c][a].y, sft, 64);
            }
    }
    if (g == 0 && tv) {
#pragma unroll
        for (int c = 0; c < RC; ++c)
            if (c < rc)
#pragma unroll
                for (int a = 0; a < NA; ++a)
                    out[((int64_t)i * R + r0 + c) * NA + a] = acc[c][a];
    }
}

template <int RC>
static hipError_t p2p_rc(const int2 *items, int64_t nitems, const float4 *pts,
                         const int32_t *pt_start, const int32_t *near_start,
                         const int32_t *near_idx, const int32_t *coord, float leaf, float kw,
                         const float2 *qs, int R, int field, float2 *out, hipStream_t s)
{
    dim3 grid((unsigned)nitems, (R + RC - 1) / RC);
    if (field)
        hipLaunchKernelGGL((k_p2p<RC, true>), grid, dim3(64), 0, s, items, pts, pt_start,
                           near_start, near_idx, coord, leaf, kw, qs, R, out);
    else
        hipLaunchKernelGGL((k_p2p<RC, false>), grid, dim3(64), 0, s, items, pts, pt_start,
                           near_start, near_idx, coord, leaf, kw, qs, R, out);
    return hipGetLastError();
}

hipError_t p2p(const int2 *items, int64_t nitems, const float4 *pts, const int32_t *pt_start,
               const int32_t *near_start, const int32_t *near_idx, const int32_t *coord,
               float leaf, float kw, const float2 *qs, int R, int field, float2 *out,
               hipStream_t s)
{
    if (nitems == 0) return hipSuccess;
#define P2P_RC(RCV) \
    return p2p_rc<RCV>(items, nitems, pts, pt_start, near_start, near_idx, coord, leaf, kw, qs, \
                       R, field, out, s)
    if (R == 1) P2P_RC(1);
    if (R == 2) P2P_RC(2);
    if (R <= 4) P2P_RC(4);
    if (R <= 8 || field) P2P_RC(8);
    P2P_RC(16);
#undef P2P_RC
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
    } else if (R <= 4) {
        hipLaunchKernelGGL(k_c2m<4>, dim3((unsigned)nleaf, 1), dim3(256), 0, s, pts,
                           pt_start, khat_w, K, kw, qs, R, S);
    } else {
        hipLaunchKernelGGL(k_c2m<16>, dim3((unsigned)nleaf, (R + 15) / 16), dim3(256), 0, s, pts,
                           pt_start, khat_w, K, kw, qs, R, S);
    }
    return hipGetLastError();
}


// ------------------------------------------- position-gradient combine --
template <typename Tc, typename Tr>
__global__ void k_posgrad(const Tc *__restrict__ q, const Tc *__restrict__ g,
                          const float2 *__restrict__ Fq, const float2 *__restrict__ Fg, int64_t n,
                          int R, Tr *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float acc[3] = {0.f, 0.f, 0.f};
    for (int r = 0; r < R; ++r) {
        const Tc gv = g[i * R + r], qv = q[i * R + r];
        const float gx = (float)gv.x, gy = (float)gv.y, qx = (float)qv.x, qy = (float)qv.y;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float2 f1 = Fq[(i * R + r) * 3 + a], f2 = Fg[(i * R + r) * 3 + a];
            // Re(conj(g) f1) + Re(q f2)
            acc[a] += gx * f1.x + gy * f1.y + qx * f2.x - qy * f2.y;
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) out[i * 3 + a] = (Tr)acc[a];
}

hipError_t position_grad_combine(const void *q, const void *g, int dtype, const float2 *Fq,
                                 const float2 *Fg, int64_t n, int R, void *out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    dim3 grid(nblocks(n, 256)), block(256);
    if (dtype == 0)
        hipLaunchKernelGGL((k_posgrad<float2, float>), grid, block, 0, s, (const float2 *)q,
                           (const float2 *)g, Fq, Fg, n, R, (float *)out);
    else
        hipLaunchKernelGGL((k_posgrad<double2, double>), grid, block, 0, s, (const double2 *)q,
                           (const double2 *)g, Fq, Fg, n, R, (double *)out);
    return hipGetLastError();
}

// ------------------------------------------------------ L2O + scatter --
template <typename Tout, bool FIELD, int RC>
__global__ void k_l2o_scatter(const float4 *__restrict__ pts,
                              const int32_t *__restrict__ pt_leaf,
                              const int32_t *__restrict__ perm,
                              const float4 *__restrict__ khat_w, int64_t K, float kw,
                              const float2 *__restrict__ L, const float2 *__restrict__ near,
                              int64_t n, int R, int far, int conj_out, Tout *__restrict__ out)
{
    // one thread per (point, chunk of RC right-hand sides): the plane-wave
    // factor of each sample is computed once and used for the whole chunk
    constexpr int NA = FIELD ? 3 : 1;
    const int nch = (R + RC - 1) / RC;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * nch) return;
    const int64_t s = idx / nch;
    const int r0 = (int)(idx - s * nch) * RC;
    const int rc = min(RC, R - r0);
    float2 acc[RC][NA];
#pragma unroll
    for (int c = 0; c < RC; ++c)
#pragma unroll
        for (int a = 0; a < NA; ++a) acc[c][a] = make_float2(0.f, 0.f);
    if (far) {
        const float4 d = pts[s];
        const float2 *Lb = L + ((int64_t)pt_leaf[s] * R + r0) * K;
        for (int64_t k = 0; k < K; ++k) {
            const float4 kh = khat_w[k];
            float sn, cs;
            __sincosf(kw * (kh.x * d.x + kh.y * d.y + kh.z * d.z), &sn, &cs);
            const float2 e = make_float2(cs * kh.w, sn * kh.w);
#pragma unroll
            for (int c = 0; c < RC; ++c) {
                if (c < rc) {
                    const float2 v = cmul(e, Lb[c * K + k]);
                    if (FIELD) {
                        const float kd[3] = {kh.x, kh.y, kh.z};
#pragma unroll
                        for (int a = 0; a < NA; ++a) {
                            acc[c][a].x = fmaf(v.x, kd[a], acc[c][a].x);
                            acc[c][a].y = fmaf(v.y, kd[a], acc[c][a].y);
                        }
                    } else {
                        acc[c][0].x += v.x;
                        acc[c][0].y += v.y;
                    }
                }
            }
        }
        // potential: (i kw / 4pi) acc;  gradient: (i kw)^2 / 4pi = -kw^2/4pi
#pragma unroll
        for (int c = 0; c < RC; ++c)
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                if (FIELD) {
                    const float sc = -kw * kw * kInv4Pi;
                    acc[c][a] = make_float2(sc * acc[c][a].x, sc * acc[c][a].y);
                } else {
                    const float sc = kw * kInv4Pi;
                    acc[c][a] = make_float2(-sc * acc[c][a].y, sc * acc[c][a].x);
                }
            }
    }
    const int64_t o = (int64_t)perm[s] * R;
#pragma unroll
    for (int c = 0; c < RC; ++c) {
        if (c < rc) {
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                float2 v = near[((s * R) + r0 + c) * NA + a];
                v.x += acc[c][a].x;
                v.y += acc[c][a].y;
                if (conj_out) v.y = -v.y;
                out[(o + r0 + c) * NA + a].x = v.x;
                out[(o + r0 + c) * NA + a].y = v.y;
            }
        }
    }
}

template <int RC>
static hipError_t l2o_rc(const float4 *pts, const int32_t *pt_leaf, const int32_t *perm,
                         const float4 *khat_w, int64_t K, float kw, const float2 *L,
                         const float2 *near, int64_t n, int R, int field, int far, int conj_out,
                         int dtype, void *out, hipStream_t s)
{
    const int64_t total = n * ((R + RC - 1) / RC);
    dim3 grid(nblocks(total, 256)), block(256);
#define L2O_LAUNCH(T, F)                                                                       \
    hipLaunchKernelGGL((k_l2o_scatter<T, F, RC>), grid, block, 0, s, pts, pt_leaf, perm, khat_w, \
                       K, kw, L, near, n, R, far, conj_out, (T *)out)
    if (dtype == 0) {
        if (field) L2O_LAUNCH(float2, true); else L2O_LAUNCH(float2, false);
    } else {
        if (field) L2O_LAUNCH(double2, true); else L2O_LAUNCH(double2, false);
    }
#undef L2O_LAUNCH
    return hipGetLastError();
}

hipError_t l2o_scatter(const float4 *pts, const int32_t *pt_leaf, const int32_t *perm,
                       const float4 *khat_w, int64_t K, float kw, const float2 *L,
                       const float2 *near, int64_t n, int R, int field, int far, int conj_out,
                       int dtype, void *out, hipStream_t s)
{
    if (n * R == 0) return hipSuccess;
    if (R == 1)
        return l2o_rc<1>(pts, pt_leaf, perm, khat_w, K, kw, L, near, n, R, field, far, conj_out,
                         dtype, out, s);
    if (R <= 4 || field)
        return l2o_rc<4>(pts, pt_leaf, perm, khat_w, K, kw, L, near, n, R, field, far, conj_out,
                         dtype, out, s);
    return l2o_rc<16>(pts, pt_leaf, perm, khat_w, K, kw, L, near, n, R, field, far, conj_out,
                      dtype, out, s);
}

}  // namespace dev
}  // namespace mlfma
