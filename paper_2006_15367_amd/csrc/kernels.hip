// HIP kernels of the MLFMA matvec for gfx950.
//
// Layouts (all in HBM, sorted = Morton order of the points):
//   pts      [n] float4 (x, y, z offsets from the point's leaf-box centre, 0)
//   qs, near [n][R] complex64
//   spectra  [nbox][R][K] complex64, samples [theta][phi] (phi fastest)
//   tables   FP32 copies of the FP64 host precompute
#include <hip/hip_runtime.h>

#include <algorithm>

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

// ------------------------------------------------------------------- M2L --
// Copy T[t][k0 .. k0+KC) (zero beyond K) for all t < ntypes into Ts[t][KC]
// with 8 loads in flight per thread before the LDS stores.
template <int KC>
__device__ __forceinline__ void stage_t_slice(float2 *Ts, const float2 *__restrict__ T,
                                              int ntypes, int64_t K, int64_t k0)
{
    const int total = ntypes * KC;
    for (int base = threadIdx.x; base < total; base += 8 * blockDim.x) {
        float2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = base + u * blockDim.x;
            const int t = idx / KC, kk = idx % KC;
            v[u] = (idx < total && k0 + kk < K) ? T[(int64_t)t * K + k0 + kk] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = base + u * blockDim.x;
            if (idx < total) Ts[idx] = v[u];
        }
    }
}

// One wave per (observer box, chunk of 64 samples): the far list of the box
// is wave-uniform (scalar loads), lanes run over samples, each translation
// operator and source spectrum is read once per wave and reused for RC
// right-hand sides.  Workgroups are renumbered so that each of the 8 XCDs
// (which take workgroups round-robin) gets a contiguous, Morton-ordered
// range of observers and keeps their shared sources in its own L2.
__device__ __forceinline__ int64_t xcd_contiguous(int64_t bid, int64_t nb)
{
    const int64_t q = nb / 8, rem = nb % 8;
    const int64_t x = bid % 8, i = bid / 8;
    return x * q + (x < rem ? x : rem) + i;
}

template <int RC>
__global__ void __launch_bounds__(256)
k_m2l(int64_t nbox, int64_t K, const int32_t *__restrict__ far_start,
      const int32_t *__restrict__ far_src, const int16_t *__restrict__ far_type,
      const float2 *__restrict__ T, const float2 *__restrict__ S, int R,
      float2 *__restrict__ Lout)
{
    const int64_t nkc = (K + 63) / 64;
    const int64_t bid = xcd_contiguous(blockIdx.x, gridDim.x);
    const int64_t wave = bid * 4 + (threadIdx.x >> 6);
    if (wave >= nbox * nkc) return;
    const int lane = threadIdx.x & 63;
    const int64_t b = wave / nkc;
    const int64_t k = (wave - b * nkc) * 64 + lane;
    const bool valid = k < K;
    const int64_t kk = valid ? k : K - 1;
    const int r0 = blockIdx.y * RC;
    const int rc = min(RC, R - r0);
    float2 acc[RC];
#pragma unroll
    for (int c = 0; c < RC; ++c) acc[c] = make_float2(0.f, 0.f);
    const int e0 = __builtin_amdgcn_readfirstlane(far_start[b]);
    const int e1 = __builtin_amdgcn_readfirstlane(far_start[b + 1]);
    for (int eb = e0; eb < e1; eb += 8) {
        int src[8], typ[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = eb + u < e1 ? eb + u : e0;
            src[u] = __builtin_amdgcn_readfirstlane(far_src[e]);
            typ[u] = __builtin_amdgcn_readfirstlane((int)far_type[e]);
        }
        float2 t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            t[u] = eb + u < e1 ? T[(int64_t)typ[u] * K + kk] : make_float2(0.f, 0.f);
#pragma unroll
        for (int c = 0; c < RC; ++c) {
            if (c < rc) {
                float2 sv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) sv[u] = S[((int64_t)src[u] * R + r0 + c) * K + kk];
#pragma unroll
                for (int u = 0; u < 8; ++u) acc[c] = cfma(t[u], sv[u], acc[c]);
            }
        }
    }
    if (valid) {
#pragma unroll
        for (int c = 0; c < RC; ++c)
            if (c < rc) Lout[(b * R + r0 + c) * K + k] = acc[c];
    }
}

// Sibling-group M2L.  The far list of a box o (child of P) is the set of
// children s of the neighbours Q of P with Chebyshev distance >= 2, so the
// children of one parent share every source.  One wave takes one parent:
// it walks the children of P's neighbours once, loads each source spectrum
// once (lanes 0-31 and 32-63 take alternate sources) and applies it to all
// siblings in registers.  The translation operators of the level for a chunk
// of 32 samples sit in LDS (offset code -> operator index map alongside), so
// each complex multiply-add reads 8 bytes of LDS and, per sibling sharing the
// source, a fraction of 8 bytes of L2.
//   code(o, s) = base[o] - base[s] + 171,  base = 49 cx + 7 cy + cz,
//   equal to (dx+3)*49 + (dy+3)*7 + (dz+3) for |d| <= 3 per axis.
template <int RC, int KC>
__global__ void __launch_bounds__(1024)
k_m2l_sg(int64_t nparent, int64_t K, int ntypes, const int32_t *__restrict__ child_start,
         const int32_t *__restrict__ nbr_start, const int32_t *__restrict__ nbr_idx,
         const int32_t *__restrict__ base, const int16_t *__restrict__ typemap,
         const float2 *__restrict__ T, const float2 *__restrict__ S, int R, int ppb,
         float2 *__restrict__ Lout)
{
    constexpr int NS = 64 / KC;                        // interleaved source streams
    extern __shared__ float2 lds[];
    float2 *Ts = lds;                                  // [ntypes][KC]
    int16_t *map = (int16_t *)(lds + (size_t)ntypes * KC);  // [343]
    const int64_t k0 = (int64_t)blockIdx.x * KC;
    stage_t_slice<KC>(Ts, T, ntypes, K, k0);
    for (int idx = threadIdx.x; idx < 343; idx += blockDim.x) map[idx] = typemap[idx];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kl = lane % KC, part = lane / KC;
    const int64_t k = k0 + kl;
    const bool valid = k < K;
    const int64_t kk = valid ? k : K - 1;
    const int r0 = blockIdx.z * RC;
    const int rc = min(RC, R - r0);
    const int64_t pend = min(nparent, (int64_t)(blockIdx.y + 1) * ppb);
    for (int64_t P = (int64_t)blockIdx.y * ppb + wave; P < pend; P += 16) {
        const int o0 = __builtin_amdgcn_readfirstlane(child_start[P]);
        const int no = __builtin_amdgcn_readfirstlane(child_start[P + 1]) - o0;
        int bo[8];
#pragma unroll
        for (int i = 0; i < 8; ++i)
            bo[i] = i < no ? __builtin_amdgcn_readfirstlane(base[o0 + i]) + 171 : 0;
        float2 acc[8][RC];
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int c = 0; c < RC; ++c) acc[i][c] = make_float2(0.f, 0.f);
        const int e1 = __builtin_amdgcn_readfirstlane(nbr_start[P + 1]);
        for (int e = __builtin_amdgcn_readfirstlane(nbr_start[P]); e < e1; ++e) {
            const int Q = __builtin_amdgcn_readfirstlane(nbr_idx[e]);
            const int s1 = __builtin_amdgcn_readfirstlane(child_start[Q + 1]);
            for (int s = __builtin_amdgcn_readfirstlane(child_start[Q]) + part; s < s1; s += NS) {
                const int bs = base[s];
                float2 sv[RC];
#pragma unroll
                for (int c = 0; c < RC; ++c)
                    sv[c] = c < rc ? S[((int64_t)s * R + r0 + c) * K + kk] : make_float2(0.f, 0.f);
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    if (i < no) {
                        const int t = map[bo[i] - bs];
                        const float2 tv = t >= 0 ? Ts[t * KC + kl] : make_float2(0.f, 0.f);
#pragma unroll
                        for (int c = 0; c < RC; ++c) acc[i][c] = cfma(tv, sv[c], acc[i][c]);
                    }
                }
            }
        }
        // add the NS partial sums of each sample (lanes kl, kl+KC, ...)
        for (int off = KC; off < 64; off <<= 1) {
#pragma unroll
            for (int i = 0; i < 8; ++i)
#pragma unroll
                for (int c = 0; c < RC; ++c) {
                    acc[i][c].x += __shfl_xor(acc[i][c].x, off, 64);
                    acc[i][c].y += __shfl_xor(acc[i][c].y, off, 64);
                }
        }
        if (part == 0 && valid) {
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (i < no)
#pragma unroll
                    for (int c = 0; c < RC; ++c)
                        if (c < rc) Lout[((int64_t)(o0 + i) * R + r0 + c) * K + k] = acc[i][c];
        }
    }
}

hipError_t m2l_sg(int64_t nparent, int64_t K, int ntypes, const int32_t *child_start,
                  const int32_t *nbr_start, const int32_t *nbr_idx, const int32_t *base,
                  const int16_t *typemap, const float2 *T, const float2 *S, int R,
                  float2 *Lout, hipStream_t s)
{
    if (nparent == 0 || K == 0) return hipSuccess;
    const int ppb = 64;
    // 32 samples per wave when the operator slice fits in 64 KB, else 16
    const int KC = ((size_t)ntypes * 32 * sizeof(float2) + 343 * 2 <= 65536) ? 32 : 16;
    const size_t lds = (size_t)ntypes * KC * sizeof(float2) + 343 * sizeof(int16_t);
    const int RC = R == 1 ? 1 : 4;
    dim3 grid((unsigned)((K + KC - 1) / KC), (unsigned)((nparent + ppb - 1) / ppb),
              (unsigned)((R + RC - 1) / RC));
    dim3 block(1024);
#define M2L_SG(RCV, KCV)                                                                 \
    hipLaunchKernelGGL((k_m2l_sg<RCV, KCV>), grid, block, lds, s, nparent, K, ntypes,    \
                       child_start, nbr_start, nbr_idx, base, typemap, T, S, R, ppb, Lout)
    if (RC == 1) {
        if (KC == 32) M2L_SG(1, 32); else M2L_SG(1, 16);
    } else {
        if (KC == 32) M2L_SG(4, 32); else M2L_SG(4, 16);
    }
#undef M2L_SG
    return hipGetLastError();
}

// Per-observer M2L with the operator slice in LDS: a workgroup takes a chunk
// of KC samples and a range of observers; the level's operators for those
// samples are staged once in LDS; each wave walks one observer's far list
// with 64/KC interleaved lane streams (partial sums added by shuffles), so a
// complex multiply-add reads 8 bytes of L2 (the source) and 8 of LDS.
template <int RC, int KC>
__global__ void __launch_bounds__(1024)
k_m2l_lds(int64_t nbox, int64_t K, int ntypes, const int32_t *__restrict__ far_start,
          const int32_t *__restrict__ far_src, const int16_t *__restrict__ far_type,
          const float2 *__restrict__ T, const float2 *__restrict__ S, int R, int opb,
          float2 *__restrict__ Lout)
{
    constexpr int NS = 64 / KC;
    extern __shared__ float2 Ts[];  // [ntypes][KC]
    const int64_t k0 = (int64_t)blockIdx.x * KC;
    stage_t_slice<KC>(Ts, T, ntypes, K, k0);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kl = lane % KC, part = lane / KC;
    const int64_t k = k0 + kl;
    const bool valid = k < K;
    const int64_t kk = valid ? k : K - 1;
    const int r0 = blockIdx.z * RC;
    const int rc = min(RC, R - r0);
    const int64_t bend = min(nbox, (int64_t)(blockIdx.y + 1) * opb);
    for (int64_t b = (int64_t)blockIdx.y * opb + wave; b < bend; b += 16) {
        const int e0 = __builtin_amdgcn_readfirstlane(far_start[b]);
        const int e1 = __builtin_amdgcn_readfirstlane(far_start[b + 1]);
        float2 acc[RC];
#pragma unroll
        for (int c = 0; c < RC; ++c) acc[c] = make_float2(0.f, 0.f);
        // 8 far-list entries per lane stream in flight: indices first, then
        // the 8 source loads, then the multiply-adds
        for (int eb = e0 + part; eb < e1; eb += 8 * NS) {
            int src[8], typ[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = eb + u * NS;
                const bool ok = e < e1;
                src[u] = far_src[ok ? e : e0];
                typ[u] = ok ? (int)far_type[e] : -1;
            }
            float2 tv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                tv[u] = typ[u] >= 0 ? Ts[typ[u] * KC + kl] : make_float2(0.f, 0.f);
#pragma unroll
            for (int c = 0; c < RC; ++c) {
                if (c < rc) {
                    float2 sv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) sv[u] = S[((int64_t)src[u] * R + r0 + c) * K + kk];
#pragma unroll
                    for (int u = 0; u < 8; ++u) acc[c] = cfma(tv[u], sv[u], acc[c]);
                }
            }
        }
        for (int off = KC; off < 64; off <<= 1) {
#pragma unroll
            for (int c = 0; c < RC; ++c) {
                acc[c].x += __shfl_xor(acc[c].x, off, 64);
                acc[c].y += __shfl_xor(acc[c].y, off, 64);
            }
        }
        if (part == 0 && valid) {
#pragma unroll
            for (int c = 0; c < RC; ++c)
                if (c < rc) Lout[(b * R + r0 + c) * K + k] = acc[c];
        }
    }
}

hipError_t m2l_lds(int64_t nbox, int64_t K, int ntypes, const int32_t *far_start,
                   const int32_t *far_src, const int16_t *far_type, const float2 *T,
                   const float2 *S, int R, float2 *Lout, hipStream_t s)
{
    if (nbox == 0 || K == 0) return hipSuccess;
    const int opb = 64;
    const int KC = ((size_t)ntypes * 32 * sizeof(float2) <= 65536) ? 32 : 16;
    const size_t lds = (size_t)ntypes * KC * sizeof(float2);
    const int RC = R == 1 ? 1 : 4;
    dim3 grid((unsigned)((K + KC - 1) / KC), (unsigned)((nbox + opb - 1) / opb),
              (unsigned)((R + RC - 1) / RC));
    dim3 block(1024);
#define M2L_LDS(RCV, KCV)                                                                \
    hipLaunchKernelGGL((k_m2l_lds<RCV, KCV>), grid, block, lds, s, nbox, K, ntypes,      \
                       far_start, far_src, far_type, T, S, R, opb, Lout)
    if (RC == 1) {
        if (KC == 32) M2L_LDS(1, 32); else M2L_LDS(1, 16);
    } else {
        if (KC == 32) M2L_LDS(4, 32); else M2L_LDS(4, 16);
    }
#undef M2L_LDS
    return hipGetLastError();
}

// Sibling-group M2L with per-source records (variant 3).  One wave takes one
// parent P and 64 samples; the records of P list every source s (children
// of P's neighbours) that interacts with at least one child of P, with 8
// byte offsets into the LDS operator slice: slot i is the operator of
// (child i of P, s), or a zero row where the pair is near or child i does
// not exist.  Per source the wave issues one scalar record load, one vector
// load of the source spectrum and, per sibling, one LDS read and four FMAs:
// no per-pair branches, no per-pair scalar arithmetic.  The operators of
// the level for the 64 samples sit in LDS ((316 + 1) x 64 x 8 B <= 160 KB).
template <int RC, int NO>
__device__ __forceinline__ void m2l_rec_parent(const char *Tsb, int lane8, int e0, int e1,
                                               const int32_t *__restrict__ rec_src,
                                               const int32_t *__restrict__ rec_off,
                                               const float2 *__restrict__ S, int64_t K, int R,
                                               int r0, int rc, int64_t kk, float2 (&acc)[8][RC])
{
    constexpr int U = 4;  // records in flight per wave
    for (int eb = e0; eb < e1; eb += U) {
        float2 sv[U][RC];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = eb + u < e1 ? eb + u : e0;
            const int64_t s = __builtin_amdgcn_readfirstlane(rec_src[e]);
            const float2 *Sr = S + (s * R + r0) * K;
#pragma unroll
            for (int c = 0; c < RC; ++c)
                sv[u][c] = c < rc ? Sr[c * K + kk] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (eb + u < e1) {
                const int32_t *off = rec_off + 8 * (int64_t)(eb + u);
#pragma unroll
                for (int i = 0; i < NO; ++i) {
                    const float2 tv = *(const float2 *)(Tsb + (__builtin_amdgcn_readfirstlane(off[i]) + lane8));
#pragma unroll
                    for (int c = 0; c < RC; ++c) acc[i][c] = cfma(tv, sv[u][c], acc[i][c]);
                }
            }
        }
    }
}

template <int RC>
__global__ void __launch_bounds__(1024)
k_m2l_rec(int64_t nparent, int64_t K, int ntypes, const int32_t *__restrict__ child_start,
          const int32_t *__restrict__ rec_start, const int32_t *__restrict__ rec_src,
          const int32_t *__restrict__ rec_off, const float2 *__restrict__ T,
          const float2 *__restrict__ S, int R, int nkc, int64_t ppb, float2 *__restrict__ Lout)
{
    // workgroup b serves sample chunk b % nkc and the contiguous parent range
    // (b / nkc) * ppb ... + ppb; its 16 waves take those parents round-robin.
    // About one workgroup per CU, so the LDS staging of the operators is
    // amortised over many parents.
    extern __shared__ float2 Ts[];  // [ntypes + 1][64], row ntypes = 0
    const int kc = blockIdx.x % nkc;
    const int64_t k0 = (int64_t)kc * 64;
    stage_t_slice<64>(Ts, T, ntypes, K, k0);
    for (int idx = threadIdx.x; idx < 64; idx += blockDim.x)
        Ts[ntypes * 64 + idx] = make_float2(0.f, 0.f);
    __syncthreads();
    const char *Tsb = (const char *)Ts;
    const int lane = threadIdx.x & 63;
    const int lane8 = lane * 8;
    const int64_t k = k0 + lane;
    const bool valid = k < K;
    const int64_t kk = valid ? k : K - 1;
    const int r0 = blockIdx.z * RC;
    const int rc = min(RC, R - r0);
    const int64_t pbeg = (int64_t)(blockIdx.x / nkc) * ppb;
    const int64_t pend = min(nparent, pbeg + ppb);
    for (int64_t P = pbeg + (threadIdx.x >> 6); P < pend; P += 16) {
        const int o0 = __builtin_amdgcn_readfirstlane(child_start[P]);
        const int no = __builtin_amdgcn_readfirstlane(child_start[P + 1]) - o0;
        const int e0 = __builtin_amdgcn_readfirstlane(rec_start[P]);
        const int e1 = __builtin_amdgcn_readfirstlane(rec_start[P + 1]);
        float2 acc[8][RC];
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int c = 0; c < RC; ++c) acc[i][c] = make_float2(0.f, 0.f);
        switch (no) {
#define REC_CASE(N)                                                                          \
    case N:                                                                                  \
        m2l_rec_parent<RC, N>(Tsb, lane8, e0, e1, rec_src, rec_off, S, K, R, r0, rc, kk, acc); \
        break;
            REC_CASE(1) REC_CASE(2) REC_CASE(3) REC_CASE(4)
            REC_CASE(5) REC_CASE(6) REC_CASE(7) REC_CASE(8)
#undef REC_CASE
        default: break;
        }
        if (valid) {
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (i < no)
#pragma unroll
                    for (int c = 0; c < RC; ++c)
                        if (c < rc) Lout[((int64_t)(o0 + i) * R + r0 + c) * K + k] = acc[i][c];
        }
    }
}

hipError_t m2l_rec(int64_t nparent, int64_t K, int ntypes, const int32_t *child_start,
                   const int32_t *rec_start, const int32_t *rec_src, const int32_t *rec_off,
                   const float2 *T, const float2 *S, int R, float2 *Lout, hipStream_t s)
{
    if (nparent == 0 || K == 0) return hipSuccess;
    const size_t lds = (size_t)(ntypes + 1) * 64 * sizeof(float2);
    if (lds > 163840) return hipErrorInvalidValue;
    const int RC = R == 1 ? 1 : 4;
    const int nkc = (int)((K + 63) / 64);
    const int nz = (R + RC - 1) / RC;
    // about one workgroup per CU (the LDS slice takes the CU), at least 16
    // parents (one per wave) per workgroup
    const int64_t per = std::max<int64_t>(1, std::min<int64_t>((256 + nkc * nz - 1) / (nkc * nz),
                                                               (nparent + 15) / 16));
    const int64_t ppb = (nparent + per - 1) / per;
    dim3 grid((unsigned)(nkc * ((nparent + ppb - 1) / ppb)), 1, (unsigned)nz);
    if (RC == 1)
        hipLaunchKernelGGL(k_m2l_rec<1>, grid, dim3(1024), lds, s, nparent, K, ntypes,
                           child_start, rec_start, rec_src, rec_off, T, S, R, nkc, ppb, Lout);
    else
        hipLaunchKernelGGL(k_m2l_rec<4>, grid, dim3(1024), lds, s, nparent, K, ntypes,
                           child_start, rec_start, rec_src, rec_off, T, S, R, nkc, ppb, Lout);
    return hipGetLastError();
}

hipError_t m2l(int64_t nbox, int64_t K, const int32_t *far_start, const int32_t *far_src,
               const int16_t *far_type, const float2 *T, const float2 *S, int R,
               float2 *Lout, hipStream_t s)
{
    if (nbox * K == 0) return hipSuccess;
    const int64_t waves = nbox * ((K + 63) / 64);
    const unsigned blocks = (unsigned)((waves + 3) / 4);
    if (R == 1)
        hipLaunchKernelGGL(k_m2l<1>, dim3(blocks, 1), dim3(256), 0, s, nbox, K, far_start,
                           far_src, far_type, T, S, R, Lout);
    else if (R <= 4)
        hipLaunchKernelGGL(k_m2l<4>, dim3(blocks, 1), dim3(256), 0, s, nbox, K, far_start,
                           far_src, far_type, T, S, R, Lout);
    else
        hipLaunchKernelGGL(k_m2l<8>, dim3(blocks, (R + 7) / 8), dim3(256), 0, s, nbox, K,
                           far_start, far_src, far_type, T, S, R, Lout);
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
