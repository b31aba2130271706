// M2L (Sec. 3.2.3): the diagonal translation L_b += sum_{b' in IL(b)}
// T_{l,t(b,b')} (.) S_b' over the interaction lists, elementwise over the
// K_l samples and every right-hand side.  Kernel forms: per observer from
// L2, operator slice in LDS, sibling groups, and sibling groups with
// per-source records (three parent schedules, a 32-sample slice and
// antipodal slices for one RHS); the autotuner picks one per level.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>

#include "devmath.h"
#include "kernels.h"

namespace mlfma {
namespace dev {

thread_local LaunchTiming launch_timing;

// hipLaunchKernelGGL, or hipExtLaunchKernelGGL with the armed timing events
#define M2L_LAUNCH(kernel, grid, block, shm, stream, ...)                                   \
    do {                                                                                     \
        if (launch_timing.start) {                                                           \
            hipExtLaunchKernelGGL(kernel, grid, block, shm, stream, launch_timing.start,     \
                                  launch_timing.stop, 0, __VA_ARGS__);                       \
            launch_timing.used = true;                                                       \
        } else {                                                                             \
            hipLaunchKernelGGL(kernel, grid, block, shm, stream, __VA_ARGS__);               \
        }                                                                                    \
    } while (0)

// Compute units of the current device (cached per device).
int cu_count()
{
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cache[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        cache[dev] = n;
    }
    return cache[dev];
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

// The same slice interpolated from sampled operators: for operator t and
// sample k, gamma = the angle between khat_k and the integer offset d_t
// (atan2 of the norm of the cross product and the dot product, in FP64:
// the interpolant moves by up to 0.4 max|T| per table spacing, and an FP32
// angle would be off by about 1e-5 of a spacing at M = 456), x = gamma M /
// pi, and T = sum_j w_j tab[row][m0 + j], m0 = floor(x) - 4, j = 0..9,
// with the Lagrange weights w_j = prod_{i != j} (f + 4 - i) / (j - i) of
// the fraction f = x - floor(x) in FP32; indices below 0 or above M mirror
// (T is even about 0 and about pi).
template <int KC>
__device__ void stage_t_interp(float2 *Ts, SampledT st, int ntypes, int64_t K, int64_t k0)
{
    constexpr int P = 10;
    // 1 / prod_{i != j} (j - i)
    constexpr float cw[P] = {1.f / -362880.f, 1.f / 40320.f, 1.f / -10080.f, 1.f / 4320.f,
                             1.f / -2880.f,   1.f / 2880.f,  1.f / -4320.f,  1.f / 10080.f,
                             1.f / -40320.f,  1.f / 362880.f};
    const int total = ntypes * KC;
    const int M = st.M;
    const double scale = (double)M * 0.318309886183790671537767526745;  // M / pi
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int t = idx / KC, kk = idx % KC;
        float2 v = make_float2(0.f, 0.f);
        if (k0 + kk < K) {
            const int ki = (int)(k0 + kk);
            const int ti = ki / st.nph, pj = ki - ti * st.nph;
            const double ct = st.trig[2 * ti], sn = st.trig[2 * ti + 1];
            const double cp = st.trig[2 * st.nth + 2 * pj], sp = st.trig[2 * st.nth + 2 * pj + 1];
            const double kx = sn * cp, ky = sn * sp, kz = ct;
            const float4 xr = st.xr[t];
            const double dx = xr.x, dy = xr.y, dz = xr.z;
            const double c = kx * dx + ky * dy + kz * dz;
            const double cx = ky * dz - kz * dy, cy = kz * dx - kx * dz, cz = kx * dy - ky * dx;
            const double x = atan2(sqrt(cx * cx + cy * cy + cz * cz), c) * scale;
            const double fl = floor(x);
            const float f = (float)(x - fl);
            const int m0 = (int)fl - 4;
            float pre[P], suf[P];
            pre[0] = 1.f;
#pragma unroll
            for (int j = 1; j < P; ++j) pre[j] = pre[j - 1] * (f + (float)(5 - j));
            suf[P - 1] = 1.f;
#pragma unroll
            for (int j = P - 2; j >= 0; --j) suf[j] = suf[j + 1] * (f + (float)(3 - j));
            const float2 *row = st.tab + (int64_t)(int)xr.w * (M + 1);
#pragma unroll
            for (int j = 0; j < P; ++j) {
                int m = m0 + j;
                m = m < 0 ? -m : m;
                m = m > M ? 2 * M - m : m;
                const float w = pre[j] * suf[j] * cw[j];
                const float2 tv = row[m];
                v.x += w * tv.x;
                v.y += w * tv.y;
            }
        }
        Ts[idx] = v;
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
    M2L_LAUNCH((k_m2l_sg<RCV, KCV>), grid, block, lds, s, nparent, K, ntypes,    \
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
    M2L_LAUNCH((k_m2l_lds<RCV, KCV>), grid, block, lds, s, nbox, K, ntypes,      \
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
// The records of a parent are walked in batches of U (the host pads every
// list to a multiple of 4 and appends 8 zero records after the last list).
// The spectra of source s for right-hand side c sit at S + s * sstride +
// voff[c] (32-bit lane offsets).
//
// One right-hand side: a three-stage software pipeline.  The record data
// and the source spectra of batches j+1 and j+2 are requested before batch
// j is computed, so a wave has three batches of loads in flight; the two
// batches past the end of the list are fetched and never used (they read
// the next list or the appended records).  The spectra are read through a buffer resource based
// at the source (scalar address arithmetic only).
template <int NO, bool ANTI = false>
__device__ __forceinline__ void m2l_rec_parent1(const char *Tsb, int lane8, int e0, int e1,
                                                const int32_t *__restrict__ rec_src,
                                                const int32_t *__restrict__ rec_off,
                                                const char *__restrict__ Sb, uint64_t sstride,
                                                uint32_t voff, float2 (&acc)[8][1])
{
    constexpr int U = NO > 4 ? 2 : 4;  // records per batch
    const int nb = (e1 - e0) / U;
    if (nb <= 0) return;
    const int32_t *rs = rec_src + e0;
    const int32_t *ro = rec_off + 8 * (int64_t)e0;
    float2 va[U], vb[U], vc[U];
    int oa[U][NO], ob[U][NO], oc[U][NO];
    auto fetch = [&](int j, float2 (&v)[U], int (&of)[U][NO]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int sidx = rs[j * U + u];
#pragma unroll
            for (int i = 0; i < NO; ++i) of[u][i] = ro[8 * (j * U + u) + i];
            const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(Sb + (uint64_t)(uint32_t)sidx * sstride), (short)0, (int)sstride,
                0x00020000);
            // two 32-bit loads: this compiler lowers the 64-bit buffer-load
            // builtin to a 32-bit load
            const uint32_t re = __builtin_amdgcn_raw_buffer_load_b32(rsrc, voff, 0, 0);
            const uint32_t im = __builtin_amdgcn_raw_buffer_load_b32(rsrc, voff + 4, 0, 0);
            v[u] = make_float2(__builtin_bit_cast(float, re), __builtin_bit_cast(float, im));
        }
    };
    auto compute = [&](const float2 (&v)[U], const int (&of)[U][NO]) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int i = 0; i < NO; ++i) {
                // ANTI: the offset carries the mirror mask in its low bits
                const int a = ANTI ? (of[u][i] ^ lane8) : (of[u][i] + lane8);
                const float2 tv = *(const float2 *)(Tsb + a);
                acc[i][0] = cfma(tv, v[u], acc[i][0]);
            }
    };
    fetch(0, va, oa);
    fetch(1, vb, ob);
    for (int j = 0;;) {
        fetch(j + 2, vc, oc);
        compute(va, oa);
        if (++j >= nb) break;
        fetch(j + 2, va, oa);
        compute(vb, ob);
        if (++j >= nb) break;
        fetch(j + 2, vb, ob);
        compute(vc, oc);
        if (++j >= nb) break;
    }
}

// Several right-hand sides: batches of U records, the scalar record data of
// the next batch loaded while the current one computes (one scalar-load
// latency per batch); the spectrum loads of a batch are shared by RC
// right-hand sides.  (The two-stage pipeline of the one-RHS loop measured
// slower here: 7.1 against 6.0 ms at 64 right-hand sides on the 262k sphere.)
template <int RC, int NO>
__device__ __forceinline__ void m2l_rec_parent(const char *Tsb, int lane8, int e0, int e1,
                                               const int32_t *__restrict__ rec_src,
                                               const int32_t *__restrict__ rec_off,
                                               const char *__restrict__ Sb, uint64_t sstride,
                                               const uint32_t (&voff)[RC], float2 (&acc)[8][RC])
{
    constexpr int U = 4;
    int src[U], off[U][NO];
    auto load_rec = [&](int eb, int (&sr)[U], int (&of)[U][NO]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            sr[u] = rec_src[eb + u];
#pragma unroll
            for (int i = 0; i < NO; ++i) of[u][i] = rec_off[8 * (eb + u) + i];
        }
    };
    if (e1 <= e0) return;
    load_rec(e0, src, off);
    for (int eb = e0; eb < e1; eb += U) {
        float2 sv[U][RC];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const char *base = Sb + (uint64_t)(uint32_t)src[u] * sstride;
#pragma unroll
            for (int c = 0; c < RC; ++c) sv[u][c] = *(const float2 *)(base + voff[c]);
        }
        // the batch after the last reads the next list or the appended records
        int nsrc[U], noff[U][NO];
        load_rec(eb + U, nsrc, noff);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int i = 0; i < NO; ++i) {
                const float2 tv = *(const float2 *)(Tsb + (off[u][i] + lane8));
#pragma unroll
                for (int c = 0; c < RC; ++c) acc[i][c] = cfma(tv, sv[u][c], acc[i][c]);
            }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            src[u] = nsrc[u];
#pragma unroll
            for (int i = 0; i < NO; ++i) off[u][i] = noff[u][i];
        }
    }
}

template <int RC, int NW, bool SAMPLED>
__global__ void __launch_bounds__(64 * NW)
k_m2l_rec(int64_t nparent, int64_t K, int ntypes, const int32_t *__restrict__ child_start,
          const int32_t *__restrict__ rec_start, const int32_t *__restrict__ rec_src,
          const int32_t *__restrict__ rec_off, const float2 *__restrict__ T,
          const float2 *__restrict__ S, int R, int nkc, int nrange, int nwg, int balanced,
          float2 *__restrict__ Lout, SampledT sampled)
{
    // Two schedules (about one workgroup per CU either way, so the LDS
    // staging of the operators is amortised over many parents):
    //  nwg == 0: workgroup w serves sample chunk w % nkc, right-hand-side
    //    chunk blockIdx.z and parent range w / nkc of nrange contiguous
    //    ranges.  balanced == 0: ranges of equal parent counts, taken by the
    //    NW waves round-robin.  balanced == 1: ranges holding equal numbers
    //    of records (bounds found by binary search in the record offsets),
    //    the waves taking parents one at a time from a counter in LDS, so a
    //    wave that drew short lists takes more of them.  (Numbering the
    //    workgroups so that each XCD gets a contiguous run of ranges
    //    measured slower at one RHS.)
    //  nwg > 0: slice-major sweep for many right-hand sides.  The nwg
    //    workgroups of one (sample chunk, RHS chunk) slice are consecutive,
    //    so the resident workgroups share a slice and sweep the parents
    //    interleaved (parent = (w nwg ... ) + wave): the sources they re-read
    //    stay within one window of the Morton order, small enough for the
    //    Infinity Cache, instead of every slice streaming at once.
    extern __shared__ float2 Ts[];  // [ntypes + 1][64], row ntypes = 0
    __shared__ int next_parent;
    // balanced: workgroups renumbered so that each XCD (they are dealt to
    // the 8 XCDs round-robin) serves a contiguous run of ranges
    const int64_t w = nwg ? blockIdx.x % nwg
                          : (balanced ? xcd_contiguous(blockIdx.x, gridDim.x) : blockIdx.x);
    const int64_t slice = nwg ? blockIdx.x / nwg : 0;
    const int kc = nwg ? (int)(slice % nkc) : (int)(w % nkc);
    const int64_t k0 = (int64_t)kc * 64;
    if constexpr (SAMPLED)
        stage_t_interp<64>(Ts, sampled, ntypes, K, k0);
    else
        stage_t_slice<64>(Ts, T, ntypes, K, k0);
    for (int idx = threadIdx.x; idx < 64; idx += blockDim.x)
        Ts[ntypes * 64 + idx] = make_float2(0.f, 0.f);
    if (threadIdx.x == 0) next_parent = 0;
    __syncthreads();
    const char *Tsb = (const char *)Ts;
    const int lane = threadIdx.x & 63;
    const int lane8 = lane * 8;
    const int64_t k = k0 + lane;
    const bool valid = k < K;
    const int64_t kk = valid ? k : K - 1;
    const int r0 = (nwg ? (int)(slice / nkc) : (int)blockIdx.z) * RC;
    const int rc = min(RC, R - r0);
    // lane offsets of the right-hand sides (a missing one re-reads r0)
    const uint64_t sstride = (uint64_t)R * (uint64_t)K * sizeof(float2);
    uint32_t voff[RC];
#pragma unroll
    for (int c = 0; c < RC; ++c)
        // (a multiple of 8 below 2^31: the mask states it, so the two
        // 32-bit loads of a value merge into one 64-bit load)
        voff[c] = (uint32_t)(((int64_t)(r0 + (c < rc ? c : 0)) * K + kk) * (int64_t)sizeof(float2)) &
                  0x7ffffff8u;
    const char *Sb = (const char *)S;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int64_t pbeg, pend;
    if (nwg) {
        pbeg = w * NW + wave;
        pend = nparent;
    } else if (!balanced) {
        const int64_t ppb = (nparent + nrange - 1) / nrange;
        pbeg = (w / nkc) * ppb;
        pend = min(nparent, pbeg + ppb);
    } else {
        // first parent whose records start at or after the target
        const int64_t total = rec_start[nparent];
        const int64_t rg = w / nkc;
        auto lower = [&](int64_t target) -> int64_t {
            int64_t lo = 0, hi = nparent;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if ((int64_t)__builtin_amdgcn_readfirstlane(rec_start[mid]) < target) lo = mid + 1;
                else hi = mid;
            }
            return lo;
        };
        pbeg = rg == 0 ? 0 : lower(total * rg / nrange);
        pend = rg == nrange - 1 ? nparent : lower(total * (rg + 1) / nrange);
    }
    // the next parent of this wave: interleaved (sweep) or from the counter
    auto take = [&](int64_t prev) -> int64_t {
        if (nwg) return prev + (int64_t)nwg * NW;
        if (!balanced) return prev + NW;
        int t = 0;
        if (lane == 0) t = atomicAdd(&next_parent, 1);
        return pbeg + __builtin_amdgcn_readfirstlane(t);
    };
    for (int64_t P = nwg ? pbeg : (balanced ? take(0) : pbeg + wave); P < pend; P = take(P)) {
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
        if constexpr (RC == 1)                                                               \
            m2l_rec_parent1<N>(Tsb, lane8, e0, e1, rec_src, rec_off, Sb, sstride, voff[0], acc); \
        else                                                                                 \
            m2l_rec_parent<RC, N>(Tsb, lane8, e0, e1, rec_src, rec_off, Sb, sstride, voff, acc); \
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

// One right-hand side with a 32-sample operator slice: (316 + 1) x 32 x 8 B
// of LDS, so two workgroups share a CU and twice the waves hide latency.
// The two half-waves take the even and the odd records of the parent on
// the same 32 samples (lane k and k + 32 hold partial sums of one sample,
// added by a lane swap at the end); records are walked in batches of two
// pairs, the next batch's loads issued before the current batch computes.
// Record offsets address 64-sample rows and are halved here.
template <int NO>
__device__ __forceinline__ void m2l_rec_parent_half(const char *Tsb, int lane8, int half, int e0,
                                                    int e1, const int32_t *__restrict__ rec_src,
                                                    const int32_t *__restrict__ rec_off,
                                                    const float2 *__restrict__ S, int64_t K,
                                                    int64_t kk, float2 (&acc)[8])
{
    constexpr int U = 2;  // record pairs per batch (lists are padded to 4)
    const int nb = (e1 - e0) / (2 * U);
    if (nb <= 0) return;
    float2 va[U], vb[U];
    int oa[U][NO], ob[U][NO];
    auto fetch = [&](int j, float2 (&v)[U], int (&of)[U][NO]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + 2 * (j * U + u);
            const int s0 = rec_src[e], s1 = rec_src[e + 1];
            const int src = half ? s1 : s0;
#pragma unroll
            for (int i = 0; i < NO; ++i) {
                const int f0 = rec_off[8 * e + i] >> 1, f1 = rec_off[8 * (e + 1) + i] >> 1;
                of[u][i] = half ? f1 : f0;
            }
            v[u] = S[(int64_t)src * K + kk];
        }
    };
    auto compute = [&](const float2 (&v)[U], const int (&of)[U][NO]) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int i = 0; i < NO; ++i) {
                const float2 tv = *(const float2 *)(Tsb + (of[u][i] + lane8));
                acc[i] = cfma(tv, v[u], acc[i]);
            }
    };
    fetch(0, va, oa);
    for (int j = 0;;) {
        fetch(j + 1, vb, ob);
        compute(va, oa);
        if (++j >= nb) break;
        fetch(j + 1, va, oa);
        compute(vb, ob);
        if (++j >= nb) break;
    }
}

template <int NW>
__global__ void __launch_bounds__(64 * NW, 8)  // two workgroups: 8 waves per SIMD
k_m2l_rec_half(int64_t nparent, int64_t K, int ntypes, const int32_t *__restrict__ child_start,
               const int32_t *__restrict__ rec_start, const int32_t *__restrict__ rec_src,
               const int32_t *__restrict__ rec_off, const float2 *__restrict__ T,
               const float2 *__restrict__ S, int nkc, int nrange, float2 *__restrict__ Lout)
{
    // the balanced schedule of k_m2l_rec (record-balanced XCD-contiguous
    // parent ranges, parents handed to waves from an LDS counter)
    extern __shared__ float2 Ts[];  // [ntypes + 1][32], row ntypes = 0
    __shared__ int next_parent;
    const int64_t w = xcd_contiguous(blockIdx.x, gridDim.x);
    const int kc = (int)(w % nkc);
    const int64_t k0 = (int64_t)kc * 32;
    stage_t_slice<32>(Ts, T, ntypes, K, k0);
    for (int idx = threadIdx.x; idx < 32; idx += blockDim.x)
        Ts[ntypes * 32 + idx] = make_float2(0.f, 0.f);
    if (threadIdx.x == 0) next_parent = 0;
    __syncthreads();
    const char *Tsb = (const char *)Ts;
    const int lane = threadIdx.x & 63;
    const int kl = lane & 31, half = lane >> 5;
    const int lane8 = kl * 8;
    const int64_t k = k0 + kl;
    const bool valid = k < K;
    const int64_t kk = valid ? k : K - 1;
    const int64_t total = rec_start[nparent];
    const int64_t rg = w / nkc;
    auto lower = [&](int64_t target) -> int64_t {
        int64_t lo = 0, hi = nparent;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)__builtin_amdgcn_readfirstlane(rec_start[mid]) < target) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    const int64_t pbeg = rg == 0 ? 0 : lower(total * rg / nrange);
    const int64_t pend = rg == nrange - 1 ? nparent : lower(total * (rg + 1) / nrange);
    auto take = [&]() -> int64_t {
        int t = 0;
        if (lane == 0) t = atomicAdd(&next_parent, 1);
        return pbeg + __builtin_amdgcn_readfirstlane(t);
    };
    for (int64_t P = take(); P < pend; P = take()) {
        const int o0 = __builtin_amdgcn_readfirstlane(child_start[P]);
        const int no = __builtin_amdgcn_readfirstlane(child_start[P + 1]) - o0;
        const int e0 = __builtin_amdgcn_readfirstlane(rec_start[P]);
        const int e1 = __builtin_amdgcn_readfirstlane(rec_start[P + 1]);
        float2 acc[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = make_float2(0.f, 0.f);
        switch (no) {
#define REC_HALF_CASE(N)                                                                      \
    case N:                                                                                   \
        m2l_rec_parent_half<N>(Tsb, lane8, half, e0, e1, rec_src, rec_off, S, K, kk, acc);    \
        break;
            REC_HALF_CASE(1) REC_HALF_CASE(2) REC_HALF_CASE(3) REC_HALF_CASE(4)
            REC_HALF_CASE(5) REC_HALF_CASE(6) REC_HALF_CASE(7) REC_HALF_CASE(8)
#undef REC_HALF_CASE
        default: break;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            acc[i].x += __shfl_xor(acc[i].x, 32, 64);
            acc[i].y += __shfl_xor(acc[i].y, 32, 64);
        }
        if (valid && half == 0) {
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (i < no) Lout[(int64_t)(o0 + i) * K + k] = acc[i];
        }
    }
}

// One right-hand side with antipodal slices.  The operator of offset -d is
// that of d at the opposite direction, T_{-d}(k) = T_d(-k), and the grid
// holds every direction's opposite (Gauss-Legendre nodes symmetric about
// the equator, an even number of phi samples).  A slice is 32 directions
// and their 32 opposites, ordered so that lane l and lane l ^ 63 are
// opposite (aperm: slice lane -> sample, -1 past the end); LDS then needs
// the operators of one offset of each +-pair only, (158 + 1) x 64 x 8 B,
// and two workgroups share a CU.  A record slot holds
// pair * 512 | (negated ? 504 : 0), so the lane's LDS address is that
// value XOR (8 lane): the mirrored lane for a negated offset, at the cost
// of the addition it replaces.  Parents are scheduled as in the balanced
// schedule of k_m2l_rec.
//
// The same kernel runs octant slices (variant 8, 8-wave workgroups): the
// reflection of an offset in any coordinate plane maps the operator to the
// reflected directions, T_{R d}(k) = T_d(R k), and the grid is closed
// under the three reflections (x: phi -> pi - phi, y: phi -> -phi, z:
// theta -> pi - theta).  A slice holds 8 orbits of 8 directions, lane
// 8 o + g carrying reflection g (3 bits) of orbit o's first direction, and
// LDS the operators of the offsets (|dx|, |dy|, |dz|) only (at most 56 + 1
// rows, 29 KB: several workgroups per CU).  A record slot holds
// row * 512 | 8 g for the offset R_g (|d|), so the same XOR with 8 lane
// lands on lane 8 o + (g' ^ g), the reflected direction.  A direction
// fixed by some reflection appears more than once in its orbit; only its
// first slot writes (slot codes below zero).
template <int NW>
__global__ void __launch_bounds__(64 * NW)
k_m2l_anti(int64_t nparent, int64_t K, int ntp, const int32_t *__restrict__ child_start,
           const int32_t *__restrict__ rec_start, const int32_t *__restrict__ rec_src,
           const int32_t *__restrict__ rec_off, const float2 *__restrict__ Tp,
           const int32_t *__restrict__ aperm, int64_t Kp, const float2 *__restrict__ S,
           int nkc, int nrange, float2 *__restrict__ Lout)
{
    extern __shared__ float2 Ts[];  // [ntp + 1][64], row ntp = 0
    __shared__ int next_parent;
    const int64_t w = xcd_contiguous(blockIdx.x, gridDim.x);
    const int kc = (int)(w % nkc);
    const int64_t k0 = (int64_t)kc * 64;
    stage_t_slice<64>(Ts, Tp, ntp, Kp, k0);
    for (int idx = threadIdx.x; idx < 64; idx += blockDim.x)
        Ts[ntp * 64 + idx] = make_float2(0.f, 0.f);
    if (threadIdx.x == 0) next_parent = 0;
    __syncthreads();
    const char *Tsb = (const char *)Ts;
    const int lane = threadIdx.x & 63;
    const int lane8 = lane * 8;
    // slot code: sample q >= 0 (computed and written), -(q + 2) (computed,
    // not written: a repeat of a sample earlier in the slice), -1 (padding)
    const int code = aperm[k0 + lane];
    const int k = code >= 0 ? code : (code <= -2 ? -code - 2 : 0);
    const bool valid = code >= 0;
    // (a multiple of 8 below 2^31, as the mask states: the value's two
    // 32-bit loads merge into one)
    const uint32_t voff = ((uint32_t)k * (uint32_t)sizeof(float2)) & 0x7ffffff8u;
    const uint64_t sstride = (uint64_t)K * sizeof(float2);
    const char *Sb = (const char *)S;
    const int64_t total = rec_start[nparent];
    const int64_t rg = w / nkc;
    auto lower = [&](int64_t target) -> int64_t {
        int64_t lo = 0, hi = nparent;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)__builtin_amdgcn_readfirstlane(rec_start[mid]) < target) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    const int64_t pbeg = rg == 0 ? 0 : lower(total * rg / nrange);
    const int64_t pend = rg == nrange - 1 ? nparent : lower(total * (rg + 1) / nrange);
    auto take = [&]() -> int64_t {
        int t = 0;
        if (lane == 0) t = atomicAdd(&next_parent, 1);
        return pbeg + __builtin_amdgcn_readfirstlane(t);
    };
    for (int64_t P = take(); P < pend; P = take()) {
        const int o0 = __builtin_amdgcn_readfirstlane(child_start[P]);
        const int no = __builtin_amdgcn_readfirstlane(child_start[P + 1]) - o0;
        const int e0 = __builtin_amdgcn_readfirstlane(rec_start[P]);
        const int e1 = __builtin_amdgcn_readfirstlane(rec_start[P + 1]);
        float2 acc[8][1];
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i][0] = make_float2(0.f, 0.f);
        switch (no) {
#define ANTI_CASE(N)                                                                          \
    case N:                                                                                   \
        m2l_rec_parent1<N, true>(Tsb, lane8, e0, e1, rec_src, rec_off, Sb, sstride, voff, acc); \
        break;
            ANTI_CASE(1) ANTI_CASE(2) ANTI_CASE(3) ANTI_CASE(4)
            ANTI_CASE(5) ANTI_CASE(6) ANTI_CASE(7) ANTI_CASE(8)
#undef ANTI_CASE
        default: break;
        }
        if (valid) {
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (i < no) Lout[(int64_t)(o0 + i) * K + k] = acc[i][0];
        }
    }
}

// Resident workgroups of k_m2l_anti<NW> per CU with `lds` bytes of dynamic
// LDS (occupancy query, cached per (NW, lds) on the current device).
template <int NW>
static int anti_per_cu(size_t lds)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_m2l_anti<NW>, 64 * NW, lds) !=
            hipSuccess || nb < 1) {
        (void)hipGetLastError();
        nb = (int)std::max<size_t>(1, 163840 / (lds + 16));
    }
    return nb;
}

hipError_t m2l_anti(int64_t nparent, int64_t K, int ntp, const int32_t *child_start,
                    const int32_t *rec_start, const int32_t *rec_src, const int32_t *rec_off,
                    const float2 *Tp, const int32_t *aperm, int64_t Kp, const float2 *S,
                    float2 *Lout, hipStream_t s, int max_wg, int waves)
{
    if (nparent == 0 || K == 0) return hipSuccess;
    const size_t lds = (size_t)(ntp + 1) * 64 * sizeof(float2);
    if (lds + 16 > 163840) return hipErrorInvalidValue;  // + the static counter
    if ((uint64_t)K * sizeof(float2) > 0x7fffffffull || Kp % 64 != 0) return hipErrorInvalidValue;
    if (waves != 8 && waves != 16) return hipErrorInvalidValue;
    const int nkc = (int)(Kp / 64);
    const int ncu = max_wg > 0 ? std::min(max_wg, cu_count()) : cu_count();
    // antipodal slices (16 waves): at most two workgroups per CU; octant
    // slices (8 waves, a quarter of the LDS): as many as fit
    const int per_cu = waves == 16 ? std::min(2, anti_per_cu<16>(lds)) : anti_per_cu<8>(lds);
    const int nrange = (int)std::max<int64_t>(
        1, std::min<int64_t>(per_cu * ncu / nkc, (nparent + waves - 1) / waves));
    if (waves == 16)
        M2L_LAUNCH((k_m2l_anti<16>), dim3((unsigned)(nkc * nrange)), dim3(64 * 16), lds, s,
                   nparent, K, ntp, child_start, rec_start, rec_src, rec_off, Tp, aperm, Kp, S,
                   nkc, nrange, Lout);
    else
        M2L_LAUNCH((k_m2l_anti<8>), dim3((unsigned)(nkc * nrange)), dim3(64 * 8), lds, s,
                   nparent, K, ntp, child_start, rec_start, rec_src, rec_off, Tp, aperm, Kp, S,
                   nkc, nrange, Lout);
    return hipGetLastError();
}

hipError_t m2l_rec(int64_t nparent, int64_t K, int ntypes, const int32_t *child_start,
                   const int32_t *rec_start, const int32_t *rec_src, const int32_t *rec_off,
                   const float2 *T, const float2 *S, int R, float2 *Lout, hipStream_t s,
                   int schedule, int max_wg, SampledT sampled)
{
    const bool sweep = schedule == 1;
    if (nparent == 0 || K == 0) return hipSuccess;
    // the 32-sample form copies from the full table only
    if (sampled.tab && schedule == 3) return hipErrorInvalidValue;
    if (schedule == 3 && R == 1) {
        // one RHS, 32-sample slice, two workgroups per CU
        const size_t lds2 = (size_t)(ntypes + 1) * 32 * sizeof(float2);
        if (2 * (lds2 + 16) > 163840) return hipErrorInvalidValue;
        const int NW = 16;
        const int nkc2 = (int)((K + 31) / 32);
        const int slots = 2 * (max_wg > 0 ? std::min(max_wg, cu_count()) : cu_count());
        const int nr = (int)std::max<int64_t>(1, std::min<int64_t>(slots / nkc2, (nparent + NW - 1) / NW));
        M2L_LAUNCH((k_m2l_rec_half<16>), dim3((unsigned)(nkc2 * nr)), dim3(64 * NW), lds2, s,
                           nparent, K, ntypes, child_start, rec_start, rec_src, rec_off, T, S,
                           nkc2, nr, Lout);
        return hipGetLastError();
    }
    if (schedule == 3) schedule = 2;  // several RHS: the 64-sample balanced schedule
    const size_t lds = (size_t)(ntypes + 1) * 64 * sizeof(float2);
    if (lds + 16 > 163840) return hipErrorInvalidValue;  // + the static counter
    // 32-bit lane offsets (and buffer range) within one source's spectra
    if ((uint64_t)R * (uint64_t)K * sizeof(float2) > 0x7fffffffull) return hipErrorInvalidValue;
    // right-hand sides per thread: 1 or 4 (8 per thread, with 8 waves per
    // workgroup for the registers of 8 x 8 accumulators, measured slower at
    // 64 right-hand sides: 10.1 ms against 8.3 ms on the 262k sphere)
    const int RC = R == 1 ? 1 : 4;
    const int NW = 16;
    const int nkc = (int)((K + 63) / 64);
    // the LDS slice allows one workgroup per CU: size the grid to the CU
    // count, as one workgroup more than the CUs doubles the kernel's time
    const int ncu = max_wg > 0 ? std::min(max_wg, cu_count()) : cu_count();
    const int nz = (R + RC - 1) / RC;
    dim3 grid;
    int nrange = 0;
    int nwg = 0;
    if (sweep) {
        // one workgroup per CU per slice, slices one after the other
        nwg = (int)std::max<int64_t>(1, std::min<int64_t>(ncu, (nparent + NW - 1) / NW));
        grid = dim3((unsigned)(nwg * nkc * nz), 1, 1);
    } else {
        // at most one workgroup per CU in all, at least one parent per wave
        nrange = (int)std::max<int64_t>(
            1, std::min<int64_t>(ncu / (nkc * nz), (nparent + NW - 1) / NW));
        if (schedule == 0) nrange = (int)((nparent + (nparent + nrange - 1) / nrange - 1) /
                                          ((nparent + nrange - 1) / nrange));
        grid = dim3((unsigned)(nkc * nrange), 1, (unsigned)nz);
    }
#define M2L_REC(RCV, NWV, SV)                                                                  \
    M2L_LAUNCH((k_m2l_rec<RCV, NWV, SV>), grid, dim3(64 * NWV), lds, s, nparent, K, ntypes, \
                       child_start, rec_start, rec_src, rec_off, T, S, R, nkc, nrange, nwg,   \
                       schedule == 2 ? 1 : 0, Lout, sampled)
    if (sampled.tab) {
        if (RC == 1) M2L_REC(1, 16, true);
        else M2L_REC(4, 16, true);
    } else {
        if (RC == 1) M2L_REC(1, 16, false);
        else M2L_REC(4, 16, false);
    }
#undef M2L_REC
    return hipGetLastError();
}

// Many right-hand sides on the matrix cores (variant 9).  For one sample k
// the M2L of a parent's children is a small dense product over the parent's
// source records, L[c][r] += sum_s T_{t(c,s)}[k] S[s][r].  A wave takes one
// parent, 16 samples and 4 NQ right-hand sides; v_mfma_f32_4x4x1f32 computes
// 16 independent 4x4 tiles, one per sample (block b = lane / 4, the sample
// k0 + 16 sb + b): the rows of a child pair p (child 2p real, imaginary,
// child 2p+1 real, imaginary; A from lane 4b + row), the columns four
// right-hand sides (B from lane 4b + column, D column lane % 4, row = the
// accumulator register).  Each source record takes two instructions per
// (pair, RHS block), one per part of the source value:
//   re += Tr Sr - Ti Si,  im += Ti Sr + Tr Si,
// the operator values read from the LDS slice of the record kernels
// (64 samples, the records' byte offsets), the source values from the
// spectra.  The 16 waves of a workgroup are 4 sample blocks x 4 parent
// streams over the workgroup's parent range; records one ahead in flight.
typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int NP, int NQ>
__device__ __forceinline__ void m2l_mfma_parent(const char *Tsb, int lane, int toff, int e0,
                                                int e1, const int32_t *__restrict__ rec_src,
                                                const int32_t *__restrict__ rec_off,
                                                const char *__restrict__ Sb, uint64_t sstride,
                                                const uint32_t (&voff)[NQ],
                                                floatx4 (&acc)[NQ][4])
{
    if (e1 <= e0) return;
    const bool second = (lane & 2) != 0;  // the pair's second child
    const bool imag = (lane & 1) != 0;    // imaginary row
    float2 ta[NP], tb[NP], sa[NQ], sb[NQ];
    auto fetch = [&](int e, float2 (&t)[NP], float2 (&v)[NQ]) {
        const char *base = Sb + (uint64_t)(uint32_t)rec_src[e] * sstride;
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[q] = *(const float2 *)(base + voff[q]);
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int o0 = rec_off[8 * (int64_t)e + 2 * p], o1 = rec_off[8 * (int64_t)e + 2 * p + 1];
            t[p] = *(const float2 *)(Tsb + (second ? o1 : o0) + toff);
        }
    };
    auto compute = [&](const float2 (&t)[NP], const float2 (&v)[NQ]) {
        float a1[NP], a2[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            a1[p] = imag ? t[p].y : t[p].x;
            a2[p] = imag ? t[p].x : -t[p].y;
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int p = 0; p < NP; ++p)
                acc[q][p] = __builtin_amdgcn_mfma_f32_4x4x1f32(a1[p], v[q].x, acc[q][p], 0, 0, 0);
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int p = 0; p < NP; ++p)
                acc[q][p] = __builtin_amdgcn_mfma_f32_4x4x1f32(a2[p], v[q].y, acc[q][p], 0, 0, 0);
    };
    // (the record after a list's last is the next list's first or one of
    // the zero records appended after the last list: fetched, never used)
    fetch(e0, ta, sa);
    for (int e = e0;;) {
        fetch(e + 1, tb, sb);
        compute(ta, sa);
        if (++e >= e1) break;
        fetch(e + 1, ta, sa);
        compute(tb, sb);
        if (++e >= e1) break;
    }
}

template <int NQ, bool SAMPLED>
__global__ void __launch_bounds__(1024)
k_m2l_mfma(int64_t nparent, int64_t K, int ntypes, const int32_t *__restrict__ child_start,
           const int32_t *__restrict__ rec_start, const int32_t *__restrict__ rec_src,
           const int32_t *__restrict__ rec_off, const float2 *__restrict__ T,
           const float2 *__restrict__ S, int R, int nkc, int nrange, float2 *__restrict__ Lout,
           SampledT sampled)
{
    extern __shared__ float2 Ts[];  // [ntypes + 1][64], row ntypes = 0
    const int64_t w = xcd_contiguous(blockIdx.x, gridDim.x);
    const int kc = (int)(w % nkc);
    const int64_t k0 = (int64_t)kc * 64;
    if constexpr (SAMPLED)
        stage_t_interp<64>(Ts, sampled, ntypes, K, k0);
    else
        stage_t_slice<64>(Ts, T, ntypes, K, k0);
    for (int idx = threadIdx.x; idx < 64; idx += blockDim.x)
        Ts[ntypes * 64 + idx] = make_float2(0.f, 0.f);
    __syncthreads();
    const char *Tsb = (const char *)Ts;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sblk = wave & 3;  // 16-sample block
    const int pstream = wave >> 2;
    const int64_t k = k0 + 16 * sblk + (lane >> 2);
    const bool kvalid = k < K;
    const int64_t kk = kvalid ? k : K - 1;
    const int toff = (16 * sblk + (lane >> 2)) * (int)sizeof(float2);
    const int r0 = (int)blockIdx.z * 4 * NQ;
    const uint64_t sstride = (uint64_t)R * (uint64_t)K * sizeof(float2);
    uint32_t voff[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int r = r0 + 4 * q + (lane & 3);
        // (a multiple of 8 below 2^31, as the mask states)
        voff[q] = (uint32_t)(((int64_t)(r < R ? r : r0) * K + kk) * (int64_t)sizeof(float2)) &
                  0x7ffffff8u;
    }
    const char *Sb = (const char *)S;
    // parent range of the workgroup: equal record counts (binary search)
    const int64_t total = rec_start[nparent];
    const int64_t rg = w / nkc;
    auto lower = [&](int64_t target) -> int64_t {
        int64_t lo = 0, hi = nparent;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)__builtin_amdgcn_readfirstlane(rec_start[mid]) < target) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    const int64_t pbeg = rg == 0 ? 0 : lower(total * rg / nrange);
    const int64_t pend = rg == nrange - 1 ? nparent : lower(total * (rg + 1) / nrange);
    for (int64_t P = pbeg + pstream; P < pend; P += 4) {
        const int o0 = __builtin_amdgcn_readfirstlane(child_start[P]);
        const int no = __builtin_amdgcn_readfirstlane(child_start[P + 1]) - o0;
        const int e0 = __builtin_amdgcn_readfirstlane(rec_start[P]);
        const int e1 = __builtin_amdgcn_readfirstlane(rec_start[P + 1]);
        floatx4 acc[NQ][4];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int p = 0; p < 4; ++p) acc[q][p] = floatx4{0.f, 0.f, 0.f, 0.f};
        switch ((no + 1) >> 1) {
        case 1:
            m2l_mfma_parent<1, NQ>(Tsb, lane, toff, e0, e1, rec_src, rec_off, Sb, sstride, voff, acc);
            break;
        case 2:
            m2l_mfma_parent<2, NQ>(Tsb, lane, toff, e0, e1, rec_src, rec_off, Sb, sstride, voff, acc);
            break;
        case 3:
            m2l_mfma_parent<3, NQ>(Tsb, lane, toff, e0, e1, rec_src, rec_off, Sb, sstride, voff, acc);
            break;
        case 4:
            m2l_mfma_parent<4, NQ>(Tsb, lane, toff, e0, e1, rec_src, rec_off, Sb, sstride, voff, acc);
            break;
        default: break;
        }
        if (!kvalid) continue;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int r = r0 + 4 * q + (lane & 3);
            if (r >= R) continue;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                if (2 * p < no)
                    Lout[((int64_t)(o0 + 2 * p) * R + r) * K + k] =
                        make_float2(acc[q][p][0], acc[q][p][1]);
                if (2 * p + 1 < no)
                    Lout[((int64_t)(o0 + 2 * p + 1) * R + r) * K + k] =
                        make_float2(acc[q][p][2], acc[q][p][3]);
            }
        }
    }
}

hipError_t m2l_mfma(int64_t nparent, int64_t K, int ntypes, const int32_t *child_start,
                    const int32_t *rec_start, const int32_t *rec_src, const int32_t *rec_off,
                    const float2 *T, const float2 *S, int R, float2 *Lout, hipStream_t s,
                    int max_wg, SampledT sampled)
{
    if (nparent == 0 || K == 0) return hipSuccess;
    const size_t lds = (size_t)(ntypes + 1) * 64 * sizeof(float2);
    if (lds > 163840) return hipErrorInvalidValue;
    if ((uint64_t)R * (uint64_t)K * sizeof(float2) > 0x7fffffffull) return hipErrorInvalidValue;
    // right-hand sides per wave: 16, or 8 / 4 for fewer
    const int NQ = R > 8 ? 4 : R > 4 ? 2 : 1;
    const int nkc = (int)((K + 63) / 64);
    const int nz = (R + 4 * NQ - 1) / (4 * NQ);
    const int ncu = max_wg > 0 ? std::min(max_wg, cu_count()) : cu_count();
    // one workgroup per CU (the LDS slice), at least 4 parents per range
    const int nrange = (int)std::max<int64_t>(
        1, std::min<int64_t>(ncu / std::max(1, nkc * nz), (nparent + 3) / 4));
    const dim3 grid((unsigned)(nkc * nrange), 1, (unsigned)nz);
#define M2L_MFMA(NQV, SV)                                                                        \
    M2L_LAUNCH((k_m2l_mfma<NQV, SV>), grid, dim3(1024), lds, s, nparent, K, ntypes, child_start, \
               rec_start, rec_src, rec_off, T, S, R, nkc, nrange, Lout, sampled)
    if (sampled.tab) {
        if (NQ == 4) M2L_MFMA(4, true);
        else if (NQ == 2) M2L_MFMA(2, true);
        else M2L_MFMA(1, true);
    } else {
        if (NQ == 4) M2L_MFMA(4, false);
        else if (NQ == 2) M2L_MFMA(2, false);
        else M2L_MFMA(1, false);
    }
#undef M2L_MFMA
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
        M2L_LAUNCH(k_m2l<1>, dim3(blocks, 1), dim3(256), 0, s, nbox, K, far_start,
                           far_src, far_type, T, S, R, Lout);
    else if (R <= 4)
        M2L_LAUNCH(k_m2l<4>, dim3(blocks, 1), dim3(256), 0, s, nbox, K, far_start,
                           far_src, far_type, T, S, R, Lout);
    else
        M2L_LAUNCH(k_m2l<8>, dim3(blocks, (R + 7) / 8), dim3(256), 0, s, nbox, K,
                           far_start, far_src, far_type, T, S, R, Lout);
    return hipGetLastError();
}

}  // namespace dev
}  // namespace mlfma
