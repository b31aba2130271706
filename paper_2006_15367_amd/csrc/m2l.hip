// M2L (Sec. 3.2.3): the diagonal translation L_b += sum_{b' in IL(b)}
// T_{l,t(b,b')} (.) S_b' over the interaction lists, elementwise over the
// K_l samples and every right-hand side.  Four kernel variants (per
// observer from L2, operator slice in LDS, sibling groups, sibling groups
// with per-source records); the autotuner picks one per level.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "devmath.h"
#include "kernels.h"

namespace mlfma {
namespace dev {

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
    constexpr int U = RC >= 8 ? 2 : 4;  // records in flight per wave
    // the scalar record data of the next U records is loaded while the
    // current ones compute (one scalar-load latency per U records)
    int src[U], off[U][NO];
    auto load_rec = [&](int eb, int (&sr)[U], int (&of)[U][NO]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = eb + u < e1 ? eb + u : e1 - 1;
            sr[u] = rec_src[e];
#pragma unroll
            for (int i = 0; i < NO; ++i) of[u][i] = rec_off[8 * e + i];
        }
    };
    load_rec(e0, src, off);
    for (int eb = e0; eb < e1; eb += U) {
        float2 sv[U][RC];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float2 *Sr = S + ((int64_t)src[u] * R + r0) * K + kk;
#pragma unroll
            for (int c = 0; c < RC; ++c)
                sv[u][c] = (RC == 1 || c < rc) ? Sr[c * K] : make_float2(0.f, 0.f);
        }
        int nsrc[U], noff[U][NO];
        load_rec(eb + U < e1 ? eb + U : eb, nsrc, noff);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (eb + u < e1) {
#pragma unroll
                for (int i = 0; i < NO; ++i) {
                    const float2 tv = *(const float2 *)(Tsb + (off[u][i] + lane8));
#pragma unroll
                    for (int c = 0; c < RC; ++c) acc[i][c] = cfma(tv, sv[u][c], acc[i][c]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            src[u] = nsrc[u];
#pragma unroll
            for (int i = 0; i < NO; ++i) off[u][i] = noff[u][i];
        }
    }
}

template <int RC, int NW>
__global__ void __launch_bounds__(64 * NW)
k_m2l_rec(int64_t nparent, int64_t K, int ntypes, const int32_t *__restrict__ child_start,
          const int32_t *__restrict__ rec_start, const int32_t *__restrict__ rec_src,
          const int32_t *__restrict__ rec_off, const float2 *__restrict__ T,
          const float2 *__restrict__ S, int R, int nkc, int64_t ppb, int nwg,
          float2 *__restrict__ Lout)
{
    // Two schedules (about one workgroup per CU either way, so the LDS
    // staging of the operators is amortised over many parents):
    //  nwg == 0: workgroup w serves sample chunk w % nkc, right-hand-side
    //    chunk blockIdx.z and the contiguous parent range (w / nkc) * ppb
    //    ... + ppb; its NW waves take those parents round-robin.  (Numbering
    //    the workgroups so that each XCD gets a contiguous run of ranges
    //    measured slower at one RHS.)
    //  nwg > 0: slice-major sweep for many right-hand sides.  The nwg
    //    workgroups of one (sample chunk, RHS chunk) slice are consecutive,
    //    so the resident workgroups share a slice and sweep the parents
    //    interleaved (parent = (w nwg ... ) + wave): the sources they re-read
    //    stay within one window of the Morton order, small enough for the
    //    Infinity Cache, instead of every slice streaming at once.
    extern __shared__ float2 Ts[];  // [ntypes + 1][64], row ntypes = 0
    const int64_t w = nwg ? blockIdx.x % nwg : blockIdx.x;
    const int64_t slice = nwg ? blockIdx.x / nwg : 0;
    const int kc = nwg ? (int)(slice % nkc) : (int)(w % nkc);
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
    const int r0 = (nwg ? (int)(slice / nkc) : (int)blockIdx.z) * RC;
    const int rc = min(RC, R - r0);
    const int64_t pbeg = nwg ? w * NW : (w / nkc) * ppb;
    const int64_t pend = nwg ? nparent : min(nparent, pbeg + ppb);
    const int64_t pstep = nwg ? (int64_t)nwg * NW : NW;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int64_t P = pbeg + wave; P < pend; P += pstep) {
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
                   const float2 *T, const float2 *S, int R, float2 *Lout, hipStream_t s,
                   bool sweep)
{
    if (nparent == 0 || K == 0) return hipSuccess;
    const size_t lds = (size_t)(ntypes + 1) * 64 * sizeof(float2);
    if (lds > 163840) return hipErrorInvalidValue;
    // right-hand sides per thread: 1 or 4 (8 per thread, with 8 waves per
    // workgroup for the registers of 8 x 8 accumulators, measured slower at
    // 64 right-hand sides: 10.1 ms against 8.3 ms on the 262k sphere)
    const int RC = R == 1 ? 1 : 4;
    const int NW = 16;
    const int nkc = (int)((K + 63) / 64);
    const int nz = (R + RC - 1) / RC;
    dim3 grid;
    int64_t ppb = 0;
    int nwg = 0;
    if (sweep) {
        // one workgroup per CU per slice, slices one after the other
        nwg = (int)std::max<int64_t>(1, std::min<int64_t>(256, (nparent + NW - 1) / NW));
        grid = dim3((unsigned)(nwg * nkc * nz), 1, 1);
    } else {
        // about one workgroup per CU in all, at least one parent per wave
        const int64_t per = std::max<int64_t>(
            1, std::min<int64_t>((256 + nkc * nz - 1) / (nkc * nz), (nparent + NW - 1) / NW));
        ppb = (nparent + per - 1) / per;
        grid = dim3((unsigned)(nkc * ((nparent + ppb - 1) / ppb)), 1, (unsigned)nz);
    }
#define M2L_REC(RCV, NWV)                                                                      \
    hipLaunchKernelGGL((k_m2l_rec<RCV, NWV>), grid, dim3(64 * NWV), lds, s, nparent, K, ntypes, \
                       child_start, rec_start, rec_src, rec_off, T, S, R, nkc, ppb, nwg, Lout)
    if (RC == 1) M2L_REC(1, 16);
    else M2L_REC(4, 16);
#undef M2L_REC
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

}  // namespace dev
}  // namespace mlfma
