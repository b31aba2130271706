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
// One workgroup of NW waves per work item (a target leaf, or a chunk of 64
// of its points).  The near sources are staged in LDS in batches of 256,
// their positions moved into the target leaf's frame (leaf-local offset +
// exact integer leaf offset x leaf side, which keeps FP32 accuracy for close
// pairs far from the origin).  With nt targets the 64 NW lanes form
// G = 64 NW / T groups (T = nt rounded up to a power of two): lane (g, t)
// takes target t and every G-th staged source; the partial sums of a target
// are added with cross-lane shuffles inside each wave and through LDS across
// the waves (fixed order, so the result does not depend on timing).
template <int RC, bool FIELD, int NW>
__global__ void __launch_bounds__(64 * NW)
k_p2p(const int2 *__restrict__ items, const float4 *__restrict__ pts,
      const int32_t *__restrict__ pt_start, const int32_t *__restrict__ near_start,
      const int32_t *__restrict__ near_idx, const int32_t *__restrict__ coord, float leaf,
      float kw, const float2 *__restrict__ qs, int R, float2 *__restrict__ out)
{
    constexpr int NA = FIELD ? 3 : 1;
    constexpr int CH = 256;
    constexpr int NT = 64 * NW;
    const float kwt = kw * 0.159154943f;  // wavenumber in turns per unit length
    __shared__ float4 sp[CH];
    __shared__ float2 sq[CH * RC];
    const int tid = threadIdx.x;
    const int2 it = items[blockIdx.x];
    const int b = it.x;
    const int p0 = pt_start[b];
    const int nt = min(64, pt_start[b + 1] - p0 - it.y);
    // lanes: target t = lane % nt, source group lane / nt of GW = 64 / nt
    // groups per wave (lanes past GW nt idle); G groups in all
    const int GW = 64 / nt;
    const int G = NW * GW;
    const int lane_ = tid & 63;
    const int t = lane_ % nt;
    const bool active = lane_ < GW * nt;
    const int g = (tid >> 6) * GW + lane_ / nt;
    const int i = p0 + it.y + t;
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
        for (int x = active ? g : n; x < n; x += G) {
            const float4 sj = sp[x];
            const float dx = pi.x - sj.x, dy = pi.y - sj.y, dz = pi.z - sj.z;
            const float r2 = dx * dx + dy * dy + dz * dz;
            // coincident point (self): r2 == 0 contributes nothing
            const float rinv = rsq_or_zero(r2);
            float sn, cs;
            sincos_turns(kwt * (r2 * rinv), &sn, &cs);
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

    // stage the near sources CH at a time.  The metadata of the (at most 27)
    // near leaves go to a table in LDS first (one load per lane, an
    // exclusive prefix of their point counts by shuffles); a staging slot
    // then finds its leaf by binary search in the table, and all slots'
    // loads of a chunk are issued together.
    __shared__ int nb_excl[32], nb_first[32];
    __shared__ float4 nb_off[32];
    __shared__ int nb_total;
    const int e0 = near_start[b];
    const int nn = min(32, near_start[b + 1] - e0);
    if (tid < 64) {
        int cnt = 0, first = 0;
        float4 off = make_float4(0.f, 0.f, 0.f, 0.f);
        if (tid < nn) {
            const int nb = near_idx[e0 + tid];
            first = pt_start[nb];
            cnt = pt_start[nb + 1] - first;
            off = make_float4((float)(coord[3 * nb] - cbx) * leaf,
                              (float)(coord[3 * nb + 1] - cby) * leaf,
                              (float)(coord[3 * nb + 2] - cbz) * leaf, 0.f);
        }
        int inc = cnt;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int v = __shfl_up(inc, d, 64);
            if (tid >= d) inc += v;
        }
        if (tid < 32) {
            nb_excl[tid] = tid < nn ? inc - cnt : 0x7fffffff;
            nb_first[tid] = first;
            nb_off[tid] = off;
        }
        if (tid == 63) nb_total = inc;
    }
    __syncthreads();
    const int total = nb_total;
    constexpr int SPT = CH / NT;  // staging slots per thread
    for (int c0 = 0; c0 < total; c0 += CH) {
        const int n = min(CH, total - c0);
        float4 pv[SPT];
        float2 qv[SPT][RC];
        int slot[SPT];
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            slot[u] = tid + u * NT;
            const int gidx = c0 + slot[u];
            int e = 0;
#pragma unroll
            for (int st = 16; st >= 1; st >>= 1)
                if (nb_excl[e + st] <= gidx) e += st;
            const bool ok = slot[u] < n;
            const int j = ok ? nb_first[e] + (gidx - nb_excl[e]) : 0;
            const float4 o = nb_off[e];
            const float4 pj = ok ? pts[j] : make_float4(0.f, 0.f, 0.f, 0.f);
            pv[u] = make_float4(pj.x + o.x, pj.y + o.y, pj.z + o.z, 0.f);
#pragma unroll
            for (int c = 0; c < RC; ++c)
                qv[u][c] = (ok && c < rc) ? qs[(int64_t)j * R + r0 + c] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            if (slot[u] < n) {
                sp[slot[u]] = pv[u];
#pragma unroll
                for (int c = 0; c < RC; ++c) sq[slot[u] * RC + c] = qv[u][c];
            }
        }
        process(n);
    }
    // add the partial sums of each target: lanes t + k nt of every wave,
    // through LDS; lane t < nt of wave 0 then holds the total of target t
    __shared__ float2 red[NW * 64 * RC * NA];  // [NW][64][RC][NA]
    {
        const int wv = tid >> 6;
#pragma unroll
        for (int c = 0; c < RC; ++c)
#pragma unroll
            for (int a = 0; a < NA; ++a) red[((wv * 64 + lane_) * RC + c) * NA + a] = acc[c][a];
    }
    __syncthreads();
    if (tid < nt) {
#pragma unroll
        for (int c = 0; c < RC; ++c)
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                float2 v = make_float2(0.f, 0.f);
                for (int w = 0; w < NW; ++w)
                    for (int k = 0; k < GW; ++k) {
                        const float2 u = red[((w * 64 + t + k * nt) * RC + c) * NA + a];
                        v.x += u.x;
                        v.y += u.y;
                    }
                acc[c][a] = v;
            }
#pragma unroll
        for (int c = 0; c < RC; ++c)
            if (c < rc)
#pragma unroll
                for (int a = 0; a < NA; ++a)
                    out[((int64_t)i * R + r0 + c) * NA + a] = acc[c][a];
    }
}

template <int RC, int NW>
static void p2p_launch(const int2 *items, int64_t nitems, const float4 *pts,
                       const int32_t *pt_start, const int32_t *near_start,
                       const int32_t *near_idx, const int32_t *coord, float leaf, float kw,
                       const float2 *qs, int R, int field, float2 *out, hipStream_t s)
{
    if (nitems == 0) return;
    dim3 grid((unsigned)nitems, (R + RC - 1) / RC);
    if (field)
        hipLaunchKernelGGL((k_p2p<RC, true, NW>), grid, dim3(64 * NW), 0, s, items, pts,
                           pt_start, near_start, near_idx, coord, leaf, kw, qs, R, out);
    else
        hipLaunchKernelGGL((k_p2p<RC, false, NW>), grid, dim3(64 * NW), 0, s, items, pts,
                           pt_start, near_start, near_idx, coord, leaf, kw, qs, R, out);
}

// heavy items (dense leaves: hundreds of points) with four waves each, the
// rest with one
template <int RC>
static hipError_t p2p_rc(const int2 *items, int64_t nitems, int64_t nheavy, const float4 *pts,
                         const int32_t *pt_start, const int32_t *near_start,
                         const int32_t *near_idx, const int32_t *coord, float leaf, float kw,
                         const float2 *qs, int R, int field, float2 *out, hipStream_t s)
{
    constexpr int NWH = RC <= 4 ? 4 : 1;
    p2p_launch<RC, NWH>(items, nheavy, pts, pt_start, near_start, near_idx, coord, leaf, kw, qs,
                        R, field, out, s);
    p2p_launch<RC, 1>(items + nheavy, nitems - nheavy, pts, pt_start, near_start, near_idx,
                      coord, leaf, kw, qs, R, field, out, s);
    return hipGetLastError();
}

// P2P for 8..64 right-hand sides (potential) on the matrix cores: per work
// item (a target leaf or a 64-point chunk of it), targets in tiles of 16 and
// near sources in tiles of 64: the 256 threads build the Green's function
// tile G[t][s] = e^{ikr}/r (0 for coincident points) in LDS, then wave w
// multiplies it into right-hand sides 16w .. 16w+15 (columns) with the
// sources as the reduction:  re += G_re q_re - G_im q_im,
// im += G_re q_im + G_im q_re.  Source positions are moved into the target
// leaf's frame exactly as in k_p2p.
__global__ void __launch_bounds__(256)
k_p2p_mfma(const int2 *__restrict__ items, const float4 *__restrict__ pts,
           const int32_t *__restrict__ pt_start, const int32_t *__restrict__ near_start,
           const int32_t *__restrict__ near_idx, const int32_t *__restrict__ coord, float leaf,
           float kw, const float2 *__restrict__ qs, int R, float2 *__restrict__ out)
{
    typedef float f4 __attribute__((ext_vector_type(4)));
    const float kwt = kw * 0.159154943f;  // wavenumber in turns per unit length
    __shared__ float4 sp[64];
    __shared__ int sid[64];
    __shared__ float4 tp[16];
    __shared__ float Gs[16 * 128];  // [target][G_re for 64 sources | G_im for 64 sources]
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63, lr = lane & 15, lq = lane >> 4;
    const int2 it = items[blockIdx.x];
    const int b = it.x;
    const int p0 = pt_start[b] + it.y;
    const int nt = min(64, pt_start[b + 1] - p0);
    const int cbx = coord[3 * b], cby = coord[3 * b + 1], cbz = coord[3 * b + 2];
    const int e_beg = near_start[b], e_end = near_start[b + 1];
    const int r = wave * 16 + lr;
    const bool rv = r < R;
    for (int t0 = 0; t0 < nt; t0 += 16) {
        __syncthreads();
        if (tid < 16) tp[tid] = t0 + tid < nt ? pts[p0 + t0 + tid] : make_float4(0.f, 0.f, 0.f, 0.f);
        f4 dre = {0.f, 0.f, 0.f, 0.f}, dim = dre;
        int e = e_beg, j = e < e_end ? pt_start[near_idx[e]] : 0;
        for (;;) {
            // ---- the next tile of up to 64 near sources
            __syncthreads();
            int fill = 0;
            while (fill < 64 && e < e_end) {
                const int nb = near_idx[e];
                const int j1 = pt_start[nb + 1];
                const int cnt = min(64 - fill, j1 - j);
                if (tid < cnt) {
                    const float4 pj = pts[j + tid];
                    sp[fill + tid] = make_float4(pj.x + (float)(coord[3 * nb] - cbx) * leaf,
                                                 pj.y + (float)(coord[3 * nb + 1] - cby) * leaf,
                                                 pj.z + (float)(coord[3 * nb + 2] - cbz) * leaf, 0.f);
                    sid[fill + tid] = j + tid;
                }
                fill += cnt;
                j += cnt;
                if (j >= j1) {
                    ++e;
                    if (e < e_end) j = pt_start[near_idx[e]];
                }
            }
            if (fill == 0) break;
            __syncthreads();
            for (int i = tid; i < 16 * 64; i += blockDim.x) {
                const int t = i >> 6, sx = i & 63;
                float gr = 0.f, gi = 0.f;
                if (t0 + t < nt && sx < fill) {
                    const float4 pi = tp[t], sj = sp[sx];
                    const float dx = pi.x - sj.x, dy = pi.y - sj.y, dz = pi.z - sj.z;
                    const float r2 = dx * dx + dy * dy + dz * dz;
                    const float rinv = rsq_or_zero(r2);
                    float sn, cs;
                    sincos_turns(kwt * (r2 * rinv), &sn, &cs);
                    gr = cs * rinv;
                    gi = sn * rinv;
                }
                Gs[t * 128 + sx] = gr;
                Gs[t * 128 + 64 + sx] = gi;
            }
            __syncthreads();
            if (wave * 16 >= R) continue;
            const float *Gr = Gs + lr * 128, *Gi = Gr + 64;
#pragma unroll
            for (int ks = 0; ks < 16; ++ks) {
                const int sx = ks * 4 + lq;
                const float2 x = (rv && sx < fill) ? qs[(int64_t)sid[sx] * R + r]
                                                   : make_float2(0.f, 0.f);
                const float ar = Gr[sx], ai = Gi[sx];
                dre = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, x.x, dre, 0, 0, 0);
                dre = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, -x.y, dre, 0, 0, 0);
                dim = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, x.y, dim, 0, 0, 0);
                dim = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, x.x, dim, 0, 0, 0);
            }
        }
        if (rv) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int t = t0 + 4 * lq + v;
                if (t < nt) out[(int64_t)(p0 + t) * R + r] = make_float2(dre[v], dim[v]);
            }
        }
    }
}

hipError_t p2p(const int2 *items, int64_t nitems, int64_t nheavy, const float4 *pts,
               const int32_t *pt_start,
               const int32_t *near_start, const int32_t *near_idx, const int32_t *coord,
               float leaf, float kw, const float2 *qs, int R, int field, float2 *out,
               hipStream_t s)
{
    if (nitems == 0) return hipSuccess;
    if (!field && R >= 8 && R <= 64) {
        hipLaunchKernelGGL(k_p2p_mfma, dim3((unsigned)nitems), dim3(256), 0, s, items, pts,
                           pt_start, near_start, near_idx, coord, leaf, kw, qs, R, out);
        return hipGetLastError();
    }
#define P2P_RC(RCV) \
    return p2p_rc<RCV>(items, nitems, nheavy, pts, pt_start, near_start, near_idx, coord, leaf, \
                       kw, qs, R, field, out, s)
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
    const float kwt = kw * 0.159154943f;  // wavenumber in turns per unit length
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
        for (int j0 = p0; j0 < p1; j0 += (int)blockDim.x) {
            const int nj = min((int)blockDim.x, p1 - j0);
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
                const float ph = -kwt * (kh.x * d.x + kh.y * d.y + kh.z * d.z);
                float sn, cs;
                sincos_turns(ph, &sn, &cs);
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

// C2M for 8..64 right-hand sides on the matrix cores: per leaf box
// S[r][k] = sum_p F[p][k] q[p][r], F[p][k] = e^{-i kw khat_k.d_p}; rows are
// samples (up to 12 tiles of 16), columns right-hand sides, the reduction
// runs over the box's points in tiles of 16 (phase tile in LDS, shared by
// the 4 waves; wave w takes right-hand sides 16w .. 16w+15).  Complex as
// real MFMAs: re += F_re q_re - F_im q_im, im += F_re q_im + F_im q_re.
constexpr int kC2mRowTiles = 12;

__global__ void __launch_bounds__(256)
k_c2m_mfma(const float4 *__restrict__ pts, const int32_t *__restrict__ pt_start,
           const float4 *__restrict__ khat_w, int K, float kw, const float2 *__restrict__ qs,
           int R, float2 *__restrict__ S)
{
    const float kwt = kw * 0.159154943f;  // wavenumber in turns per unit length
    typedef float f4 __attribute__((ext_vector_type(4)));
    extern __shared__ float Fs[];  // [16][2K]: F_re in columns 0..K-1, F_im in K..2K-1
    const int64_t b = blockIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, lr = lane & 15, lq = lane >> 4;
    const int p0 = pt_start[b], np = pt_start[b + 1] - p0;
    const int nrt = (K + 15) / 16;
    const int r = wave * 16 + lr;
    const bool rv = r < R;
    f4 dre[kC2mRowTiles], dim[kC2mRowTiles];
#pragma unroll
    for (int t = 0; t < kC2mRowTiles; ++t) dre[t] = dim[t] = f4{0.f, 0.f, 0.f, 0.f};
    __shared__ float4 Pt[16];  // the points of the tile
    for (int t0 = 0; t0 < np; t0 += 16) {
        __syncthreads();
        if (threadIdx.x < 16)
            Pt[threadIdx.x] = t0 + (int)threadIdx.x < np ? pts[p0 + t0 + threadIdx.x]
                                                        : make_float4(0.f, 0.f, 0.f, 0.f);
        __syncthreads();
        // thread = sample k: one direction load, 16 phases from the staged points
        for (int k = threadIdx.x; k < K; k += blockDim.x) {
            const float4 kh = khat_w[k];
#pragma unroll 4
            for (int p = 0; p < 16; ++p) {
                const float4 d = Pt[p];
                float sn, cs;
                sincos_turns(-kwt * (kh.x * d.x + kh.y * d.y + kh.z * d.z), &sn, &cs);
                const bool pv = t0 + p < np;
                Fs[p * 2 * K + k] = pv ? cs : 0.f;
                Fs[p * 2 * K + K + k] = pv ? sn : 0.f;
            }
        }
        __syncthreads();
        if (wave * 16 >= R) continue;
#pragma unroll
        for (int ps = 0; ps < 4; ++ps) {
            const int p = ps * 4 + lq;
            const float2 x = (rv && t0 + p < np) ? qs[(int64_t)(p0 + t0 + p) * R + r]
                                                 : make_float2(0.f, 0.f);
            const float *Fr = Fs + p * 2 * K, *Fi = Fr + K;
#pragma unroll
            for (int t = 0; t < kC2mRowTiles; ++t) {
                if (t < nrt) {
                    const int k = t * 16 + lr;
                    const float ar = k < K ? Fr[k] : 0.f, ai = k < K ? Fi[k] : 0.f;
                    dre[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, x.x, dre[t], 0, 0, 0);
                    dre[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, -x.y, dre[t], 0, 0, 0);
                    dim[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, x.y, dim[t], 0, 0, 0);
                    dim[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, x.x, dim[t], 0, 0, 0);
                }
            }
        }
    }
    if (!rv) return;
    float2 *Sr = S + (b * R + r) * K;
#pragma unroll
    for (int t = 0; t < kC2mRowTiles; ++t) {
        if (t < nrt) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int k = t * 16 + 4 * lq + v;
                if (k < K) Sr[k] = make_float2(dre[t][v], dim[t][v]);
            }
        }
    }
}

hipError_t c2m(const float4 *pts, const int32_t *pt_start, int64_t nleaf,
               const float4 *khat_w, int64_t K, float kw, const float2 *qs, int R,
               float2 *S, hipStream_t s)
{
    if (nleaf == 0) return hipSuccess;
    if (R >= 8 && R <= 64 && K <= 16 * kC2mRowTiles) {
        const size_t lds = (size_t)16 * 2 * K * sizeof(float);
        hipLaunchKernelGGL(k_c2m_mfma, dim3((unsigned)nleaf), dim3(256), lds, s, pts, pt_start,
                           khat_w, (int)K, kw, qs, R, S);
        return hipGetLastError();
    }
    // one thread per sample: whole waves up to 256 threads (162 leaf samples
    // take 3 waves, not 4)
    const dim3 blk((unsigned)std::min<int64_t>(256, (K + 63) / 64 * 64));
    if (R == 1) {
        hipLaunchKernelGGL(k_c2m<1>, dim3((unsigned)nleaf, 1), blk, 0, s, pts, pt_start,
                           khat_w, K, kw, qs, R, S);
    } else if (R <= 4) {
        hipLaunchKernelGGL(k_c2m<4>, dim3((unsigned)nleaf, 1), blk, 0, s, pts,
                           pt_start, khat_w, K, kw, qs, R, S);
    } else {
        hipLaunchKernelGGL(k_c2m<16>, dim3((unsigned)nleaf, (R + 15) / 16), blk, 0, s, pts,
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
    const float kwt = kw * 0.159154943f;  // wavenumber in turns per unit length
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
        // samples in batches of 8: the batch's loads are issued together
        // (a missing right-hand side re-reads the first and is not added)
        auto sample = [&](const float4 &kh, const float2 (&lv)[RC]) {
            float sn, cs;
            sincos_turns(kwt * (kh.x * d.x + kh.y * d.y + kh.z * d.z), &sn, &cs);
            const float2 e = make_float2(cs * kh.w, sn * kh.w);
#pragma unroll
            for (int c = 0; c < RC; ++c) {
                const float2 v = cmul(e, lv[c]);
                const float m = c < rc ? 1.f : 0.f;
                if (FIELD) {
                    const float kd[3] = {kh.x * m, kh.y * m, kh.z * m};
#pragma unroll
                    for (int a = 0; a < NA; ++a) {
                        acc[c][a].x = fmaf(v.x, kd[a], acc[c][a].x);
                        acc[c][a].y = fmaf(v.y, kd[a], acc[c][a].y);
                    }
                } else {
                    acc[c][0].x = fmaf(v.x, m, acc[c][0].x);
                    acc[c][0].y = fmaf(v.y, m, acc[c][0].y);
                }
            }
        };
        int64_t k = 0;
        for (; k + 8 <= K; k += 8) {
            float4 kh[8];
            float2 lv[8][RC];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                kh[u] = khat_w[k + u];
#pragma unroll
                for (int c = 0; c < RC; ++c) lv[u][c] = Lb[(c < rc ? c : 0) * K + k + u];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) sample(kh[u], lv[u]);
        }
        for (; k < K; ++k) {
            float2 lv[RC];
#pragma unroll
            for (int c = 0; c < RC; ++c) lv[c] = Lb[(c < rc ? c : 0) * K + k];
            sample(khat_w[k], lv);
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

// L2O for many right-hand sides as a per-leaf product on the matrix cores:
// far[p][r] = (i kw / 4 pi) sum_k E[p][k] L[b][r][k], E[p][k] = w_k e^{i kw khat.d_p}.
// One workgroup per leaf box; its points in tiles of 16 rows.  The 4 waves
// share the phase tile E (LDS, computed once per tile) and take chunks of 16
// right-hand sides.  Complex product as real MFMAs: with x = L[r][k],
//   re += E_re x_re - E_im x_im,  im += E_re x_im + E_im x_re,
// so per k step two A fragments (E_re, E_im) and one complex load of L.
// Lane l of v_mfma_f32_16x16x4_f32 feeds A[l%16][l/16], B[l/16][l%16] and
// receives D[4(l/16)+v][l%16]: rows are points, columns right-hand sides.
typedef float l2o_floatx4 __attribute__((ext_vector_type(4)));

template <typename Tout>
__global__ void __launch_bounds__(256)
k_l2o_mfma(const float4 *__restrict__ pts, const int32_t *__restrict__ pt_start,
           const int32_t *__restrict__ perm, const float4 *__restrict__ khat_w, int K, float kw,
           const float2 *__restrict__ L, const float2 *__restrict__ near, int R, int conj_out,
           Tout *__restrict__ out)
{
    const float kwt = kw * 0.159154943f;  // wavenumber in turns per unit length
    extern __shared__ float Es[];  // [16][2K]: E_re in columns 0..K-1, E_im in K..2K-1
    __shared__ float4 Pt[16];      // the points of the tile
    const int64_t b = blockIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, lr = lane & 15, lq = lane >> 4;
    const int p0 = pt_start[b], np = pt_start[b + 1] - p0;
    const int nchunk = (R + 15) / 16;
    const float sc = kw * kInv4Pi;
    for (int t0 = 0; t0 < np; t0 += 16) {
        __syncthreads();
        if (threadIdx.x < 16)
            Pt[threadIdx.x] = t0 + (int)threadIdx.x < np ? pts[p0 + t0 + threadIdx.x]
                                                        : make_float4(0.f, 0.f, 0.f, 0.f);
        __syncthreads();
        // thread = sample k: one direction load, 16 phases from the staged points
        for (int k = threadIdx.x; k < K; k += blockDim.x) {
            const float4 kh = khat_w[k];
#pragma unroll 4
            for (int p = 0; p < 16; ++p) {
                const float4 d = Pt[p];
                float sn, cs;
                sincos_turns(kwt * (kh.x * d.x + kh.y * d.y + kh.z * d.z), &sn, &cs);
                const bool pv = t0 + p < np;
                Es[p * 2 * K + k] = pv ? cs * kh.w : 0.f;
                Es[p * 2 * K + K + k] = pv ? sn * kh.w : 0.f;
            }
        }
        __syncthreads();
        const float *Ere = Es + lr * 2 * K, *Eim = Ere + K;
        for (int ch = wave; ch < nchunk; ch += 4) {
            const int r = ch * 16 + lr;
            const bool rv = r < R;
            const float2 *Lr = L + (b * R + (rv ? r : 0)) * K;
            l2o_floatx4 dre = {0.f, 0.f, 0.f, 0.f}, dim = dre;
            // the locals stream from L2 in batches of 8 k steps, the next
            // batch in flight while the current one runs on the matrix cores
            constexpr int B = 8;
            float2 xa[B], xb[B];
            auto load = [&](float2 (&x)[B], int kb) {
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    const int k = kb + 4 * u + lq;
                    x[u] = (rv && k < K) ? Lr[k] : make_float2(0.f, 0.f);
                }
            };
            auto run = [&](const float2 (&x)[B], int kb) {
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    const int k = kb + 4 * u + lq;
                    const float are = k < K ? Ere[k] : 0.f, aim = k < K ? Eim[k] : 0.f;
                    dre = __builtin_amdgcn_mfma_f32_16x16x4f32(are, x[u].x, dre, 0, 0, 0);
                    dre = __builtin_amdgcn_mfma_f32_16x16x4f32(aim, -x[u].y, dre, 0, 0, 0);
                    dim = __builtin_amdgcn_mfma_f32_16x16x4f32(are, x[u].y, dim, 0, 0, 0);
                    dim = __builtin_amdgcn_mfma_f32_16x16x4f32(aim, x[u].x, dim, 0, 0, 0);
                }
            };
            int kb = 0;
            load(xa, 0);
            for (; kb + 4 * B < K; kb += 8 * B) {
                load(xb, kb + 4 * B);
                run(xa, kb);
                if (kb + 8 * B < K) load(xa, kb + 8 * B);
                run(xb, kb + 4 * B);
            }
            if (kb < K) run(xa, kb);
            if (!rv) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int p = t0 + 4 * lq + v;
                if (p < np) {
                    const int64_t sidx = p0 + p;
                    // (i kw / 4 pi) (re + i im)
                    float2 o = near[sidx * R + r];
                    o.x += -sc * dim[v];
                    o.y += sc * dre[v];
                    if (conj_out) o.y = -o.y;
                    Tout &dst = out[(int64_t)perm[sidx] * R + r];
                    dst.x = o.x;
                    dst.y = o.y;
                }
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

hipError_t l2o_leaf_mfma(const float4 *pts, const int32_t *pt_start, int64_t nleaf,
                         const int32_t *perm, const float4 *khat_w, int64_t K, float kw,
                         const float2 *L, const float2 *near, int R, int conj_out, int dtype,
                         void *out, hipStream_t s)
{
    if (nleaf == 0) return hipSuccess;
    const size_t lds = (size_t)16 * 2 * K * sizeof(float);
    if (lds > 163840) return hipErrorInvalidValue;
    if (dtype == 0)
        hipLaunchKernelGGL(k_l2o_mfma<float2>, dim3((unsigned)nleaf), dim3(256), lds, s, pts,
                           pt_start, perm, khat_w, (int)K, kw, L, near, R, conj_out,
                           (float2 *)out);
    else
        hipLaunchKernelGGL(k_l2o_mfma<double2>, dim3((unsigned)nleaf), dim3(256), lds, s, pts,
                           pt_start, perm, khat_w, (int)K, kw, L, near, R, conj_out,
                           (double2 *)out);
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
