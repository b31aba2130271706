// Interpolation (M2M, Sec. 3.2.2) and anterpolation (L2L, Sec. 3.2.4) as
// dense contractions on the matrix cores (gfx950 MFMA).
//
// The exact band-limited map between two sample grids is three real
// matrices applied to complex spectra:
//   s1  phi-DFT       [rows = (box, rhs, theta_in)] x F [nphi_in x M]
//   s2  theta map     per Fourier column m: [rows = (box, rhs)] x A_m^T
//   s3  phi-synthesis [rows = (box, rhs, theta_out)] x G [M x nphi_out]
// Each stage is a "row GEMM": C[rows x N] = A[rows x K] * B[K x N] with A
// complex (data) and B real (operator).  The intermediates are written
// transposed so that every stage reads K-contiguous rows:
//   s1 writes T1[col][(box, rhs)][theta_in]
//   s2 writes T2[(box, rhs)][col][theta_out]
// M2M s3 fuses the shift exp(-ik khat.(c_c - c_p)) and the sum over the
// siblings (parent-centric, no atomics); L2L s1 fuses the conjugate shift of
// the parent's local expansion and L2L s3 adds into the child's local.
//
// MFMA mapping (v_mfma_f32_16x16x4_f32, D = A(16x4) B(4x16) + C): one wave
// computes 8 complex rows x 16 columns per instruction.  MFMA row 2t+h is
// the real (h=0) or imaginary (h=1) part of complex row t; lane l feeds
// A[l%16][l/16] and B[l/16][l%16] and receives D[4(l/16)+v][l%16], i.e. the
// complex values of rows 2(l/16) (v=0,1) and 2(l/16)+1 (v=2,3).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace mlfma {
namespace dev {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

static inline unsigned waves_to_blocks(int64_t waves) { return (unsigned)((waves + 3) / 4); }

// ------------------------------------------------------- problem types --
// M2M s1: rows (c, r, theta) of the child spectra, K = nphi_c, N = M.
struct ProbS1 {
    static constexpr bool rows_fast = false;
    const float2 *X;
    const float *F;
    float2 *out;
    int64_t nrows, BR;
    int K, N, nth;
    __device__ float2 a(int64_t row, int k) const { return X[row * K + k]; }
    struct Row {
        const float2 *x;
    };
    __device__ Row row_at(int64_t row) const { return Row{X + row * K}; }
    __device__ float2 at(const Row &w, int k) const { return w.x[k]; }
    __device__ float b(int k, int n) const { return F[k * N + n]; }
    __device__ void store(int64_t row, int n, float2 v) const
    {
        const int64_t cr = row / nth;
        const int th = (int)(row - cr * nth);
        out[((int64_t)n * BR + cr) * nth + th] = v;
    }
    __device__ void set_col(int) {}
};

// L2L s1: rows (c, r, theta_p); A = conj(shift[oct c]) * L_parent(c).
struct ProbS1L {
    static constexpr bool rows_fast = false;
    const float2 *Lp, *shift;
    const int32_t *parent;
    const uint8_t *oct;
    const float *F;
    float2 *out;
    int64_t nrows, BR, Kp;
    int K, N, nth, R;
    __device__ float2 a(int64_t row, int k) const
    {
        const int cr = (int)row / nth;
        const int th = (int)row - cr * nth;
        const int c = cr / R;
        const int r = cr - c * R;
        const float2 x = Lp[((int64_t)parent[c] * R + r) * Kp + th * K + k];
        const float2 s = shift[(int64_t)oct[c] * Kp + th * K + k];
        return make_float2(s.x * x.x + s.y * x.y, s.x * x.y - s.y * x.x);
    }
    // row (c, r, theta) decoded once; then K contiguous samples of the
    // parent's local and of the shift
    struct Row {
        const float2 *x, *s;
    };
    __device__ Row row_at(int64_t row) const
    {
        const int cr = (int)row / nth;
        const int th = (int)row - cr * nth;
        const int c = cr / R;
        const int r = cr - c * R;
        return Row{Lp + ((int64_t)parent[c] * R + r) * Kp + th * K,
                   shift + (int64_t)oct[c] * Kp + th * K};
    }
    __device__ float2 at(const Row &w, int k) const
    {
        const float2 x = w.x[k], s = w.s[k];
        return make_float2(s.x * x.x + s.y * x.y, s.x * x.y - s.y * x.x);
    }
    __device__ float b(int k, int n) const { return F[k * N + n]; }
    __device__ void store(int64_t row, int n, float2 v) const
    {
        const int64_t cr = row / nth;
        const int th = (int)(row - cr * nth);
        out[((int64_t)n * BR + cr) * nth + th] = v;
    }
    __device__ void set_col(int) {}
};

// s2 for one Fourier column `col`: rows (c, r), K = nth_in, N = nth_out,
// B(k, n) = mapsT[m][k][n].
struct ProbS2 {
    const float2 *T1;
    const float *maps;
    float2 *out;
    int64_t nrows;  // BR
    int K, N, M, col;
    __device__ float2 a(int64_t row, int k) const
    {
        return T1[((int64_t)col * nrows + row) * K + k];
    }
    struct Row {
        const float2 *x;
    };
    __device__ Row row_at(int64_t row) const { return Row{T1 + ((int64_t)col * nrows + row) * K}; }
    __device__ float2 at(const Row &w, int k) const { return w.x[k]; }
    __device__ float b(int k, int n) const
    {
        const int m = (col + 1) >> 1;
        return maps[((int64_t)m * K + k) * N + n];
    }
    __device__ void store(int64_t row, int n, float2 v) const
    {
        out[(row * M + col) * N + n] = v;
    }
    __device__ void set_col(int c) { col = c; }
    static constexpr bool rows_fast = false;
};

// L2L s3: rows (c, r, theta_c), K = M, N = nphi_c; adds into the local.
// T2 is [(c, r)][col][theta_c], so consecutive rows are contiguous for a
// fixed k (rows_fast: the LDS staging walks rows fastest).
struct ProbS3L {
    const float2 *T2;
    const float *G;
    float2 *Lc;
    int64_t nrows;
    int K, N, nth;
    static constexpr bool rows_fast = true;
    __device__ float2 a(int64_t row, int k) const
    {
        const int cr = (int)row / nth;
        const int th = (int)row - cr * nth;
        return T2[((int64_t)cr * K + k) * nth + th];
    }
    // row (c, r, theta) decoded once; sample k of it sits k * nth further
    struct Row {
        const float2 *x;
        int stride;
    };
    __device__ Row row_at(int64_t row) const
    {
        const int cr = (int)row / nth;
        const int th = (int)row - cr * nth;
        return Row{T2 + (int64_t)cr * K * nth + th, nth};
    }
    __device__ float2 at(const Row &w, int k) const { return w.x[(int64_t)k * w.stride]; }
    __device__ float b(int k, int n) const { return G[k * N + n]; }
    __device__ void store(int64_t row, int n, float2 v) const
    {
        float2 *p = Lc + row * N + n;
        float2 o = *p;
        o.x += v.x;
        o.y += v.y;
        *p = o;
    }
    __device__ void set_col(int) {}
};

// ------------------------------------------------ generic wave row GEMM --
// A workgroup of 4 waves takes 32 complex rows (8 per wave).  The real
// operator is staged in LDS once per workgroup, 16*NT columns at a time
// (NT chosen so that the staged block is <= 64 KB); the data rows stream
// from global memory, one float per lane per k-step.
__device__ __forceinline__ int64_t xcd_contiguous_i(int64_t bid, int64_t nb)
{
    const int64_t q = nb / 8, rem = nb % 8;
    const int64_t x = bid % 8, i = bid / 8;
    return x * q + (x < rem ? x : rem) + i;
}

template <class P, int NT>
__device__ __forceinline__ void wave_tile(const P &p, const float *Bs, int64_t row0, int n0,
                                          int lane)
{
    constexpr int NC = 16 * NT;
    const int t = (lane & 15) >> 1, part = lane & 1, kq = lane >> 4;
    const int64_t myrow = row0 + t;
    const bool rv = myrow < p.nrows;
    floatx4 acc[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
    int kb = 0;
    for (; kb + 8 <= p.K; kb += 8) {
        float av[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const float2 x = rv ? p.a(myrow, kb + 4 * u + kq) : make_float2(0.f, 0.f);
            av[u] = part ? x.y : x.x;
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int j = 0; j < NT; ++j)
                acc[j] = mfma4(av[u], Bs[(kb + 4 * u + kq) * NC + 16 * j + (lane & 15)], acc[j]);
    }
    for (; kb < p.K; kb += 4) {
        const int k = kb + kq;
        float av = 0.f;
        if (rv && k < p.K) {
            const float2 x = p.a(myrow, k);
            av = part ? x.y : x.x;
        }
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const float bv = k < p.K ? Bs[k * NC + 16 * j + (lane & 15)] : 0.f;
            acc[j] = mfma4(av, bv, acc[j]);
        }
    }
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int n = n0 + 16 * j + (lane & 15);
        if (n < p.N) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int64_t row = row0 + 2 * kq + h;
                if (row < p.nrows) p.store(row, n, make_float2(acc[j][2 * h], acc[j][2 * h + 1]));
            }
        }
    }
}

template <class P, int NT>
__device__ __forceinline__ void stage_b(const P &p, float *Bs, int n0)
{
    constexpr int NC = 16 * NT;
    for (int base = threadIdx.x; base < p.K * NC; base += 8 * blockDim.x) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = base + u * blockDim.x;
            const int k = idx / NC, n = idx - (idx / NC) * NC;
            v[u] = (idx < p.K * NC && n0 + n < p.N) ? p.b(k, n0 + n) : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = base + u * blockDim.x;
            if (idx < p.K * NC) Bs[idx] = v[u];
        }
    }
}

template <class P, int NT>
__global__ void __launch_bounds__(256) k_rowgemm(P p)
{
    extern __shared__ float Bs[];
    const int lane = threadIdx.x & 63;
    const int64_t blk = xcd_contiguous_i(blockIdx.x, gridDim.x);
    const int64_t row0 = (blk * 4 + (threadIdx.x >> 6)) * 8;
    for (int n0 = 0; n0 < p.N; n0 += 16 * NT) {
        __syncthreads();
        stage_b<P, NT>(p, Bs, n0);
        __syncthreads();
        if (row0 < p.nrows) wave_tile<P, NT>(p, Bs, row0, n0, lane);
    }
}

// s2: one Fourier column per blockIdx.y
template <int NT>
__global__ void __launch_bounds__(256) k_s2(ProbS2 p)
{
    extern __shared__ float Bs[];
    p.col = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 8;
    for (int n0 = 0; n0 < p.N; n0 += 16 * NT) {
        __syncthreads();
        stage_b<ProbS2, NT>(p, Bs, n0);
        __syncthreads();
        if (row0 < p.nrows) wave_tile<ProbS2, NT>(p, Bs, row0, n0, lane);
    }
}

// Same contraction with the data tile staged in LDS as well: a workgroup
// loops over tiles of 32 complex rows (grid-stride), copies each tile into
// LDS, and its 4 waves read their MFMA fragments from LDS.  The operator
// block is staged once per workgroup and column chunk (16*NT columns, NT =
// 1..8).  The loads of the next tile go to registers (at most 16 values a
// thread) before the MFMAs of the current one, so they are in flight while
// it computes.  Used when K <= 128; QMAX >= (K rounded up to 4) / 8.
template <class P, int NT, int QMAX>
__global__ void __launch_bounds__(256) k_rowgemm_lds(P p, int col_override)
{
    extern __shared__ float smem[];
    constexpr int NC = 16 * NT;
    const int K = p.K;
    const int K4 = (K + 3) & ~3;
    const int KP = K4 + 1;                    // row pitch in float2 (odd: spreads banks)
    const int nq = (K4 + 7) / 8;              // values per thread per tile
    float *Bs = smem;                         // [K4][NC]
    float2 *As = (float2 *)(smem + K4 * NC);  // [32][KP]
    if (col_override >= 0) p.set_col(col_override + blockIdx.y);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int t = (lane & 15) >> 1, part = lane & 1, kq = lane >> 4;
    const int64_t ntiles = (p.nrows + 31) / 32;
    float2 pre[QMAX];
    // rows_fast: thread value q is sample (tid >> 5) + 8 q of row tid & 31
    // (the tile walked rows fastest); else 8 threads per row, value q is
    // sample (tid & 7) + 8 q of row tid / 8; rows are decoded once
    auto load_tile = [&](int64_t tile) {
        const int64_t rbase = tile * 32;
        if (P::rows_fast) {
            const int64_t row = rbase + (tid & 31);
            const bool ok = row < p.nrows;
            const typename P::Row w = p.row_at(ok ? row : 0);
#pragma unroll
            for (int q = 0; q < QMAX; ++q) {
                const int k = (tid >> 5) + 8 * q;
                pre[q] = (q < nq && ok && k < K) ? p.at(w, k) : make_float2(0.f, 0.f);
            }
        } else {
            const int64_t row = rbase + (tid >> 3);
            const bool ok = row < p.nrows;
            const typename P::Row w = p.row_at(ok ? row : 0);
#pragma unroll
            for (int q = 0; q < QMAX; ++q) {
                const int k = (tid & 7) + 8 * q;
                pre[q] = (q < nq && ok && k < K) ? p.at(w, k) : make_float2(0.f, 0.f);
            }
        }
    };
    auto store_tile = [&]() {
#pragma unroll
        for (int q = 0; q < QMAX; ++q) {
            if (q >= nq) break;
            int k, rl;
            if (P::rows_fast) {
                k = (tid >> 5) + 8 * q;
                rl = tid & 31;
            } else {
                k = (tid & 7) + 8 * q;
                rl = tid >> 3;
            }
            if (k < K4) As[rl * KP + k] = pre[q];
        }
    };
    for (int n0 = 0; n0 < p.N; n0 += NC) {
        __syncthreads();
        for (int base = tid; base < K4 * NC; base += 8 * blockDim.x) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int idx = base + u * blockDim.x;
                const int k = idx / NC, n = idx - (idx / NC) * NC;
                v[u] = (idx < K4 * NC && k < K && n0 + n < p.N) ? p.b(k, n0 + n) : 0.f;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int idx = base + u * blockDim.x;
                if (idx < K4 * NC) Bs[idx] = v[u];
            }
        }
        int64_t tile = blockIdx.x;
        if (tile < ntiles) load_tile(tile);
        for (; tile < ntiles; tile += gridDim.x) {
            __syncthreads();  // the previous tile's MFMAs are done with As
            store_tile();
            __syncthreads();
            if (tile + gridDim.x < ntiles) load_tile(tile + gridDim.x);
            const int64_t row0 = tile * 32 + wave * 8;
            if (row0 >= p.nrows) continue;
            const float2 *arow = As + (wave * 8 + t) * KP;
            floatx4 acc[NT];
#pragma unroll
            for (int j = 0; j < NT; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
            for (int kb = 0; kb < K4; kb += 4) {
                const float2 x = arow[kb + kq];
                const float av = part ? x.y : x.x;
#pragma unroll
                for (int j = 0; j < NT; ++j)
                    acc[j] = mfma4(av, Bs[(kb + kq) * NC + 16 * j + (lane & 15)], acc[j]);
            }
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const int n = n0 + 16 * j + (lane & 15);
                if (n < p.N) {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int64_t row = row0 + 2 * kq + h;
                        if (row < p.nrows)
                            p.store(row, n, make_float2(acc[j][2 * h], acc[j][2 * h + 1]));
                    }
                }
            }
        }
    }
}

// ------------------------------------------------ BF16 split precision --
// The same contraction with each FP32 operand split x = hi + lo, hi =
// bf16(x), lo = bf16(x - hi), and the product taken as hi*hi + hi*lo +
// lo*hi on v_mfma_f32_16x16x32_bf16 with FP32 accumulation (relative error
// about 2^-16).  Lane l feeds A[l%16][8(l/16) .. 8(l/16)+7] and
// B[8(l/16) .. +7][l%16] and receives the same D layout as the FP32 path.
// LDS holds the data tile as hi/lo planes [32 rows x 2 parts][K32] and the
// operator as hi/lo planes [NC][K32] (transposed), so every fragment is one
// 16-byte LDS read.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned short bf16_bits_rn(float x)
{
    const unsigned u = __float_as_uint(x);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_bits_to_float(unsigned short b)
{
    return __uint_as_float((unsigned)b << 16);
}
__device__ __forceinline__ void split_bf16(float x, unsigned short &hi, unsigned short &lo)
{
    hi = bf16_bits_rn(x);
    lo = bf16_bits_rn(x - bf16_bits_to_float(hi));
}

// four values split at once: hi and lo as 4 packed bf16 each (one 8-byte
// LDS store per plane; gfx950 converts pairs)
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void split_bf16x4(const float (&x)[4], uint2 &h, uint2 &l)
{
    bf16x4 hb;
#pragma unroll
    for (int e = 0; e < 4; ++e) hb[e] = (__bf16)x[e];
    const uint2 hu = __builtin_bit_cast(uint2, hb);
    bf16x4 lb;
    lb[0] = (__bf16)(x[0] - __uint_as_float(hu.x << 16));
    lb[1] = (__bf16)(x[1] - __uint_as_float(hu.x & 0xffff0000u));
    lb[2] = (__bf16)(x[2] - __uint_as_float(hu.y << 16));
    lb[3] = (__bf16)(x[3] - __uint_as_float(hu.y & 0xffff0000u));
    h = hu;
    l = __builtin_bit_cast(uint2, lb);
}

template <class P, int NT>
__global__ void __launch_bounds__(256) k_rowgemm_bf16x3(P p, int col_override)
{
    extern __shared__ unsigned short sm16[];
    constexpr int NC = 16 * NT;
    const int K = p.K;
    const int K32 = (K + 31) & ~31;
    const int KP = K32 + 8;                       // row pitch (bf16): +16 B spreads banks
    unsigned short *Bh = sm16;                    // [NC][KP]
    unsigned short *Bl = Bh + NC * KP;
    unsigned short *Ah = Bl + NC * KP;            // [64][KP]: row 2t+part
    unsigned short *Al = Ah + 64 * KP;
    if (col_override >= 0) p.set_col(col_override + blockIdx.y);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kq = lane >> 4, i16 = lane & 15;
    const int64_t ntiles = (p.nrows + 31) / 32;
    for (int n0 = 0; n0 < p.N; n0 += NC) {
        __syncthreads();
        for (int base = threadIdx.x; base < K32 * NC; base += 4 * blockDim.x) {
            float v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int idx = base + u * blockDim.x;
                const int n = idx / K32, k = idx - (idx / K32) * K32;
                v[u] = (idx < K32 * NC && k < K && n0 + n < p.N) ? p.b(k, n0 + n) : 0.f;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int idx = base + u * blockDim.x;
                if (idx < K32 * NC) {
                    const int n = idx / K32, k = idx - (idx / K32) * K32;
                    unsigned short h, l;
                    split_bf16(v[u], h, l);
                    Bh[n * KP + k] = h;
                    Bl[n * KP + k] = l;
                }
            }
        }
        for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
            const int64_t rbase = tile * 32;
            __syncthreads();
            // the tile's 32 complex rows as hi/lo planes: each thread takes
            // 4 consecutive k of one row (real and imaginary rows 2t, 2t + 1)
            if (P::rows_fast) {
                // rows fastest across threads (consecutive rows are
                // contiguous in memory for a fixed k)
                const int rl = threadIdx.x & 31;
                const int64_t row = rbase + rl;
                const bool ok = row < p.nrows;
                for (int k0 = 4 * (threadIdx.x >> 5); k0 < K32; k0 += 4 * (blockDim.x >> 5)) {
                    float re[4], im[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float2 v = (ok && k0 + e < K) ? p.a(row, k0 + e)
                                                            : make_float2(0.f, 0.f);
                        re[e] = v.x;
                        im[e] = v.y;
                    }
                    uint2 h, l;
                    split_bf16x4(re, h, l);
                    *(uint2 *)(Ah + (2 * rl) * KP + k0) = h;
                    *(uint2 *)(Al + (2 * rl) * KP + k0) = l;
                    split_bf16x4(im, h, l);
                    *(uint2 *)(Ah + (2 * rl + 1) * KP + k0) = h;
                    *(uint2 *)(Al + (2 * rl + 1) * KP + k0) = l;
                }
            } else {
                // 8 threads per row, row decoded once
                const int rl = threadIdx.x >> 3;
                const int64_t row = rbase + rl;
                const bool ok = row < p.nrows;
                const typename P::Row w = p.row_at(ok ? row : 0);
                for (int k0 = 4 * (threadIdx.x & 7); k0 < K32; k0 += 32) {
                    float re[4], im[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float2 v = (ok && k0 + e < K) ? p.at(w, k0 + e)
                                                            : make_float2(0.f, 0.f);
                        re[e] = v.x;
                        im[e] = v.y;
                    }
                    uint2 h, l;
                    split_bf16x4(re, h, l);
                    *(uint2 *)(Ah + (2 * rl) * KP + k0) = h;
                    *(uint2 *)(Al + (2 * rl) * KP + k0) = l;
                    split_bf16x4(im, h, l);
                    *(uint2 *)(Ah + (2 * rl + 1) * KP + k0) = h;
                    *(uint2 *)(Al + (2 * rl + 1) * KP + k0) = l;
                }
            }
            __syncthreads();
            const int64_t row0 = rbase + wave * 8;
            if (row0 >= p.nrows) continue;
            const int arow = wave * 16 + i16;     // real row 2t+part of this wave
            floatx4 acc[NT];
#pragma unroll
            for (int j = 0; j < NT; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
            for (int kb = 0; kb < K32; kb += 32) {
                const int kk = kb + 8 * kq;
                const bf16x8 ah = *(const bf16x8 *)(Ah + arow * KP + kk);
                const bf16x8 al = *(const bf16x8 *)(Al + arow * KP + kk);
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    const int n = 16 * j + i16;
                    const bf16x8 bh = *(const bf16x8 *)(Bh + n * KP + kk);
                    const bf16x8 bl = *(const bf16x8 *)(Bl + n * KP + kk);
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[j], 0, 0, 0);
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[j], 0, 0, 0);
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[j], 0, 0, 0);
                }
            }
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const int n = n0 + 16 * j + i16;
                if (n < p.N) {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int64_t row = row0 + 2 * kq + h;
                        if (row < p.nrows)
                            p.store(row, n, make_float2(acc[j][2 * h], acc[j][2 * h + 1]));
                    }
                }
            }
        }
    }
}

static size_t lds_bytes_bf16x3(int K, int nt)
{
    const int KP = ((K + 31) & ~31) + 8;
    return (size_t)(2 * 16 * nt * KP + 2 * 64 * KP) * sizeof(unsigned short);
}

static size_t lds_bytes_rowgemm(int K, int nt)
{
    const int K4 = (K + 3) & ~3;
    return (size_t)K4 * 16 * nt * sizeof(float) + (size_t)32 * (K4 + 1) * sizeof(float2);
}

// column tiles per pass: enough for N, and K x 16 NT floats <= 64 KB
static int pick_nt(int K, int N)
{
    int nt = 1;
    while (nt < 8 && 16 * nt < N) nt <<= 1;
    while (nt > 1 && (size_t)K * 16 * nt * sizeof(float) > 65536) nt >>= 1;
    return nt;
}

template <class P>
static hipError_t launch_rowgemm(const P &p, hipStream_t s, int gridy = 1, int col0 = -1,
                                 bool bf16x3 = false)
{
    if (p.nrows == 0) return hipSuccess;
    if (bf16x3 && p.K <= 256) {
        int nt = 1;
        while (nt < 8 && 16 * nt < p.N) nt <<= 1;
        while (nt > 1 && lds_bytes_bf16x3(p.K, nt) > 81920) nt >>= 1;
        const int64_t ntiles = (p.nrows + 31) / 32;
        const unsigned gx = (unsigned)std::min<int64_t>(ntiles, 2048 / gridy + 1);
        dim3 grid(gx, gridy), block(256);
        const size_t lds = lds_bytes_bf16x3(p.K, nt);
        switch (nt) {
        case 1: hipLaunchKernelGGL((k_rowgemm_bf16x3<P, 1>), grid, block, lds, s, p, col0); break;
        case 2: hipLaunchKernelGGL((k_rowgemm_bf16x3<P, 2>), grid, block, lds, s, p, col0); break;
        case 4: hipLaunchKernelGGL((k_rowgemm_bf16x3<P, 4>), grid, block, lds, s, p, col0); break;
        default: hipLaunchKernelGGL((k_rowgemm_bf16x3<P, 8>), grid, block, lds, s, p, col0); break;
        }
        return hipGetLastError();
    }
    if (p.K <= 128) {
        // column tiles: as many as N needs (at most 8, several passes
        // beyond), fewer while the LDS exceeds 80 KB (two workgroups per CU)
        int nt = std::min(8, (p.N + 15) / 16);
        while (nt > 1 && lds_bytes_rowgemm(p.K, nt) > 81920) --nt;
        const int64_t ntiles = (p.nrows + 31) / 32;
        const unsigned gx = (unsigned)std::min<int64_t>(ntiles, 2048 / gridy + 1);
        dim3 grid(gx, gridy), block(256);
        const size_t lds = lds_bytes_rowgemm(p.K, nt);
        // staging registers per thread: (K rounded up to 4) / 8, in classes
        const int nq = (((p.K + 3) & ~3) + 7) / 8;
        const int q = nq <= 4 ? 4 : nq <= 8 ? 8 : 16;
#define ROWGEMM_LDS(NTV, QV) \
    hipLaunchKernelGGL((k_rowgemm_lds<P, NTV, QV>), grid, block, lds, s, p, col0)
#define ROWGEMM_LDS_NT(QV)                     \
    switch (nt) {                              \
    case 1: ROWGEMM_LDS(1, QV); break;         \
    case 2: ROWGEMM_LDS(2, QV); break;         \
    case 3: ROWGEMM_LDS(3, QV); break;         \
    case 4: ROWGEMM_LDS(4, QV); break;         \
    case 5: ROWGEMM_LDS(5, QV); break;         \
    case 6: ROWGEMM_LDS(6, QV); break;         \
    case 7: ROWGEMM_LDS(7, QV); break;         \
    default: ROWGEMM_LDS(8, QV); break;        \
    }
        if (q == 4) { ROWGEMM_LDS_NT(4) }
        else if (q == 8) { ROWGEMM_LDS_NT(8) }
        else { ROWGEMM_LDS_NT(16) }
#undef ROWGEMM_LDS_NT
#undef ROWGEMM_LDS
        return hipGetLastError();
    }
    const int64_t waves = (p.nrows + 7) / 8;
    const int nt = pick_nt(p.K, p.N);
    dim3 grid(waves_to_blocks(waves)), block(256);
    const size_t lds = (size_t)p.K * 16 * nt * sizeof(float);
    switch (nt) {
    case 1: hipLaunchKernelGGL((k_rowgemm<P, 1>), grid, block, lds, s, p); break;
    case 2: hipLaunchKernelGGL((k_rowgemm<P, 2>), grid, block, lds, s, p); break;
    case 4: hipLaunchKernelGGL((k_rowgemm<P, 4>), grid, block, lds, s, p); break;
    default: hipLaunchKernelGGL((k_rowgemm<P, 8>), grid, block, lds, s, p); break;
    }
    return hipGetLastError();
}

// M2M s3: one wave per (parent p, rhs r, block of 8 theta' rows, chunk of
// 16*NT phi' columns); the 4 waves of a workgroup share the column chunk,
// whose slice of the synthesis matrix G (zero rows past M) is staged in
// LDS.  The wave walks its children in steps of 4*MKB orders: the lane
// loads all MKB of its A values of a step (one float each: the real or the
// imaginary part of the child's row) one step ahead, so the loads of the
// next step (possibly the next child's) are in flight during the MFMAs of
// this one; a child's shift values are requested at its first step and
// applied after its last, accumulating the parent in registers.
template <int NT, int MKB>
__global__ void __launch_bounds__(256)
k_m2m_s3(const float2 *__restrict__ T2, const float *__restrict__ G,
         const float2 *__restrict__ shift, const int32_t *__restrict__ child_start,
         const uint8_t *__restrict__ child_oct, float2 *__restrict__ Sp, int64_t nboxp,
         int R, int nthp, int nphp, int M)
{
    extern __shared__ float Gs[];
    constexpr int NC = 16 * NT;
    constexpr int KS = 4 * MKB;  // orders per step
    const int lane = threadIdx.x & 63;
    const int nch = (nphp + NC - 1) / NC;
    const int nkb = (M + KS - 1) / KS;  // steps per child
    const int MP = nkb * KS;            // staged rows (zeros past M)
    const int64_t blk = xcd_contiguous_i(blockIdx.x, gridDim.x);
    const int chunk = (int)(blk % nch);
    const int n0 = chunk * NC;
    const int64_t wave = (blk / nch) * 4 + (threadIdx.x >> 6);
    const int ntb = (nthp + 7) / 8;
    for (int base = threadIdx.x; base < MP * NC; base += 8 * blockDim.x) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = base + u * blockDim.x;
            const int k = idx / NC, n = idx - (idx / NC) * NC;
            v[u] = (idx < MP * NC && k < M && n0 + n < nphp) ? G[k * nphp + n0 + n] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = base + u * blockDim.x;
            if (idx < MP * NC) Gs[idx] = v[u];
        }
    }
    __syncthreads();
    if (wave >= nboxp * R * ntb) return;
    const int tb = (int)(wave % ntb);
    const int64_t pr = wave / ntb;
    const int r = (int)(pr % R);
    const int64_t p = pr / R;
    const int64_t Kp = (int64_t)nthp * nphp;
    const int t = (lane & 15) >> 1, part = lane & 1, kq = lane >> 4;
    const int th_a = tb * 8 + t;
    const bool rv = th_a < nthp;
    const int c0 = child_start[p], c1 = child_start[p + 1];
    const int nsteps = (c1 - c0) * nkb;
    float2 par[NT][2];
#pragma unroll
    for (int j = 0; j < NT; ++j) par[j][0] = par[j][1] = make_float2(0.f, 0.f);
    if (nsteps == 0) {
        float2 *out = Sp + (p * R + r) * Kp;
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int n = n0 + 16 * j + (lane & 15);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int th = tb * 8 + 2 * kq + h;
                if (n < nphp && th < nthp) out[(int64_t)th * nphp + n] = par[j][h];
            }
        }
        return;
    }
    auto load_step = [&](int st, float (&a)[MKB]) {
        const int c = c0 + st / nkb;
        const int kb0 = (st % nkb) * KS;
        const float *A = (const float *)(T2 + ((int64_t)c * R + r) * M * nthp + th_a) + part;
#pragma unroll
        for (int u = 0; u < MKB; ++u) {
            const int k = kb0 + 4 * u + kq;
            a[u] = (rv && k < M) ? A[2 * (int64_t)k * nthp] : 0.f;
        }
    };
    float2 sv[NT][2];
    auto load_shift = [&](int c) {
        const float2 *sh = shift + (int64_t)child_oct[c] * Kp;
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int n = n0 + 16 * j + (lane & 15);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int th = tb * 8 + 2 * kq + h;
                sv[j][h] = (n < nphp && th < nthp) ? sh[(int64_t)th * nphp + n] : make_float2(0.f, 0.f);
            }
        }
    };
    floatx4 acc[NT];
    auto compute = [&](int st, const float (&a)[MKB]) {
        const int kb0 = (st % nkb) * KS;
        if (kb0 == 0) {
#pragma unroll
            for (int j = 0; j < NT; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
            // narrow chunks: the shift values in flight during the MFMAs
            // (wide ones load them after, to keep their registers free)
            if constexpr (NT <= 2) load_shift(c0 + st / nkb);
        }
#pragma unroll
        for (int u = 0; u < MKB; ++u)
#pragma unroll
            for (int j = 0; j < NT; ++j)
                acc[j] = mfma4(a[u], Gs[(kb0 + 4 * u + kq) * NC + 16 * j + (lane & 15)], acc[j]);
        if (kb0 + KS >= M) {
            if constexpr (NT > 2) load_shift(c0 + st / nkb);
#pragma unroll
            for (int j = 0; j < NT; ++j)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const float yr = acc[j][2 * h], yi = acc[j][2 * h + 1];
                    par[j][h].x += sv[j][h].x * yr - sv[j][h].y * yi;
                    par[j][h].y += sv[j][h].x * yi + sv[j][h].y * yr;
                }
        }
    };
    float a0[MKB], a1[MKB];
    load_step(0, a0);
    for (int st = 0;;) {
        if (st + 1 < nsteps) load_step(st + 1, a1);
        compute(st, a0);
        if (++st >= nsteps) break;
        if (st + 1 < nsteps) load_step(st + 1, a0);
        compute(st, a1);
        if (++st >= nsteps) break;
    }
    float2 *out = Sp + (p * R + r) * Kp;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int n = n0 + 16 * j + (lane & 15);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int th = tb * 8 + 2 * kq + h;
            if (n < nphp && th < nthp) out[(int64_t)th * nphp + n] = par[j][h];
        }
    }
}

// ------------------------------------------------------------ launchers --
hipError_t interp_s1(const float2 *Sc, int64_t BR, int nthc, int nphc, const float *F, int M,
                     float2 *T1, hipStream_t s, bool bf16x3)
{
    ProbS1 p{Sc, F, T1, BR * nthc, BR, nphc, M, nthc};
    return launch_rowgemm(p, s, 1, -1, bf16x3);
}

hipError_t anterp_s1(const float2 *Lp, const int32_t *parent, const uint8_t *oct, int64_t nchild,
                     int R, int nthp, int nphp, const float2 *shift, const float *F, int M,
                     float2 *T1, hipStream_t s, bool bf16x3)
{
    ProbS1L p{Lp, shift, parent, oct, F, T1, nchild * R * nthp, nchild * R,
              (int64_t)nthp * nphp, nphp, M, nthp, R};
    return launch_rowgemm(p, s, 1, -1, bf16x3);
}

hipError_t theta_map(const float2 *T1, int64_t BR, int nin, int M, const float *mapsT, int nout,
                     float2 *T2, hipStream_t s, bool bf16x3)
{
    if (BR == 0) return hipSuccess;
    ProbS2 p{T1, mapsT, T2, BR, nin, nout, M, 0};
    if (nin <= 128 || (bf16x3 && nin <= 256)) return launch_rowgemm(p, s, M, 0, bf16x3);
    const int64_t waves = (BR + 7) / 8;
    dim3 grid(waves_to_blocks(waves), M), block(256);
    const int nt = pick_nt(nin, nout);
    const size_t lds = (size_t)nin * 16 * nt * sizeof(float);
    switch (nt) {
    case 1: hipLaunchKernelGGL((k_s2<1>), grid, block, lds, s, p); break;
    case 2: hipLaunchKernelGGL((k_s2<2>), grid, block, lds, s, p); break;
    case 4: hipLaunchKernelGGL((k_s2<4>), grid, block, lds, s, p); break;
    default: hipLaunchKernelGGL((k_s2<8>), grid, block, lds, s, p); break;
    }
    return hipGetLastError();
}

hipError_t interp_s3(int64_t nboxp, int R, int nthp, int nphp, int M, const int32_t *child_start,
                     const uint8_t *child_oct, const float2 *T2, const float *G,
                     const float2 *shift, float2 *Sp, hipStream_t s)
{
    const int64_t waves = nboxp * R * ((nthp + 7) / 8);
    if (waves == 0) return hipSuccess;
    // widest column chunk that still gives >= 2048 waves (and fits 64 KB)
    // orders per step: one step per child up to 68 orders
    const int mkb = M <= 20 ? 5 : M <= 28 ? 7 : M <= 44 ? 11 : 17;
    const int mp = (M + 4 * mkb - 1) / (4 * mkb) * 4 * mkb;
    // column chunks of 16 NT (NT = 1..8, as even as nphp allows): the
    // fewest chunks that give >= 2048 waves and keep the slice <= 64 KB
    int nch = 1, nt = 8;
    for (;; ++nch) {
        nt = (nphp + 16 * nch - 1) / (16 * nch);
        if (nt > 8) continue;
        if ((size_t)mp * 16 * nt * sizeof(float) > 65536 && nt > 1) continue;
        if (waves * nch >= 2048 || nt == 1) break;
    }
    nch = (nphp + 16 * nt - 1) / (16 * nt);  // the chunk count the kernel derives
    dim3 grid((unsigned)(waves_to_blocks(waves) * nch)), block(256);
    const size_t lds = (size_t)mp * 16 * nt * sizeof(float);
#define M2M_S3(NTV, MKBV)                                                                        \
    hipLaunchKernelGGL((k_m2m_s3<NTV, MKBV>), grid, block, lds, s, T2, G, shift, child_start,    \
                       child_oct, Sp, nboxp, R, nthp, nphp, M)
#define M2M_S3_NT(MKBV)                  \
    switch (nt) {                        \
    case 1: M2M_S3(1, MKBV); break;      \
    case 2: M2M_S3(2, MKBV); break;      \
    case 3: M2M_S3(3, MKBV); break;      \
    case 4: M2M_S3(4, MKBV); break;      \
    case 5: M2M_S3(5, MKBV); break;      \
    case 6: M2M_S3(6, MKBV); break;      \
    case 7: M2M_S3(7, MKBV); break;      \
    default: M2M_S3(8, MKBV); break;     \
    }
    switch (mkb) {
    case 5: M2M_S3_NT(5); break;
    case 7: M2M_S3_NT(7); break;
    case 11: M2M_S3_NT(11); break;
    default: M2M_S3_NT(17); break;
    }
#undef M2M_S3_NT
#undef M2M_S3
    return hipGetLastError();
}

hipError_t anterp_s3(int64_t nboxc, int R, int nthc, int nphc, int M, const float2 *T2,
                     const float *G, float2 *Lc, hipStream_t s, bool bf16x3)
{
    ProbS3L p{T2, G, Lc, nboxc * R * nthc, M, nphc, nthc};
    return launch_rowgemm(p, s, 1, -1, bf16x3);
}

}  // namespace dev
}  // namespace mlfma
