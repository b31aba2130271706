// One-pass interpolation (M2M, Sec. 3.2.2) and anterpolation (L2L,
// Sec. 3.2.4) between two adjacent levels.
//
// The exact band-limited map between two sample grids is the three real
// maps phi-DFT (F [nphi_in][M]), theta map per Fourier column
// (A_m [ntheta_in][ntheta_out]) and phi-synthesis (G [M][nphi_out]).  The
// staged path writes the two intermediates to HBM; here the three maps run
// back to back with the intermediates in LDS, so HBM sees only the input
// and the output spectra:
//
//   M2M  S_p[r]  = sum_c shift_c (.) Y3_c,  Y3_c = G^T A_m (S_c[r] F)
//   L2L  L_c[r] += G^T A_m ((conj(shift_c) (.) L_p[r]) F)
//
// The grids of a level pair are compile-time shapes (band L_child, band
// L_parent), so every loop is unrolled and every index is a constant or a
// per-lane offset.  Pairs without an instantiation take the staged path.
//
// Work split: a workgroup of NW waves stages the operators of the pair
// (zero-padded to whole MFMA tiles) and the three axis factors of the shift
// in LDS once; then every wave runs its own sequence of items (parent box,
// right-hand side, group of BW children) in a private LDS region with no
// workgroup barrier.  The input of the next item is loaded into registers
// while the current item computes.
//
// Each map is an MFMA product with the operator as the A operand (rows =
// output index) and the data as the B operand, whose columns run over
// (child, theta, re/im), so small per-box maps still fill 16-wide tiles:
//   s1   Y1[col][(b, theta_in, part)]      = F^T  X^T       K = nphi_in
//   s2   Y2[(b, col, theta_out, part)]     = A_m^T Y1       K = ntheta_in, per m,
//        columns (b, cos/sin column of m, part)
//   s3   Y3[phi_out][(b, theta_out, part)] = G^T  Y2^T      K = M
// The operators are zero beyond their true K, so B values read past a row
// end (finite data of the next row) contribute nothing.  M2M multiplies Y3
// by the child's shift (the re/im partner is the neighbouring lane) and sums
// over the children in registers; L2L adds Y3 into the child's local with
// one atomic add per value (a single writer per value, so the result does
// not depend on ordering).
//
// The shift of octant (bx, by, bz) is the product of three axis factors
// E_a = exp(-i k (a_l / 4) khat_a), conjugated where the octant bit is 0;
// E_x and E_y are tables over the parent grid, E_z over its theta nodes.
//
// MFMA v_mfma_f32_16x16x4_f32: lane l feeds A[l%16][l/16] and B[l/16][l%16]
// and receives D[4(l/16)+v][l%16], v = 0..3.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace mlfma {
namespace dev {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mma(float a, float b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Orders the LDS accesses of one wave: DS instructions of a wave execute in
// order, so only compiler reordering has to be prevented.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }
constexpr int up4(int x) { return (x + 3) & ~3; }
constexpr int up16(int x) { return (x + 15) & ~15; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }
// smallest y >= x with y = r (mod m): LDS pitches chosen against bank
// conflicts (32 banks of 4 bytes, 32 lanes per LDS pass)
constexpr int pad_to(int x, int r, int m) { return x + ((r - x % m) % m + m) % m; }

__device__ __forceinline__ float2 cmulf(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Compile-time shape of one level pair and direction.  LC, LP: bands of
// the child and parent levels; BW children per item; NW waves per group;
// MINW resident waves per SIMD.
template <int LC, int LP, bool DOWN_, int BW_, int NW_, int MINW_>
struct Shape {
    static constexpr bool DOWN = DOWN_;
    static constexpr int BW = BW_, NW = NW_;
    // resident waves per SIMD asked of the register allocator (two
    // workgroups per CU where the LDS plan allows it)
    static constexpr int MINW = MINW_;
    static constexpr int LI = DOWN ? LP : LC, LO = DOWN ? LC : LP;
    static constexpr int TI = LI + 1, PI = 2 * LI + 2, TO = LO + 1, PO = 2 * LO + 2;
    static constexpr int M = 2 * LC + 1, NM = LC + 1;
    static constexpr int KIN = TI * PI, KOUT = TO * PO;
    static constexpr int KP = DOWN ? KIN : KOUT, THP = DOWN ? TI : TO;
    // s1 (one spare operator row: the zero row that stands for the missing
    // sine column of m = 0)
    static constexpr int KS1 = cdiv(PI, 4), RT1 = cdiv(M + 1, 16), R1 = 16 * RT1;
    static constexpr int N1 = BW * 2 * TI, CT1 = cdiv(N1, 16), N1P = 16 * CT1;
    // s2
    static constexpr int KS2 = cdiv(TI, 4), RT2 = cdiv(TO, 16), TO16 = 16 * RT2;
    static constexpr int N2 = 4 * BW, CT2 = cdiv(N2, 16);
    static constexpr int MC = M + 1;  // Y2 columns per child incl. the zero column
    // s3
    static constexpr int KS3 = cdiv(M, 4), RT3 = cdiv(PO, 16), CT3 = up16(2 * TO) / 16;
    // LDS pitches: input rows (float2), Y1 rows, Y2 column rows and Y2
    // child blocks (floats), shift-factor rows (float2)
    static constexpr int XP = pad_to(PI, 2, 4);
    static constexpr int P1 = N1P + 4;
    static constexpr int P2 = pad_to(2 * TO16, 16, 32);
    static constexpr int YB = pad_to(MC * P2, 2, 32);
    static constexpr int PHP = DOWN ? PI : PO;  // parent grid phi samples
    static constexpr int EP = pad_to(PHP, 2, 4);
    // shared LDS (floats)
    static constexpr int F_SZ = 4 * KS1 * R1;
    static constexpr int A_SZ = NM * 4 * KS2 * TO16;
    static constexpr int G_SZ = 4 * KS3 * 16 * RT3;
    static constexpr int E_N = 2 * THP * EP + THP;  // float2: Ex, Ey [THP][EP], Ez [THP]
    static constexpr int O_F = 0, O_A = F_SZ, O_G = O_A + A_SZ, O_E = up4(O_G + G_SZ);
    static constexpr int O_W = up4(O_E + 2 * E_N);
    // per-wave LDS (floats): region 0 = input / Y2 / M2M output;
    // region 1 = Y1 / L2L output
    static constexpr int X_SZ = 2 * (DOWN ? 1 : BW) * TI * XP + 8;
    static constexpr int Y2_SZ = BW * YB;
    static constexpr int RG0 = up4(cmax(cmax(X_SZ, Y2_SZ), DOWN ? 0 : 2 * KOUT));
    static constexpr int RG1 = up4(cmax(R1 * P1, DOWN ? 2 * BW * KOUT : 0));
    static constexpr int WSZ = RG0 + RG1;
    static constexpr int TOTAL = O_W + NW * WSZ;  // floats
    // prefetched input values per lane
    static constexpr int XR = cdiv(DOWN ? KIN : BW * KIN, 64);
};

template <class S>
__global__ void __launch_bounds__(64 * S::NW, S::MINW)
k_onepass(const float2 *__restrict__ In, const int32_t *__restrict__ child_start,
          const uint8_t *__restrict__ child_oct, const float *__restrict__ F,
          const float *__restrict__ Am, const float *__restrict__ G,
          const float2 *__restrict__ E3, float2 *__restrict__ Out, int64_t nparent, int R)
{
    constexpr bool DOWN = S::DOWN;
    extern __shared__ float smem[];
    const int tid = threadIdx.x;
    float *Fs = smem + S::O_F, *As = smem + S::O_A, *Gs = smem + S::O_G;
    float2 *Es = (float2 *)(smem + S::O_E);
    // operators, zero-padded: Fs[k][row], As[m][k][row], Gs[k][row]
    for (int i = tid; i < S::F_SZ; i += blockDim.x) {
        const int k = i / S::R1, row = i - k * S::R1;
        Fs[i] = (k < S::PI && row < S::M) ? F[k * S::M + row] : 0.f;
    }
    for (int i = tid; i < S::A_SZ; i += blockDim.x) {
        const int mk = i / S::TO16, row = i - mk * S::TO16;
        const int m = mk / (4 * S::KS2), k = mk - m * (4 * S::KS2);
        As[i] = (k < S::TI && row < S::TO) ? Am[(m * S::TI + k) * S::TO + row] : 0.f;
    }
    for (int i = tid; i < S::G_SZ; i += blockDim.x) {
        const int k = i / (16 * S::RT3), row = i - k * (16 * S::RT3);
        Gs[i] = (k < S::M && row < S::PO) ? G[k * S::PO + row] : 0.f;
    }
    for (int i = tid; i < 2 * S::THP * S::EP; i += blockDim.x) {
        const int a = i / (S::THP * S::EP), rem = i - a * (S::THP * S::EP);
        const int th = rem / S::EP, ph = rem - th * S::EP;
        Es[i] = ph < S::PHP ? E3[a * S::KP + th * S::PHP + ph] : make_float2(0.f, 0.f);
    }
    for (int i = tid; i < S::THP; i += blockDim.x) Es[2 * S::THP * S::EP + i] = E3[2 * S::KP + i];
    // wave regions start zeroed: padding reads see finite values only
    for (int i = tid; i < S::NW * S::WSZ; i += blockDim.x) smem[S::O_W + i] = 0.f;
    __syncthreads();  // the only workgroup barrier

    // the wave index is uniform: tasks, child ranges and loop bounds stay
    // in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63, lr = lane & 15, lq = lane >> 4;
    float *W0 = smem + S::O_W + wave * S::WSZ;
    float *W1 = W0 + S::RG0;
    float2 *X = (float2 *)W0;  // M2M: inputs [b][TI][XP]; L2L: parent local [TI][XP]
    float *Y2 = W0;            // [b: YB][MC: P2][TO16][2]
    float *Y1 = W1;            // [R1][P1]
    float *R2 = W1;            // L2L: output staging [b][KOUT][2]
    const float2 *Ez = Es + 2 * S::THP * S::EP;

    // operator fragments of s1 (F^T) and s3 (G^T), read from LDS per use
    const float *a1p = Fs + lq * S::R1 + lr;
    const float *a3p = Gs + lq * (16 * S::RT3) + lr;

    const int64_t ntasks = nparent * R;
    const int64_t stride = (int64_t)gridDim.x * S::NW;
    int64_t task = (int64_t)blockIdx.x * S::NW + wave;
    if (task >= ntasks) return;

    // current item: task (P, r), children c0 + g0 .. c0 + g0 + nb - 1
    int64_t P = task / R;
    int r = (int)(task - P * R);
    int c0 = child_start[P], nch = child_start[P + 1] - c0, g0 = 0;
    // the next task and its child range, loaded one task ahead
    int64_t ntask = task + stride;
    int nc0 = 0, nnch = 0;
    if (ntask < ntasks) {
        const int64_t nP = ntask / R;
        nc0 = child_start[nP];
        nnch = child_start[nP + 1] - nc0;
    }
    float2 xr[S::XR];
    int octr = 0;  // lane b < nb: octant of child b of the item
    auto prefetch = [&](int64_t pP, int pr, int pc, int pnb) {
        if (!DOWN) {
#pragma unroll
            for (int i = 0; i < S::XR; ++i) {
                const int e = lane + 64 * i;
                const int b = e / S::KIN, j = e - b * S::KIN;
                if (b < pnb) xr[i] = In[((int64_t)(pc + b) * R + pr) * S::KIN + j];
            }
        } else {
            const float2 *src = In + ((int64_t)pP * R + pr) * S::KIN;
#pragma unroll
            for (int i = 0; i < S::XR; ++i) {
                const int e = lane + 64 * i;
                if (e < S::KIN) xr[i] = src[e];
            }
        }
        octr = lane < pnb ? child_oct[pc + lane] : 0;
    };
    prefetch(P, r, c0, min(S::BW, nch));

    floatx4 acc[S::CT3][S::RT3];
    for (;;) {
        const int nb = min(S::BW, nch - g0);
        const int cg = c0 + g0;
        if (!DOWN && g0 == 0) {
#pragma unroll
            for (int t = 0; t < S::CT3; ++t)
#pragma unroll
                for (int rt = 0; rt < S::RT3; ++rt) acc[t][rt] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
        // ---- the prefetched input into LDS
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < S::XR; ++i) {
            const int e = lane + 64 * i;
            const int b = e / S::KIN, j = e - b * S::KIN;
            const int th = j / S::PI, ph = j - th * S::PI;
            if (e < (DOWN ? S::KIN : nb * S::KIN)) X[(b * S::TI + th) * S::XP + ph] = xr[i];
        }
        const int oct_lane = octr;
        // ---- next item and its prefetch
        int64_t n_P = P;
        int n_r = r, n_c0 = c0, n_nch = nch, n_g0 = g0 + S::BW;
        bool n_valid = true, n_new = false;
        if (n_g0 >= nch) {
            n_new = true;
            n_g0 = 0;
            if (ntask < ntasks) {
                n_P = ntask / R;
                n_r = (int)(ntask - n_P * R);
                n_c0 = nc0;
                n_nch = nnch;
            } else {
                n_valid = false;
            }
        }
        if (n_valid) prefetch(n_P, n_r, n_c0 + n_g0, min(S::BW, n_nch - n_g0));
        wave_lds_sync();

        // ---- s1: Y1[col][n], n = (b, theta_in, part)
#pragma unroll
        for (int ct = 0; ct < S::CT1; ++ct) {
            const int n = ct * 16 + lr;
            const int bn = n / (2 * S::TI), j = n - bn * (2 * S::TI);
            const int b = bn < S::BW ? bn : 0;  // padding columns read child 0
            const int th = j >> 1, part = j & 1;
            floatx4 d[S::RT1];
#pragma unroll
            for (int rt = 0; rt < S::RT1; ++rt) d[rt] = floatx4{0.f, 0.f, 0.f, 0.f};
            if (!DOWN) {
                const float *xb = (const float *)X + ((b * S::TI + th) * S::XP + lq) * 2 + part;
#pragma unroll
                for (int ks = 0; ks < S::KS1; ++ks) {
                    const float bv = xb[8 * ks];
#pragma unroll
                    for (int rt = 0; rt < S::RT1; ++rt)
                        d[rt] = mma(a1p[4 * ks * S::R1 + rt * 16], bv, d[rt]);
                }
            } else {
                const int oc = __shfl(oct_lane, b, 64);
                float2 ez = Ez[th];
                if (oc & 1) ez.y = -ez.y;
                const int e0 = th * S::XP + lq;
#pragma unroll
                for (int ks = 0; ks < S::KS1; ++ks) {
                    const int e = e0 + 4 * ks;
                    // conj(shift) = factors E where the bit is 0, conj(E) where 1
                    float2 ex = Es[e], ey = Es[S::THP * S::EP + e];
                    if (oc & 4) ex.y = -ex.y;
                    if (oc & 2) ey.y = -ey.y;
                    const float2 z = cmulf(cmulf(ex, ey), cmulf(ez, X[e]));
                    const float bv = part ? z.y : z.x;
#pragma unroll
                    for (int rt = 0; rt < S::RT1; ++rt)
                        d[rt] = mma(a1p[4 * ks * S::R1 + rt * 16], bv, d[rt]);
                }
            }
#pragma unroll
            for (int rt = 0; rt < S::RT1; ++rt)
#pragma unroll
                for (int v = 0; v < 4; ++v) Y1[(rt * 16 + 4 * lq + v) * S::P1 + n] = d[rt][v];
        }
        wave_lds_sync();
        // ---- s2: per m, columns n = (b, cos/sin, part)
#pragma unroll
        for (int m = 0; m < S::NM; ++m) {
#pragma unroll
            for (int ct = 0; ct < S::CT2; ++ct) {
                const int n = ct * 16 + lr;
                const int bn = n >> 2, cs = (n >> 1) & 1, part = n & 1;
                const int b = bn < S::BW ? bn : 0;  // padding columns read child 0
                // row M of Y1 is zero: it stands for the sine column of m = 0
                const int col = m == 0 ? (cs ? S::M : 0) : 2 * m - 1 + cs;
                const float *yp = Y1 + col * S::P1 + b * 2 * S::TI + 2 * lq + part;
                const float *ap = As + (m * 4 * S::KS2 + lq) * S::TO16 + lr;
                floatx4 d[S::RT2];
#pragma unroll
                for (int rt = 0; rt < S::RT2; ++rt) d[rt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < S::KS2; ++ks) {
                    const float bv = yp[8 * ks];
#pragma unroll
                    for (int rt = 0; rt < S::RT2; ++rt)
                        d[rt] = mma(ap[4 * ks * S::TO16 + rt * 16], bv, d[rt]);
                }
                if (n < S::N2) {
                    float *dst = Y2 + b * S::YB + col * S::P2 + 8 * lq + part;
#pragma unroll
                    for (int rt = 0; rt < S::RT2; ++rt)
#pragma unroll
                        for (int v = 0; v < 4; ++v) dst[(rt * 16 + v) * 2] = d[rt][v];
                }
            }
        }
        wave_lds_sync();
        // ---- s3: Y3[phi_out][(theta_out, part)] per child
        for (int b = 0; b < nb; ++b) {
            floatx4 d[S::CT3][S::RT3];
#pragma unroll
            for (int t = 0; t < S::CT3; ++t)
#pragma unroll
                for (int rt = 0; rt < S::RT3; ++rt) d[t][rt] = floatx4{0.f, 0.f, 0.f, 0.f};
            // B[k = col][n = (theta_out, part)]: Y2[b][col][theta_out][part],
            // column t*16 + lr is float offset t*16 + lr within the row
            const float *yb = Y2 + b * S::YB + lq * S::P2 + lr;
#pragma unroll
            for (int ks = 0; ks < S::KS3; ++ks) {
                float av[S::RT3];
#pragma unroll
                for (int rt = 0; rt < S::RT3; ++rt) av[rt] = a3p[4 * ks * 16 * S::RT3 + rt * 16];
#pragma unroll
                for (int t = 0; t < S::CT3; ++t) {
                    const float bv = yb[4 * ks * S::P2 + t * 16];
#pragma unroll
                    for (int rt = 0; rt < S::RT3; ++rt) d[t][rt] = mma(av[rt], bv, d[t][rt]);
                }
            }
            const int oc = __shfl(oct_lane, b, 64);
            const int part = lr & 1;
#pragma unroll
            for (int t = 0; t < S::CT3; ++t) {
                const int tho = (t * 16 + lr) >> 1;
#pragma unroll
                for (int rt = 0; rt < S::RT3; ++rt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int ph = rt * 16 + 4 * lq + v;
                        const bool ok = tho < S::TO && ph < S::PO;
                        if (!DOWN) {
                            const float mine = d[t][rt][v];
                            const float other = __shfl_xor(mine, 1, 64);
                            if (ok) {
                                const int e = tho * S::EP + ph;
                                float2 ex = Es[e], ey = Es[S::THP * S::EP + e], ez = Ez[tho];
                                if (!(oc & 4)) ex.y = -ex.y;
                                if (!(oc & 2)) ey.y = -ey.y;
                                if (!(oc & 1)) ez.y = -ez.y;
                                const float2 sh = cmulf(cmulf(ex, ey), ez);
                                const float re = part ? other : mine;
                                const float im = part ? mine : other;
                                acc[t][rt][v] += part ? sh.x * im + sh.y * re : sh.x * re - sh.y * im;
                            }
                        } else if (ok) {
                            R2[(b * S::KOUT + tho * S::PO + ph) * 2 + part] = d[t][rt][v];
                        }
                    }
            }
        }
        wave_lds_sync();
        if (DOWN) {
            // add into the children's locals (single writer per value)
            for (int b = 0; b < nb; ++b) {
                float *dst = (float *)(Out + ((int64_t)(cg + b) * R + r) * S::KOUT);
                const float *src = R2 + b * S::KOUT * 2;
                for (int e = lane; e < 2 * S::KOUT; e += 64) atomicAdd(dst + e, src[e]);
            }
        } else if (g0 + S::BW >= nch) {
            // last group of the parent: write its spectrum through LDS
            float *St = W0;
            const int part = lr & 1;
#pragma unroll
            for (int t = 0; t < S::CT3; ++t) {
                const int tho = (t * 16 + lr) >> 1;
#pragma unroll
                for (int rt = 0; rt < S::RT3; ++rt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int ph = rt * 16 + 4 * lq + v;
                        if (tho < S::TO && ph < S::PO) St[(tho * S::PO + ph) * 2 + part] = acc[t][rt][v];
                    }
            }
            wave_lds_sync();
            float2 *dst = Out + ((int64_t)P * R + r) * S::KOUT;
            for (int e = lane; e < S::KOUT; e += 64) dst[e] = X[e];
        }
        // ---- advance
        if (!n_valid) break;
        if (n_new) {
            task = ntask;
            ntask = task + stride;
            if (ntask < ntasks) {
                const int64_t nP = ntask / R;
                nc0 = child_start[nP];
                nnch = child_start[nP + 1] - nc0;
            }
        }
        P = n_P;
        r = n_r;
        c0 = n_c0;
        nch = n_nch;
        g0 = n_g0;
    }
}

constexpr size_t kLdsPerCU = 163840;

template <class S>
hipError_t launch_shape(const float2 *In, const int32_t *child_start, const uint8_t *oct,
                        const float *F, const float *Am, const float *G, const float2 *E3,
                        float2 *Out, int64_t nparent, int R, hipStream_t st)
{
    static_assert((size_t)S::TOTAL * sizeof(float) <= kLdsPerCU, "LDS plan too large");
    const size_t lds = (size_t)S::TOTAL * sizeof(float);
    const int per_cu = std::max<int>(1, std::min<int>(kLdsPerCU / lds, 32 / S::NW));
    const int64_t nwg = (nparent * R + S::NW - 1) / S::NW;
    const unsigned grid = (unsigned)std::min<int64_t>(nwg, 256 * per_cu);
    hipLaunchKernelGGL(k_onepass<S>, dim3(grid), dim3(64 * S::NW), lds, st, In, child_start, oct,
                       F, Am, G, E3, Out, nparent, R);
    return hipGetLastError();
}

// The instantiated level pairs (the bands of a 0.25-wavelength leaf at 3
// digits and its parent), each in several work splits (children per item
// BW, waves per workgroup NW, resident waves per SIMD MINW) that trade LDS
// occupancy against MFMA tile fill: one child per item leaves 3/4 of the
// s2 tiles' columns empty, two children halve that.  The autotuner times
// them.
//   (8, 13):  0: BW 1, NW 8;  1: BW 2, NW 4 (two workgroups per CU);
//             2: BW 1, NW 4 (three workgroups per CU)
//   (13, 20): 0: BW 1, NW 8;  1: BW 2, NW 4
template <bool DOWN>
hipError_t dispatch(int Lc, int Lp, int shape, const float2 *In, const int32_t *cs,
                    const uint8_t *oct, const float *F, const float *Am, const float *G,
                    const float2 *E3, float2 *Out, int64_t nparent, int R, hipStream_t st)
{
    if (Lc == 8 && Lp == 13) {
        if (shape == 1)
            return launch_shape<Shape<8, 13, DOWN, 2, 4, 2>>(In, cs, oct, F, Am, G, E3, Out, nparent, R, st);
        if (shape == 2)
            return launch_shape<Shape<8, 13, DOWN, 1, 4, 3>>(In, cs, oct, F, Am, G, E3, Out, nparent, R, st);
        return launch_shape<Shape<8, 13, DOWN, 1, 8, 4>>(In, cs, oct, F, Am, G, E3, Out, nparent, R, st);
    }
    if (Lc == 13 && Lp == 20) {
        if (shape == 1)
            return launch_shape<Shape<13, 20, DOWN, 2, 4, 1>>(In, cs, oct, F, Am, G, E3, Out, nparent, R, st);
        return launch_shape<Shape<13, 20, DOWN, 1, 8, 2>>(In, cs, oct, F, Am, G, E3, Out, nparent, R, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

bool pair_onepass_fits(int Lc, int Lp) { return pair_onepass_shapes(Lc, Lp) > 0; }

int pair_onepass_shapes(int Lc, int Lp)
{
    if (Lc == 8 && Lp == 13) return 3;
    if (Lc == 13 && Lp == 20) return 2;
    return 0;
}

hipError_t interp_fused(int64_t nboxp, int R, int Lc, int Lp, int shape,
                        const int32_t *child_start, const uint8_t *child_oct, const float2 *Sc,
                        const float *F, const float *A, const float *G, const float2 *E3,
                        float2 *Sp, hipStream_t s)
{
    if (nboxp == 0) return hipSuccess;
    return dispatch<false>(Lc, Lp, shape, Sc, child_start, child_oct, F, A, G, E3, Sp, nboxp, R,
                           s);
}

hipError_t anterp_fused(int64_t nboxp, int R, int Lc, int Lp, int shape,
                        const int32_t *child_start, const uint8_t *child_oct, const float2 *Lpar,
                        const float *F, const float *B, const float *G, const float2 *E3,
                        float2 *Lch, hipStream_t s)
{
    if (nboxp == 0) return hipSuccess;
    return dispatch<true>(Lc, Lp, shape, Lpar, child_start, child_oct, F, B, G, E3, Lch, nboxp,
                          R, s);
}

}  // namespace dev
}  // namespace mlfma
