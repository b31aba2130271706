// Fused level-pair interpolation (M2M, Sec. 3.2.2) and anterpolation (L2L,
// Sec. 3.2.4): the three maps of a level pair, the shift and the sum over
// siblings (M2M) or the add into the child's local (L2L) in one launch, a
// workgroup of NW waves working together on a tile of parent boxes.
//
// Per item (child c, right-hand side r) the exact band-limited map is
//   s1  Y1[col][theta_in]    = sum_phi  X[theta_in][phi] F[phi][col]
//   s2  Y2[col][theta_out]   = sum_theta A_|m(col)|[theta_in][theta_out] Y1[col][theta_in]
//   s3  Y3[theta_out][phi_o] = sum_col  Y2[col][theta_out] G[col][phi_o]
// with X the child's multipole (M2M) or conj(shift_c) (.) the parent's
// local (L2L, on the parent grid), and
//   M2M  S_p = sum_{c of p} shift_c (.) Y3_c        (written)
//   L2L  L_c += Y3_c                                 (read-modify-write)
// The tile is a run of whole parents with at most NB = 8 children, so the
// sibling sum never leaves the workgroup and a child's local has exactly
// one writer; a host-built descriptor per tile names its parents, children,
// the octant of each child and the first child of each parent.
//
// Every map is an MFMA product (v_mfma_f32_16x16x4_f32; lane l feeds
// A[l%16][l/16], B[l/16][l%16] and receives D[4(l/16)+v][l%16]).  The data
// of all items of the tile are stacked along the free dimension, so the
// small per-box maps still fill 16-wide tiles:
//   s1  rows (item, theta_in, re/im) x K = phi_in   x N = col         (A = data)
//   s2  rows theta_out x K = theta_in x N = (item, cos/sin, re/im)     (B = data)
//   s3  rows (theta_out, re/im) x K = col x N = phi_out                (A = data)
// In s1 and s3 a row pair (2t, 2t + 1) is the real and imaginary part of
// one complex row, so the complex shift of the epilogue needs no lane
// exchange.  The operators are host-built fragment tables in lane order
// (zero past their true extent): s1 and s3 sit in registers for the whole
// kernel, s2 streams from L1.  LDS holds the tile's input (region A), the
// first intermediate (region B), the second (region A again: the input is
// dead once s1 is done; its padding columns meet zero operator rows) and
// the three axis factors of the shift (its value for an octant is their
// product, each conjugated where the octant bit is 0).  The next tile's
// description and input are loaded into registers while the current tile
// computes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "kernels.h"

namespace mlfma {
namespace dev {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mma(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }
// input row pitch (float2): PI if PI = 2 (mod 4), else PI + 2, so that the
// 8 rows x 2 parts x 2 k-quads of a half-wave s1 read hit distinct banks
constexpr int xpitch(int pi) { return (pi % 4 == 2) ? pi : pi + 2; }

template <int LC_, int LP_, bool DOWN_, int NB_, int NW_>
struct PairShape {
    static constexpr bool DOWN = DOWN_;
    static constexpr int LC = LC_, LP = LP_, NB = NB_, NW = NW_;
    static_assert(NB % 8 == 0, "item slots come in groups of 8");
    static constexpr int SG = NB / 8;                 // slot groups
    // input and output grids (M2M: child -> parent; L2L: parent -> child)
    static constexpr int LI = DOWN ? LP : LC, LO = DOWN ? LC : LP;
    static constexpr int TI = LI + 1, PI = 2 * LI + 2, TO = LO + 1, PO = 2 * LO + 2;
    static constexpr int KI = TI * PI, KO = TO * PO;
    // the parent grid (where the shift lives)
    static constexpr int TP = LP + 1, PP = 2 * LP + 2, KP = TP * PP;
    static constexpr int M = 2 * LC + 1, NM = LC + 1;
    static constexpr int KS1 = cdiv(PI, 4), CT1 = cdiv(M, 16), RT1 = TI * SG;
    static constexpr int KS2 = cdiv(TI, 4), RT2 = cdiv(TO, 16), TIP = 4 * KS2;
    static constexpr int KS3 = cdiv(M, 4), MP = 4 * KS3, RT3 = cdiv(2 * TO, 16), CT3 = cdiv(PO, 16);
    // LDS layouts (floats).  X: [slot][TI][XP] complex; Y1: [col][theta_in:
    // TIP][slot][part] with a theta stride = 16 (mod 32) and an odd column
    // stride; Y2: [slot][col: MP][theta_out][part]
    static constexpr int XP = xpitch(PI), XS = TI * XP * 2, X_SZ = NB * XS;
    static constexpr int Y1T = 2 * NB + ((2 * NB) % 32 == 16 ? 0 : 16);
    static constexpr int Y1C = TIP * Y1T + 1, Y1_SZ = M * Y1C;
    static constexpr int Y2T = 2 * TO, Y2S = MP * Y2T, Y2_SZ = NB * Y2S;
    static constexpr int A_SZ = cmax(X_SZ, Y2_SZ);
    static constexpr int E_SZ = (2 * KP + TP) * 2;    // axis factors of the shift
    static constexpr int LDS_FLOATS = A_SZ + Y1_SZ + E_SZ;
    static constexpr int NF1 = CT1 * KS1 * 64, NF2 = NM * RT2 * KS2 * 64, NF3 = CT3 * KS3 * 64;
    static constexpr int NT = 64 * NW;
    static constexpr int XR = cdiv(NB * KI, NT);      // prefetched input values per thread
};

// shift of octant oc on parent-grid sample (th, k): the axis factors, each
// conjugated where the octant bit is 0 (conj = true: the conjugate shift,
// conjugated where the bit is 1)
__device__ __forceinline__ float2 octant_shift(const float2 *ex, const float2 *ey,
                                               const float2 *ez, int oc, int th, int k, bool conj)
{
    float2 a = ex[k], b = ey[k], c = ez[th];
    const bool fx = ((oc & 4) != 0) == conj, fy = ((oc & 2) != 0) == conj,
               fz = ((oc & 1) != 0) == conj;
    if (fx) a.y = -a.y;
    if (fy) b.y = -b.y;
    if (fz) c.y = -c.y;
    const float2 ab = make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
    return make_float2(ab.x * c.x - ab.y * c.y, ab.x * c.y + ab.y * c.x);
}

// Tile descriptors (host-built, NB = 8 slots): d0 = (first parent, first
// child, children, parents); d1 = (octant of slot i at bits 3i, first slot
// of parent j = 1..7 at bits 4(j-1), parent of slot i at bits 3i, 0).
template <class S>
__global__ void __launch_bounds__(64 * S::NW)
k_pair(const float2 *__restrict__ In, float2 *__restrict__ Out, const int4 *__restrict__ desc,
       int64_t ntiles, int R, const float *__restrict__ fr1, const float *__restrict__ fr2,
       const float *__restrict__ fr3, const float2 *__restrict__ shift_axis,
       const float2 *__restrict__ shift)
{
    static_assert(S::NB == 8, "tile descriptors pack 8 slots");
    constexpr bool DOWN = S::DOWN;
    constexpr int NT = S::NT;
    extern __shared__ float smem[];
    float *RA = smem;               // X, then Y2
    float *Y1 = smem + S::A_SZ;
    float2 *EX = (float2 *)(Y1 + S::Y1_SZ), *EY = EX + S::KP, *EZ = EY + S::KP;
    const int tid = threadIdx.x;
    const int lane = tid & 63, lr = lane & 15, lq = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    // operator fragments, for the whole kernel: s1 and s3 whole, s2 those
    // of this wave's units (unit u = wave + j NW is (m, cos/sin))
    constexpr int NU2 = 2 * S::NM, UPW = cdiv(NU2, S::NW);
    float f1[S::CT1][S::KS1], f3[S::CT3][S::KS3], f2[UPW][S::RT2][S::KS2];
#pragma unroll
    for (int ct = 0; ct < S::CT1; ++ct)
#pragma unroll
        for (int ks = 0; ks < S::KS1; ++ks) f1[ct][ks] = fr1[(ct * S::KS1 + ks) * 64 + lane];
#pragma unroll
    for (int ct = 0; ct < S::CT3; ++ct)
#pragma unroll
        for (int ks = 0; ks < S::KS3; ++ks) f3[ct][ks] = fr3[(ct * S::KS3 + ks) * 64 + lane];
#pragma unroll
    for (int j = 0; j < UPW; ++j) {
        const int u = wave + j * S::NW;
        const int m = u < NU2 ? u >> 1 : 0;
#pragma unroll
        for (int rt = 0; rt < S::RT2; ++rt)
#pragma unroll
            for (int ks = 0; ks < S::KS2; ++ks)
                f2[j][rt][ks] = fr2[((m * S::RT2 + rt) * S::KS2 + ks) * 64 + lane];
    }
    // Y1's theta padding (read by s2 against zero operator columns) stays 0
    for (int i = tid; i < S::A_SZ + S::Y1_SZ; i += NT) smem[i] = 0.f;
    for (int i = tid; i < 2 * S::KP + S::TP; i += NT) EX[i] = shift_axis[i];

    // descriptors two tiles ahead, input values one tile ahead
    int4 dA = make_int4(0, 0, 0, 0), dB = dA, dC = dA, eA = dA, eB = dA, eC = dA;
    auto load_desc = [&](int64_t t, int4 &d0, int4 &d1) {
        if (t < ntiles) {
            const int64_t g = t / R;
            d0 = desc[2 * g];
            d1 = desc[2 * g + 1];
        }
    };
    float2 xv[S::XR], xs[DOWN ? S::XR : 1];
    auto load_input = [&](int64_t t, const int4 &d0, const int4 &d1) {
        if (t >= ntiles) return;
        const int r = (int)(t % R);
        const int nb = d0.z;
#pragma unroll
        for (int u = 0; u < S::XR; ++u) {
            const int e = tid + u * NT;
            const int sl = e / S::KI, q = e - sl * S::KI;
            if (sl < nb) {
                const int b = DOWN ? d0.x + ((d1.z >> (3 * sl)) & 7) : d0.y + sl;
                xv[u] = In[((int64_t)b * R + r) * S::KI + q];
                // L2L: the octant's shift on the parent grid, with the input
                if constexpr (DOWN) xs[u] = shift[(int64_t)((d1.x >> (3 * sl)) & 7) * S::KI + q];
            }
        }
    };
    const int64_t G = gridDim.x;
    load_desc(blockIdx.x, dA, eA);
    load_desc(blockIdx.x + G, dB, eB);
    load_input(blockIdx.x, dA, eA);

    // lane parts of the LDS addresses
    const int lx1 = (lr >> 1) * S::XS + (lr & 1) + 2 * lq;       // s1 A (X)
    const int ly1 = lr * S::Y1C + 4 * lq;                          // s1 D -> Y1
    const int lb2 = lq * S::Y1T + lr;                              // s2 B (Y1)
    const int ly2 = (lr >> 1) * S::Y2S + (lr & 1) + 8 * lq;       // s2 D -> Y2
    const int la3 = lq * S::Y2T + lr;                              // s3 A (Y2)

    for (int64_t t = blockIdx.x; t < ntiles; t += G) {
        const int r = (int)(t % R);
        const int p0 = dA.x, cb = dA.y, nb = dA.z, np = dA.w;
        const int octs = eA.x, ppf = eA.y;
        load_desc(t + 2 * G, dC, eC);
        __syncthreads();  // the previous tile is done with LDS
        // ---- stage the input of every slot (L2L: the parent's local times
        // the conjugate shift of the slot's child); unused slots 0
#pragma unroll
        for (int u = 0; u < S::XR; ++u) {
            const int e = tid + u * NT;
            const int sl = e / S::KI, q = e - sl * S::KI;
            const int th = q / S::PI, ph = q - th * S::PI;
            if (sl < S::NB) {
                float2 v = make_float2(0.f, 0.f);
                if (sl < nb) {
                    v = xv[u];
                    if constexpr (DOWN) {
                        // conj(shift) * parent local
                        const float2 sv = xs[u];
                        v = make_float2(sv.x * v.x + sv.y * v.y, sv.x * v.y - sv.y * v.x);
                    }
                }
                ((float2 *)RA)[(sl * S::TI + th) * S::XP + ph] = v;
            }
        }
        __syncthreads();
        load_input(t + G, dB, eB);
        // L2L: the child locals this wave adds to in s3 (unit u = wave +
        // j NW is (slot, block of 8 output theta rows)), requested now so
        // that s1 and s2 hide their latency
        constexpr int UPW3 = DOWN ? cdiv(S::NB * S::RT3, S::NW) : 1;
        float2 old[UPW3][S::CT3][2];
        if constexpr (DOWN) {
#pragma unroll
            for (int j = 0; j < UPW3; ++j) {
                const int u = wave + j * S::NW;
                const int i = u / S::RT3, rt = u - i * S::RT3;
                const float2 *o = Out + ((int64_t)(cb + i) * R + r) * S::KO;
#pragma unroll
                for (int ct = 0; ct < S::CT3; ++ct)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int to = rt * 8 + 2 * lq + h, po = ct * 16 + lr;
                        old[j][ct][h] = (i < nb && to < S::TO && po < S::PO)
                                            ? o[to * S::PO + po] : make_float2(0.f, 0.f);
                    }
            }
        }

        // ---- s1: rows (theta_in, slot, part), columns col
        for (int u = wave; u < S::RT1; u += S::NW) {
            const int th = u;
            const float *xa = RA + th * S::XP * 2 + lx1;
            f4 d[S::CT1];
#pragma unroll
            for (int ct = 0; ct < S::CT1; ++ct) d[ct] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < S::KS1; ++ks) {
                const float a = (4 * ks + 3 < S::PI || 4 * ks + lq < S::PI) ? xa[8 * ks] : 0.f;
#pragma unroll
                for (int ct = 0; ct < S::CT1; ++ct) d[ct] = mma(a, f1[ct][ks], d[ct]);
            }
            float *y = Y1 + th * S::Y1T + ly1;
#pragma unroll
            for (int ct = 0; ct < S::CT1; ++ct)
                if (ct * 16 + lr < S::M)
                    *(f4 *)(y + ct * 16 * S::Y1C) = d[ct];
        }
        __syncthreads();

        // ---- s2: per (|m|, cos/sin column), rows theta_out, columns (slot, part)
#pragma unroll
        for (int j = 0; j < UPW; ++j) {
            const int u = wave + j * S::NW;
            const int m = u >> 1, cs = u & 1;
            if (u >= NU2 || (m == 0 && cs == 1)) continue;
            const int col = m ? 2 * m - 1 + cs : 0;
            const float *yb = Y1 + col * S::Y1C + lb2;
            f4 d[S::RT2];
#pragma unroll
            for (int rt = 0; rt < S::RT2; ++rt) d[rt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < S::KS2; ++ks) {
                const float b = yb[4 * ks * S::Y1T];
#pragma unroll
                for (int rt = 0; rt < S::RT2; ++rt) d[rt] = mma(f2[j][rt][ks], b, d[rt]);
            }
            float *yo = RA + col * S::Y2T + ly2;
#pragma unroll
            for (int rt = 0; rt < S::RT2; ++rt)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (rt * 16 + 4 * lq + v < S::TO) yo[(rt * 16 + v) * 2] = d[rt][v];
        }
        __syncthreads();

        // ---- s3: rows (theta_out, part), K = col, columns phi_out
        auto synth = [&](int i, int rt, bool ra, f4 (&d)[S::CT3]) {
            const float *ya = RA + i * S::Y2S + rt * 16 + la3;
#pragma unroll
            for (int ct = 0; ct < S::CT3; ++ct) d[ct] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < S::KS3; ++ks) {
                const float a = ra ? ya[4 * ks * S::Y2T] : 0.f;
#pragma unroll
                for (int ct = 0; ct < S::CT3; ++ct) d[ct] = mma(a, f3[ct][ks], d[ct]);
            }
        };
        if (!DOWN) {
            // unit = (parent, 8 output theta rows): the shifted children
            // summed in registers; the axis factors of the lane's outputs
            // are read once per unit
            for (int u = wave; u < np * S::RT3; u += S::NW) {
                const int pp = u / S::RT3, rt = u - pp * S::RT3;
                const bool ra = rt * 8 + (lr >> 1) < S::TO;
                const int i0 = pp == 0 ? 0 : (ppf >> (4 * (pp - 1))) & 15;
                const int i1 = pp + 1 == np ? nb : (ppf >> (4 * pp)) & 15;
                float2 fx[S::CT3][2], fy[S::CT3][2], fz[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int to = min(rt * 8 + 2 * lq + h, S::TO - 1);
                    fz[h] = EZ[to];
#pragma unroll
                    for (int ct = 0; ct < S::CT3; ++ct) {
                        const int po = min(ct * 16 + lr, S::PO - 1);
                        fx[ct][h] = EX[to * S::PO + po];
                        fy[ct][h] = EY[to * S::PO + po];
                    }
                }
                f4 acc[S::CT3];
#pragma unroll
                for (int ct = 0; ct < S::CT3; ++ct) acc[ct] = f4{0.f, 0.f, 0.f, 0.f};
                for (int i = i0; i < i1; ++i) {
                    f4 d[S::CT3];
                    synth(i, rt, ra, d);
                    const int oc = (octs >> (3 * i)) & 7;
                    // the octant's shift: each axis factor conjugated where the bit is 0
                    const float sx = (oc & 4) ? 1.f : -1.f, sy = (oc & 2) ? 1.f : -1.f,
                                sz = (oc & 1) ? 1.f : -1.f;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const float2 c = make_float2(fz[h].x, sz * fz[h].y);
#pragma unroll
                        for (int ct = 0; ct < S::CT3; ++ct) {
                            const float2 a = make_float2(fx[ct][h].x, sx * fx[ct][h].y);
                            const float2 b = make_float2(fy[ct][h].x, sy * fy[ct][h].y);
                            const float2 ab = make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
                            const float2 sv = make_float2(ab.x * c.x - ab.y * c.y, ab.x * c.y + ab.y * c.x);
                            const float yr = d[ct][2 * h], yi = d[ct][2 * h + 1];
                            acc[ct][2 * h] += sv.x * yr - sv.y * yi;
                            acc[ct][2 * h + 1] += sv.x * yi + sv.y * yr;
                        }
                    }
                }
                float2 *o = Out + ((int64_t)(p0 + pp) * R + r) * S::KO;
#pragma unroll
                for (int ct = 0; ct < S::CT3; ++ct) {
                    const int po = ct * 16 + lr;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int to = rt * 8 + 2 * lq + h;
                        if (to < S::TO && po < S::PO)
                            o[to * S::PO + po] = make_float2(acc[ct][2 * h], acc[ct][2 * h + 1]);
                    }
                }
            }
        } else {
            // unit = (slot, 8 output theta rows): add into the slot's child
#pragma unroll
            for (int j = 0; j < UPW3; ++j) {
                const int u = wave + j * S::NW;
                const int i = u / S::RT3, rt = u - i * S::RT3;
                if (i >= nb) continue;
                const bool ra = rt * 8 + (lr >> 1) < S::TO;
                f4 d[S::CT3];
                synth(i, rt, ra, d);
                float2 *o = Out + ((int64_t)(cb + i) * R + r) * S::KO;
#pragma unroll
                for (int ct = 0; ct < S::CT3; ++ct) {
                    const int po = ct * 16 + lr;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int to = rt * 8 + 2 * lq + h;
                        if (to < S::TO && po < S::PO)
                            o[to * S::PO + po] = make_float2(old[j][ct][h].x + d[ct][2 * h],
                                                             old[j][ct][h].y + d[ct][2 * h + 1]);
                    }
                }
            }
        }
        dA = dB;
        eA = eB;
        dB = dC;
        eB = eC;
    }
}

// ---------------------------------------------------------------- BF16x3 --
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

// x = hi + lo per element (round to nearest even; gfx950 converts pairs)
__device__ __forceinline__ void split8(const float (&x)[8], bf16x8 &h, bf16x8 &l)
{
    bf16x8 hb;
#pragma unroll
    for (int e = 0; e < 8; ++e) hb[e] = (__bf16)x[e];
    const u4v hu = __builtin_bit_cast(u4v, hb);
    bf16x8 lb;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        lb[2 * i] = (__bf16)(x[2 * i] - __uint_as_float(hu[i] << 16));
        lb[2 * i + 1] = (__bf16)(x[2 * i + 1] - __uint_as_float(hu[i] & 0xffff0000u));
    }
    h = hb;
    l = lb;
}

__device__ __forceinline__ f4 mma3(bf16x8 ah, bf16x8 al, bf16x8 bh, bf16x8 bl, f4 c)
{
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
}

constexpr int rup8(int a) { return (a + 7) / 8 * 8; }

// LDS layout and fragment counts of the BF16x3 form (floats)
template <class S>
struct BfShape {
    static constexpr int KB1 = cdiv(S::PI, 32), KB2 = cdiv(S::TI, 32), KB3 = cdiv(S::M, 32);
    static constexpr int X1P = rup8(S::PI) + 4, XPS = S::TI * X1P, X_SZ = S::NB * 2 * XPS;
    static constexpr int Y1P = rup8(S::TI) + 4, Y1_SZ = S::M * 2 * S::NB * Y1P;
    static constexpr int Y2P = rup8(S::M) + 4, Y2S = S::RT3 * 16 * Y2P, Y2_SZ = S::NB * Y2S;
    static constexpr int A_SZ = cmax(X_SZ, Y2_SZ);
    static constexpr int LDS_FLOATS = A_SZ + Y1_SZ + S::E_SZ;
    // 8 floats (hi, lo: 8 bf16 each) per lane and fragment
    static constexpr int NF1 = S::CT1 * KB1 * 512, NF2 = S::NM * S::RT2 * KB2 * 512,
                         NF3 = S::CT3 * KB3 * 512;
};

// The same pair kernel with every map in BF16 split precision (BF16x3):
// each FP32 operand x = hi + lo, hi = bf16(x), lo = bf16(x - hi), and each
// product taken as lo*hi + hi*lo + hi*hi on v_mfma_f32_16x16x32_bf16 with
// FP32 accumulation (the dropped lo*lo term is 2^-16 of the product).  Lane
// l feeds A[l%16][32 kb + 8(l/16) .. +7] and B[32 kb + 8(l/16) .. +7][l%16]
// and receives D as in the FP32 kernel, so the epilogues are unchanged.
// The operator fragments are host-split (hi then lo, 8 bf16 each per lane);
// the data are split when a lane reads its 8 consecutive K values, so LDS
// keeps them in FP32 with the contraction index contiguous:
//   X   [slot][part][theta_in][phi_in]       (s1 A, K = phi_in)
//   Y1  [col][slot, part][theta_in]          (s2 B, K = theta_in)
//   Y2  [slot][theta_out, part][col]         (s3 A, K = col)
// Rows are padded to a multiple of 8 (+ 4 against bank conflicts); padding
// meets zero operator rows or columns.
template <class S>
__global__ void __launch_bounds__(64 * S::NW)
k_pair_bf(const float2 *__restrict__ In, float2 *__restrict__ Out, const int4 *__restrict__ desc,
       int64_t ntiles, int R, const float *__restrict__ fr1, const float *__restrict__ fr2,
       const float *__restrict__ fr3, const float2 *__restrict__ shift_axis,
       const float2 *__restrict__ shift)
{
    static_assert(S::NB == 8, "tile descriptors pack 8 slots");
    constexpr bool DOWN = S::DOWN;
    constexpr int NT = S::NT;
    extern __shared__ float smem[];
    using B = BfShape<S>;
    float *RA = smem;               // X, then Y2
    float *Y1 = smem + B::A_SZ;
    float2 *EX = (float2 *)(Y1 + B::Y1_SZ), *EY = EX + S::KP, *EZ = EY + S::KP;
    const int tid = threadIdx.x;
    const int lane = tid & 63, lr = lane & 15, lq = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    // operator fragments (hi, lo), for the whole kernel: s1 and s3 whole,
    // s2 those of this wave's units (unit u = wave + j NW is (m, cos/sin))
    constexpr int NU2 = 2 * S::NM, UPW = cdiv(NU2, S::NW);
    bf16x8 f1h[S::CT1][B::KB1], f1l[S::CT1][B::KB1], f3h[S::CT3][B::KB3], f3l[S::CT3][B::KB3];
    bf16x8 f2h[UPW][S::RT2][B::KB2], f2l[UPW][S::RT2][B::KB2];
    {
        const bf16x8 *g1 = (const bf16x8 *)fr1, *g2 = (const bf16x8 *)fr2,
                     *g3 = (const bf16x8 *)fr3;
#pragma unroll
        for (int ct = 0; ct < S::CT1; ++ct)
#pragma unroll
            for (int kb = 0; kb < B::KB1; ++kb) {
                f1h[ct][kb] = g1[2 * ((ct * B::KB1 + kb) * 64 + lane)];
                f1l[ct][kb] = g1[2 * ((ct * B::KB1 + kb) * 64 + lane) + 1];
            }
#pragma unroll
        for (int ct = 0; ct < S::CT3; ++ct)
#pragma unroll
            for (int kb = 0; kb < B::KB3; ++kb) {
                f3h[ct][kb] = g3[2 * ((ct * B::KB3 + kb) * 64 + lane)];
                f3l[ct][kb] = g3[2 * ((ct * B::KB3 + kb) * 64 + lane) + 1];
            }
#pragma unroll
        for (int j = 0; j < UPW; ++j) {
            const int u = wave + j * S::NW;
            const int m = u < NU2 ? u >> 1 : 0;
#pragma unroll
            for (int rt = 0; rt < S::RT2; ++rt)
#pragma unroll
                for (int kb = 0; kb < B::KB2; ++kb) {
                    const int f = ((m * S::RT2 + rt) * B::KB2 + kb) * 64 + lane;
                    f2h[j][rt][kb] = g2[2 * f];
                    f2l[j][rt][kb] = g2[2 * f + 1];
                }
        }
    }
    // Y1's theta padding (read by s2 against zero operator columns) stays 0
    for (int i = tid; i < B::A_SZ + B::Y1_SZ; i += NT) smem[i] = 0.f;
    for (int i = tid; i < 2 * S::KP + S::TP; i += NT) EX[i] = shift_axis[i];

    // descriptors two tiles ahead, input values one tile ahead
    int4 dA = make_int4(0, 0, 0, 0), dB = dA, dC = dA, eA = dA, eB = dA, eC = dA;
    auto load_desc = [&](int64_t t, int4 &d0, int4 &d1) {
        if (t < ntiles) {
            const int64_t g = t / R;
            d0 = desc[2 * g];
            d1 = desc[2 * g + 1];
        }
    };
    // LEAN (L2L with two K blocks in s1, the pair 13 -> 20): the octant's
    // shift is formed from the axis factors in LDS at staging rather than
    // prefetched, and the child locals are read in s3 next to their use, to
    // stay within 256 registers; the other shapes prefetch both
    constexpr bool LEAN = DOWN && B::KB1 > 1;
    float2 xv[LEAN ? 1 : S::XR], xs[(DOWN && !LEAN) ? S::XR : 1];
    auto load_input = [&](int64_t t, const int4 &d0, const int4 &d1) {
        if constexpr (LEAN) return;  // (LEAN: read at staging)
        if (t >= ntiles) return;
        const int r = (int)(t % R);
        const int nb = d0.z;
#pragma unroll
        for (int u = 0; u < S::XR; ++u) {
            const int e = tid + u * NT;
            const int sl = e / S::KI, q = e - sl * S::KI;
            if (sl < nb) {
                const int b = DOWN ? d0.x + ((d1.z >> (3 * sl)) & 7) : d0.y + sl;
                xv[u] = In[((int64_t)b * R + r) * S::KI + q];
                // L2L: the octant's shift on the parent grid, with the input
                if constexpr (DOWN && !LEAN)
                    xs[u] = shift[(int64_t)((d1.x >> (3 * sl)) & 7) * S::KI + q];
            }
        }
    };
    const int64_t G = gridDim.x;
    load_desc(blockIdx.x, dA, eA);
    load_desc(blockIdx.x + G, dB, eB);
    load_input(blockIdx.x, dA, eA);

    // lane parts of the LDS addresses
    const int lx1 = lr * B::XPS + 8 * lq;                          // s1 A (X plane lr)
    const int lb2 = lr * B::Y1P + 8 * lq;                          // s2 B (Y1 row lr)
    const int ly2 = (lr >> 1) * B::Y2S + (lr & 1) * B::Y2P;       // s2 D -> Y2
    const int la3 = lr * B::Y2P + 8 * lq;                          // s3 A (Y2 row)
    // 8 consecutive FP32 values from LDS (16-byte aligned), split
    auto frag = [&](const float *p, bool live, bf16x8 &h, bf16x8 &l) {
        float x[8];
        if (live) {
            const float4 a = *(const float4 *)p, b = *(const float4 *)(p + 4);
            x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
            x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) x[e] = 0.f;
        }
        split8(x, h, l);
    };

    for (int64_t t = blockIdx.x; t < ntiles; t += G) {
        const int r = (int)(t % R);
        const int p0 = dA.x, cb = dA.y, nb = dA.z, np = dA.w;
        const int octs = eA.x, ppf = eA.y;
        load_desc(t + 2 * G, dC, eC);
        __syncthreads();  // the previous tile is done with LDS
        // ---- stage the input of every slot (L2L: the parent's local times
        // the conjugate shift of the slot's child); unused slots 0
#pragma unroll
        for (int u = 0; u < S::XR; ++u) {
            const int e = tid + u * NT;
            const int sl = e / S::KI, q = e - sl * S::KI;
            const int th = q / S::PI, ph = q - th * S::PI;
            if (sl < S::NB) {
                float2 v = make_float2(0.f, 0.f);
                if (sl < nb) {
                    if constexpr (LEAN) {
                        const int b = dA.x + ((eA.z >> (3 * sl)) & 7);
                        v = In[((int64_t)b * R + r) * S::KI + q];
                    } else {
                        v = xv[u];
                    }
                    if constexpr (LEAN) {
                        // conj(shift) * parent local
                        const float2 sc = octant_shift(EX, EY, EZ, (octs >> (3 * sl)) & 7, th, q,
                                                       true);
                        v = make_float2(sc.x * v.x - sc.y * v.y, sc.x * v.y + sc.y * v.x);
                    } else if constexpr (DOWN) {
                        const float2 sv = xs[u];
                        v = make_float2(sv.x * v.x + sv.y * v.y, sv.x * v.y - sv.y * v.x);
                    }
                }
                RA[(2 * sl) * B::XPS + th * B::X1P + ph] = v.x;
                RA[(2 * sl + 1) * B::XPS + th * B::X1P + ph] = v.y;
            }
        }
        __syncthreads();
        load_input(t + G, dB, eB);
        // L2L: the child locals this wave adds to in s3 (unit u = wave +
        // j NW is (slot, block of 8 output theta rows)), requested now so
        // that s1 and s2 hide their latency (LEAN: read in s3)
        constexpr int UPW3 = DOWN ? cdiv(S::NB * S::RT3, S::NW) : 1;
        constexpr int UPW3E = (DOWN && !LEAN) ? UPW3 : 1;
        float2 old[UPW3E][S::CT3][2];
        if constexpr (DOWN && !LEAN) {
#pragma unroll
            for (int j = 0; j < UPW3; ++j) {
                const int u = wave + j * S::NW;
                const int i = u / S::RT3, rt = u - i * S::RT3;
                const float2 *o = Out + ((int64_t)(cb + i) * R + r) * S::KO;
#pragma unroll
                for (int ct = 0; ct < S::CT3; ++ct)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int to = rt * 8 + 2 * lq + h, po = ct * 16 + lr;
                        old[j][ct][h] = (i < nb && to < S::TO && po < S::PO)
                                            ? o[to * S::PO + po] : make_float2(0.f, 0.f);
                    }
            }
        }

        // ---- s1: rows (slot, part) of one theta_in, columns col
        for (int u = wave; u < S::RT1; u += S::NW) {
            const int th = u;
            f4 d[S::CT1];
#pragma unroll
            for (int ct = 0; ct < S::CT1; ++ct) d[ct] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < B::KB1; ++kb) {
                bf16x8 ah, al;
                frag(RA + th * B::X1P + lx1 + 32 * kb, 32 * kb + 8 * lq < S::PI, ah, al);
#pragma unroll
                for (int ct = 0; ct < S::CT1; ++ct)
                    d[ct] = mma3(ah, al, f1h[ct][kb], f1l[ct][kb], d[ct]);
            }
            // D row 4 lq + v is plane (slot, part), column ct 16 + lr is col
#pragma unroll
            for (int ct = 0; ct < S::CT1; ++ct) {
                const int col = ct * 16 + lr;
                if (col < S::M) {
                    float *y = Y1 + (col * 16 + 4 * lq) * B::Y1P + th;
#pragma unroll
                    for (int v = 0; v < 4; ++v) y[v * B::Y1P] = d[ct][v];
                }
            }
        }
        __syncthreads();

        // ---- s2: per (|m|, cos/sin column), rows theta_out, columns (slot, part)
#pragma unroll
        for (int j = 0; j < UPW; ++j) {
            const int u = wave + j * S::NW;
            const int m = u >> 1, cs = u & 1;
            if (u >= NU2 || (m == 0 && cs == 1)) continue;
            const int col = m ? 2 * m - 1 + cs : 0;
            f4 d[S::RT2];
#pragma unroll
            for (int rt = 0; rt < S::RT2; ++rt) d[rt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < B::KB2; ++kb) {
                bf16x8 bh, bl;
                frag(Y1 + col * 16 * B::Y1P + lb2 + 32 * kb, 32 * kb + 8 * lq < S::TI, bh, bl);
#pragma unroll
                for (int rt = 0; rt < S::RT2; ++rt)
                    d[rt] = mma3(f2h[j][rt][kb], f2l[j][rt][kb], bh, bl, d[rt]);
            }
            // D row 16 rt + 4 lq + v is theta_out, column lr is (slot, part)
            float *yo = RA + ly2 + col;
#pragma unroll
            for (int rt = 0; rt < S::RT2; ++rt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int to = rt * 16 + 4 * lq + v;
                    if (to < S::TO) yo[2 * to * B::Y2P] = d[rt][v];
                }
        }
        __syncthreads();

        // ---- s3: rows (theta_out, part), K = col, columns phi_out
        auto synth = [&](int i, int rt, bool ra, f4 (&d)[S::CT3]) {
            const float *ya = RA + i * B::Y2S + rt * 16 * B::Y2P + la3;
#pragma unroll
            for (int ct = 0; ct < S::CT3; ++ct) d[ct] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < B::KB3; ++kb) {
                bf16x8 ah, al;
                frag(ya + 32 * kb, ra && 32 * kb + 8 * lq < S::M, ah, al);
#pragma unroll
                for (int ct = 0; ct < S::CT3; ++ct)
                    d[ct] = mma3(ah, al, f3h[ct][kb], f3l[ct][kb], d[ct]);
            }
        };
        if (!DOWN) {
            // unit = (parent, 8 output theta rows): the shifted children
            // summed in registers; the axis factors of the lane's outputs
            // are read once per unit
            for (int u = wave; u < np * S::RT3; u += S::NW) {
                const int pp = u / S::RT3, rt = u - pp * S::RT3;
                const bool ra = rt * 8 + (lr >> 1) < S::TO;
                const int i0 = pp == 0 ? 0 : (ppf >> (4 * (pp - 1))) & 15;
                const int i1 = pp + 1 == np ? nb : (ppf >> (4 * pp)) & 15;
                float2 fx[S::CT3][2], fy[S::CT3][2], fz[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int to = min(rt * 8 + 2 * lq + h, S::TO - 1);
                    fz[h] = EZ[to];
#pragma unroll
                    for (int ct = 0; ct < S::CT3; ++ct) {
                        const int po = min(ct * 16 + lr, S::PO - 1);
                        fx[ct][h] = EX[to * S::PO + po];
                        fy[ct][h] = EY[to * S::PO + po];
                    }
                }
                f4 acc[S::CT3];
#pragma unroll
                for (int ct = 0; ct < S::CT3; ++ct) acc[ct] = f4{0.f, 0.f, 0.f, 0.f};
                for (int i = i0; i < i1; ++i) {
                    f4 d[S::CT3];
                    synth(i, rt, ra, d);
                    const int oc = (octs >> (3 * i)) & 7;
                    // the octant's shift: each axis factor conjugated where the bit is 0
                    const float sx = (oc & 4) ? 1.f : -1.f, sy = (oc & 2) ? 1.f : -1.f,
                                sz = (oc & 1) ? 1.f : -1.f;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const float2 c = make_float2(fz[h].x, sz * fz[h].y);
#pragma unroll
                        for (int ct = 0; ct < S::CT3; ++ct) {
                            const float2 a = make_float2(fx[ct][h].x, sx * fx[ct][h].y);
                            const float2 b = make_float2(fy[ct][h].x, sy * fy[ct][h].y);
                            const float2 ab = make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
                            const float2 sv = make_float2(ab.x * c.x - ab.y * c.y, ab.x * c.y + ab.y * c.x);
                            const float yr = d[ct][2 * h], yi = d[ct][2 * h + 1];
                            acc[ct][2 * h] += sv.x * yr - sv.y * yi;
                            acc[ct][2 * h + 1] += sv.x * yi + sv.y * yr;
                        }
                    }
                }
                float2 *o = Out + ((int64_t)(p0 + pp) * R + r) * S::KO;
#pragma unroll
                for (int ct = 0; ct < S::CT3; ++ct) {
                    const int po = ct * 16 + lr;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int to = rt * 8 + 2 * lq + h;
                        if (to < S::TO && po < S::PO)
                            o[to * S::PO + po] = make_float2(acc[ct][2 * h], acc[ct][2 * h + 1]);
                    }
                }
            }
        } else {
            // unit = (slot, 8 output theta rows): add into the slot's child
#pragma unroll
            for (int j = 0; j < UPW3; ++j) {
                const int u = wave + j * S::NW;
                const int i = u / S::RT3, rt = u - i * S::RT3;
                if (i >= nb) continue;
                const bool ra = rt * 8 + (lr >> 1) < S::TO;
                float2 *o = Out + ((int64_t)(cb + i) * R + r) * S::KO;
                float2 late[S::CT3][2];
                if constexpr (LEAN) {
#pragma unroll
                    for (int ct = 0; ct < S::CT3; ++ct)
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const int to = rt * 8 + 2 * lq + h, po = ct * 16 + lr;
                            late[ct][h] = (to < S::TO && po < S::PO) ? o[to * S::PO + po]
                                                                    : make_float2(0.f, 0.f);
                        }
                }
                f4 d[S::CT3];
                synth(i, rt, ra, d);
#pragma unroll
                for (int ct = 0; ct < S::CT3; ++ct) {
                    const int po = ct * 16 + lr;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int to = rt * 8 + 2 * lq + h;
                        if (to < S::TO && po < S::PO) {
                            const float2 ov = LEAN ? late[ct][h] : old[LEAN ? 0 : j][ct][h];
                            o[to * S::PO + po] = make_float2(ov.x + d[ct][2 * h],
                                                             ov.y + d[ct][2 * h + 1]);
                        }
                    }
                }
            }
        }
        dA = dB;
        eA = eB;
        dB = dC;
        eB = eC;
    }
}

template <class S, bool BF>
hipError_t launch_pair(const float2 *In, float2 *Out, const int4 *desc, int64_t ngroups, int R,
                       const float *fr1, const float *fr2, const float *fr3,
                       const float2 *shift_axis, const float2 *shift, hipStream_t st)
{
    const size_t lds =
        (size_t)(BF ? (int)BfShape<S>::LDS_FLOATS : (int)S::LDS_FLOATS) * sizeof(float);
    auto kern = BF ? k_pair_bf<S> : k_pair<S>;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * S::NW, lds) !=
            hipSuccess || per_cu < 1) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        ncu = 256;
    const int64_t ntiles = ngroups * R;
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(ntiles, (int64_t)per_cu * ncu));
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64 * S::NW), lds, st, In, Out, desc,
                       ntiles, R, fr1, fr2, fr3, shift_axis, shift);
    return hipGetLastError();
}

// shapes of the level pairs of a 0.25-wavelength leaf at 3 digits
typedef PairShape<8, 13, false, 8, 4> M2M_8_13;
typedef PairShape<8, 13, true, 8, 8> L2L_8_13;
typedef PairShape<13, 20, false, 8, 8> M2M_13_20;
typedef PairShape<13, 20, true, 8, 8> L2L_13_20;

template <class S>
void fill_fragments(const float *F, const float *A, const float *G, PairTables *t)
{
    // s1: B = F [PI][M]
    t->fr1.assign(S::NF1, 0.f);
    for (int ct = 0; ct < S::CT1; ++ct)
        for (int ks = 0; ks < S::KS1; ++ks)
            for (int l = 0; l < 64; ++l) {
                const int k = 4 * ks + (l >> 4), n = 16 * ct + (l & 15);
                if (k < S::PI && n < S::M) t->fr1[(ct * S::KS1 + ks) * 64 + l] = F[k * S::M + n];
            }
    // s2: A[row = theta_out][k = theta_in] = maps[m][theta_in][theta_out]
    t->fr2.assign(S::NF2, 0.f);
    for (int m = 0; m < S::NM; ++m)
        for (int rt = 0; rt < S::RT2; ++rt)
            for (int ks = 0; ks < S::KS2; ++ks)
                for (int l = 0; l < 64; ++l) {
                    const int row = 16 * rt + (l & 15), k = 4 * ks + (l >> 4);
                    if (row < S::TO && k < S::TI)
                        t->fr2[((m * S::RT2 + rt) * S::KS2 + ks) * 64 + l] =
                            A[((size_t)m * S::TI + k) * S::TO + row];
                }
    // s3: B = G [M][PO]
    t->fr3.assign(S::NF3, 0.f);
    for (int ct = 0; ct < S::CT3; ++ct)
        for (int ks = 0; ks < S::KS3; ++ks)
            for (int l = 0; l < 64; ++l) {
                const int k = 4 * ks + (l >> 4), n = 16 * ct + (l & 15);
                if (k < S::M && n < S::PO) t->fr3[(ct * S::KS3 + ks) * 64 + l] = G[k * S::PO + n];
            }
    t->max_children = S::NB;
    t->max_parents = S::NB;
}

// BF16x3 fragments: per lane 8 consecutive K values of its row (A) or
// column (B), split hi = bf16(x), lo = bf16(x - hi), stored as 8 bf16 hi
// then 8 bf16 lo (8 floats' worth)
static uint16_t bf16_rn_host(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

static void put_frag(std::vector<float> &fr, int64_t f, const float (&v)[8])
{
    uint16_t h[8], l[8];
    for (int e = 0; e < 8; ++e) {
        h[e] = bf16_rn_host(v[e]);
        uint32_t u = (uint32_t)h[e] << 16;
        float hf;
        std::memcpy(&hf, &u, 4);
        l[e] = bf16_rn_host(v[e] - hf);
    }
    std::memcpy(&fr[(size_t)f * 8], h, 16);
    std::memcpy(&fr[(size_t)f * 8 + 4], l, 16);
}

template <class S>
void fill_fragments_bf(const float *F, const float *A, const float *G, PairTables *t)
{
    using B = BfShape<S>;
    float v[8];
    // s1: B = F [PI][M]
    t->fr1.assign(B::NF1, 0.f);
    for (int ct = 0; ct < S::CT1; ++ct)
        for (int kb = 0; kb < B::KB1; ++kb)
            for (int l = 0; l < 64; ++l) {
                const int n = 16 * ct + (l & 15);
                for (int e = 0; e < 8; ++e) {
                    const int k = 32 * kb + 8 * (l >> 4) + e;
                    v[e] = (k < S::PI && n < S::M) ? F[k * S::M + n] : 0.f;
                }
                put_frag(t->fr1, (ct * B::KB1 + kb) * 64 + l, v);
            }
    // s2: A[row = theta_out][k = theta_in] = maps[m][theta_in][theta_out]
    t->fr2.assign(B::NF2, 0.f);
    for (int m = 0; m < S::NM; ++m)
        for (int rt = 0; rt < S::RT2; ++rt)
            for (int kb = 0; kb < B::KB2; ++kb)
                for (int l = 0; l < 64; ++l) {
                    const int row = 16 * rt + (l & 15);
                    for (int e = 0; e < 8; ++e) {
                        const int k = 32 * kb + 8 * (l >> 4) + e;
                        v[e] = (row < S::TO && k < S::TI)
                                   ? A[((size_t)m * S::TI + k) * S::TO + row] : 0.f;
                    }
                    put_frag(t->fr2, ((m * S::RT2 + rt) * B::KB2 + kb) * 64 + l, v);
                }
    // s3: B = G [M][PO]
    t->fr3.assign(B::NF3, 0.f);
    for (int ct = 0; ct < S::CT3; ++ct)
        for (int kb = 0; kb < B::KB3; ++kb)
            for (int l = 0; l < 64; ++l) {
                const int n = 16 * ct + (l & 15);
                for (int e = 0; e < 8; ++e) {
                    const int k = 32 * kb + 8 * (l >> 4) + e;
                    v[e] = (k < S::M && n < S::PO) ? G[k * S::PO + n] : 0.f;
                }
                put_frag(t->fr3, (ct * B::KB3 + kb) * 64 + l, v);
            }
    t->max_children = S::NB;
    t->max_parents = S::NB;
}

}  // namespace

bool pair_kernel_fits(int Lc, int Lp, bool down)
{
    (void)down;  // both directions of the instantiated pairs
    return (Lc == 8 && Lp == 13) || (Lc == 13 && Lp == 20);
}

int pair_tables(int Lc, int Lp, bool down, const float *F, const float *A, const float *G,
                PairTables *t, bool bf16x3)
{
#define FILL(S)                                                  \
    do {                                                         \
        if (bf16x3) fill_fragments_bf<S>(F, A, G, t);            \
        else fill_fragments<S>(F, A, G, t);                      \
        return 0;                                                \
    } while (0)
    if (Lc == 8 && Lp == 13) {
        if (down) FILL(L2L_8_13);
        FILL(M2M_8_13);
    }
    if (Lc == 13 && Lp == 20) {
        if (down) FILL(L2L_13_20);
        FILL(M2M_13_20);
    }
#undef FILL
    return -1;
}

hipError_t pair_map(int Lc, int Lp, bool down, const float2 *In, float2 *Out, const int4 *desc,
                    int64_t ngroups, int R, const float *fr1, const float *fr2, const float *fr3,
                    const float2 *shift_axis, const float2 *shift, hipStream_t st, bool bf16x3)
{
    if (ngroups == 0) return hipSuccess;
#define PAIR(S)                                                                              \
    return bf16x3 ? launch_pair<S, true>(In, Out, desc, ngroups, R, fr1, fr2, fr3, shift_axis, \
                                         shift, st)                                           \
                  : launch_pair<S, false>(In, Out, desc, ngroups, R, fr1, fr2, fr3,           \
                                          shift_axis, shift, st)
    if (Lc == 8 && Lp == 13) {
        if (down) PAIR(L2L_8_13);
        PAIR(M2M_8_13);
    }
    if (Lc == 13 && Lp == 20) {
        if (down) PAIR(L2L_13_20);
        PAIR(M2M_13_20);
    }
#undef PAIR
    return hipErrorInvalidValue;
}

}  // namespace dev
}  // namespace mlfma
