// FFT interpolation and anterpolation between uniform sphere grids: the
// paper's M2M interpolation (Sec. 3.2.2, paragraph "Fine-grained Parallel
// Interpolation", Fig. 3: FFT interpolation along phi, transposition and
// folding of theta into whole circles, FFT interpolation along them,
// unfolding) and its reverse for L2L (Sec. 3.2.4), as a batched operator on
// many boxes (and right-hand sides) at once.
//
// Grid with P phi samples (P even): phi_j = 2 pi j / P, theta_i =
// (i + 1/2) 2 pi / P, i < P / 2, stored [theta][phi].  The circle through
// phi_j and phi_j + pi holds P samples at (s + 1/2) 2 pi / P: s < P/2 is
// theta_s of column j, s >= P/2 theta_{P-1-s} of column j + P/2.  A
// function of degree <= Lband is a trigonometric polynomial of degree <=
// Lband along phi and along every such circle, so resampling each of them
// through its Fourier coefficients |f| <= Lband is exact.
//
// Interpolation (down = 0):  phi-resample the rows P_in -> P_out, fold
// into P_out/2 circles of P_in samples, resample the circles to P_out
// samples (half-sample offsets on both sides: a phase per frequency),
// unfold.  Anterpolation (down = 1) is the weighted adjoint
// W_out^-1 I^T W_in of the interpolation from the output grid to the input
// grid: the transposed stages in reverse order (fold, circle resample,
// unfold, phi resample), with the input rows scaled by the theta weights of
// the input grid and the output rows by (P_in / P_out) / (theta weight of
// the output grid) (Fejer's first rule; the host computes both in FP64).
//
// One workgroup of 256 threads takes `ipw` items (boxes x right-hand sides)
// of the batch; every transform runs over all rows of all its items at
// once.  LDS holds two regions of `S` complex values per item; the FFTs are
// mixed-radix Stockham (radices 4, 2, 3, 5, 7; out of place, so each stage
// goes from one region to the other), the padding, folding and unfolding
// move data between the regions.  FP32 throughout.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <new>
#include <vector>

#include "internal.h"
#include "mlfma.h"

namespace mlfma {
namespace dev {

namespace {

constexpr int kMaxThreads = 1024;
constexpr int kMaxRadices = 12;

struct FftDesc {
    int pi, po, ti, to, lb, down, ipw, S;
    int nri, nro;
    int ri[kMaxRadices], ro[kMaxRadices];
    // offsets into the table of the forward twiddles of each stage (P_in
    // and P_out transforms), then the theta phases of the circle padding
    int twi[kMaxRadices], two[kMaxRadices];
    int ntab, tab_phase;
    const float2 *tab;        // [ntab] (copied to LDS by every workgroup)
    const float *pre, *post;  // per-row scales of the input / output (or null)
};

// floor(a / d) for 0 <= a < 2^24 and small d, with inv = 1 / d in FP32:
// the product is off by at most one, which the remainder corrects
__device__ __forceinline__ int fdiv(int a, int d, float inv)
{
    int q = (int)((float)a * inv);
    const int r = a - q * d;
    q += (r >= d) - (r < 0);
    return q;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// One Stockham stage of radix R over `rows` rows of length n per item
// (item t's row r starts at t * S + r * n); Ns = product of the radices of
// the earlier stages; sign -1 forward, +1 inverse.  tw: the stage's forward
// twiddles exp(-2 pi i q k / (Ns R)) at [k (R - 1) + q - 1] (conjugated for
// the inverse).
template <int R>
__device__ void stage(const float2 *__restrict__ src, float2 *__restrict__ dst, int nitem,
                      int rows, int n, int S, int Ns, float sign, const float2 *tw)
{
    const int nb = n / R;
    const int per_item = rows * nb;
    const int total = nitem * per_item;
    const float inv_item = 1.0f / (float)per_item, inv_nb = 1.0f / (float)nb,
                inv_ns = 1.0f / (float)Ns;
    float2 root[R];
#pragma unroll
    for (int p = 0; p < R; ++p) {
        float s, c;
        sincospif(sign * 2.0f * (float)p / (float)R, &s, &c);
        root[p] = make_float2(c, s);
    }
    for (int b = threadIdx.x; b < total; b += blockDim.x) {
        const int t = fdiv(b, per_item, inv_item);
        const int rb = b - t * per_item;
        const int r = fdiv(rb, nb, inv_nb);
        const int j = rb - r * nb;
        const int jq = fdiv(j, Ns, inv_ns);
        const int k = j - jq * Ns;
        const int off = t * S + r * n;
        float2 v[R];
#pragma unroll
        for (int q = 0; q < R; ++q) v[q] = src[off + j + q * nb];
        if (Ns > 1) {
#pragma unroll
            for (int q = 1; q < R; ++q) {
                const float2 w = tw[k * (R - 1) + q - 1];
                v[q] = cmul(v[q], make_float2(w.x, sign > 0.f ? -w.y : w.y));
            }
        }
        const int base = off + jq * Ns * R + k;
#pragma unroll
        for (int p = 0; p < R; ++p) {
            float2 y = v[0];
#pragma unroll
            for (int q = 1; q < R; ++q) {
                const float2 w = root[(p * q) % R];
                y.x += v[q].x * w.x - v[q].y * w.y;
                y.y += v[q].x * w.y + v[q].y * w.x;
            }
            dst[base + p * Ns] = y;
        }
    }
}

// all stages of one transform; returns the region holding the result
__device__ float2 *fft_rows(float2 *a, float2 *b, int nitem, int rows, int n, int S,
                            const int *rad, int nrad, const int *twoff, const float2 *tab,
                            float sign)
{
    int Ns = 1;
    for (int s = 0; s < nrad; ++s) {
        const float2 *tw = tab + twoff[s];
        switch (rad[s]) {
        case 2: stage<2>(a, b, nitem, rows, n, S, Ns, sign, tw); break;
        case 3: stage<3>(a, b, nitem, rows, n, S, Ns, sign, tw); break;
        case 4: stage<4>(a, b, nitem, rows, n, S, Ns, sign, tw); break;
        case 5: stage<5>(a, b, nitem, rows, n, S, Ns, sign, tw); break;
        default: stage<7>(a, b, nitem, rows, n, S, Ns, sign, tw); break;
        }
        Ns *= rad[s];
        __syncthreads();
        float2 *t = a;
        a = b;
        b = t;
    }
    return a;
}

// spectrum of length nin -> zero-padded spectrum of length nout, keeping
// |f| <= lb, scaled by 1 / nin; `ph` (circle grids) holds the half-sample
// phase exp(i pi f (1/nout - 1/nin)) per output index, else null
__device__ void pad(const float2 *__restrict__ src, float2 *__restrict__ dst, int nitem,
                    int rows, int nin, int nout, int S, int lb, const float2 *ph)
{
    const int per_item = rows * nout;
    const int total = nitem * per_item;
    const float inv_item = 1.0f / (float)per_item, inv_out = 1.0f / (float)nout;
    const float scale = 1.0f / (float)nin;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const int t = fdiv(e, per_item, inv_item);
        const int re = e - t * per_item;
        const int r = fdiv(re, nout, inv_out);
        const int o = re - r * nout;
        const int f = (2 * o <= nout) ? o : o - nout;
        float2 v = make_float2(0.f, 0.f);
        if (f <= lb && f >= -lb) {
            const int fi = f >= 0 ? f : f + nin;
            const float2 x = src[t * S + r * nin + fi];
            v = make_float2(x.x * scale, x.y * scale);
            if (ph) v = cmul(v, ph[o]);
        }
        dst[t * S + r * nout + o] = v;
    }
}

// [nt][P] grid -> P/2 circles of 2 nt samples
__device__ void fold(const float2 *__restrict__ src, float2 *__restrict__ dst, int nitem, int nt,
                     int P, int S)
{
    const int c = 2 * nt, h = P / 2;
    const int per_item = h * c;
    const int total = nitem * per_item;
    const float inv_item = 1.0f / (float)per_item, inv_c = 1.0f / (float)c;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const int t = fdiv(e, per_item, inv_item);
        const int re = e - t * per_item;
        const int j = fdiv(re, c, inv_c);
        const int s = re - j * c;
        const int from = s < nt ? s * P + j : (c - 1 - s) * P + j + h;
        dst[t * S + re] = src[t * S + from];
    }
}

// P/2 circles of 2 nt samples -> [nt][P] grid
__device__ void unfold(const float2 *__restrict__ src, float2 *__restrict__ dst, int nitem,
                       int nt, int P, int S)
{
    const int c = 2 * nt, h = P / 2;
    const int per_item = nt * P;
    const int total = nitem * per_item;
    const float inv_item = 1.0f / (float)per_item, inv_p = 1.0f / (float)P;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const int t = fdiv(e, per_item, inv_item);
        const int re = e - t * per_item;
        const int i = fdiv(re, P, inv_p);
        const int j = re - i * P;
        const int from = j < h ? j * c + i : (j - h) * c + c - 1 - i;
        dst[t * S + re] = src[t * S + from];
    }
}

__global__ void __launch_bounds__(kMaxThreads)
k_fft_resample(const float2 *__restrict__ in, float2 *__restrict__ out, int64_t nitems,
               FftDesc d)
{
    extern __shared__ float2 lds[];
    const int64_t it0 = (int64_t)blockIdx.x * d.ipw;
    const int nitem = (int)((nitems - it0) < d.ipw ? (nitems - it0) : d.ipw);
    float2 *a = lds, *b = lds + (size_t)d.ipw * d.S;
    float2 *tab = lds + (size_t)2 * d.ipw * d.S;
    for (int e = threadIdx.x; e < d.ntab; e += blockDim.x) tab[e] = d.tab[e];
    const float2 *ph = tab + d.tab_phase;
    // load (rows scaled by the input weights when anterpolating)
    {
        const int per_item = d.ti * d.pi;
        const int total = nitem * per_item;
        const float inv_item = 1.0f / (float)per_item, inv_p = 1.0f / (float)d.pi;
        const float2 *src = in + it0 * per_item;
        for (int e = threadIdx.x; e < total; e += blockDim.x) {
            const int t = fdiv(e, per_item, inv_item);
            const int re = e - t * per_item;
            float2 v = src[e];
            if (d.pre) {
                const float w = d.pre[fdiv(re, d.pi, inv_p)];
                v = make_float2(v.x * w, v.y * w);
            }
            a[t * d.S + re] = v;
        }
    }
    __syncthreads();
    float2 *r;
    if (!d.down) {
        r = fft_rows(a, b, nitem, d.ti, d.pi, d.S, d.ri, d.nri, d.twi, tab, -1.f);
        float2 *o = r == a ? b : a;
        pad(r, o, nitem, d.ti, d.pi, d.po, d.S, d.lb, nullptr);
        __syncthreads();
        r = fft_rows(o, r, nitem, d.ti, d.po, d.S, d.ro, d.nro, d.two, tab, 1.f);
        o = r == a ? b : a;
        fold(r, o, nitem, d.ti, d.po, d.S);
        __syncthreads();
        r = fft_rows(o, r, nitem, d.po / 2, d.pi, d.S, d.ri, d.nri, d.twi, tab, -1.f);
        o = r == a ? b : a;
        pad(r, o, nitem, d.po / 2, d.pi, d.po, d.S, d.lb, ph);
        __syncthreads();
        r = fft_rows(o, r, nitem, d.po / 2, d.po, d.S, d.ro, d.nro, d.two, tab, 1.f);
        o = r == a ? b : a;
        unfold(r, o, nitem, d.to, d.po, d.S);
        __syncthreads();
        r = o;
    } else {
        fold(a, b, nitem, d.ti, d.pi, d.S);
        __syncthreads();
        r = fft_rows(b, a, nitem, d.pi / 2, d.pi, d.S, d.ri, d.nri, d.twi, tab, -1.f);
        float2 *o = r == a ? b : a;
        pad(r, o, nitem, d.pi / 2, d.pi, d.po, d.S, d.lb, ph);
        __syncthreads();
        r = fft_rows(o, r, nitem, d.pi / 2, d.po, d.S, d.ro, d.nro, d.two, tab, 1.f);
        o = r == a ? b : a;
        unfold(r, o, nitem, d.to, d.pi, d.S);
        __syncthreads();
        r = fft_rows(o, r, nitem, d.to, d.pi, d.S, d.ri, d.nri, d.twi, tab, -1.f);
        o = r == a ? b : a;
        pad(r, o, nitem, d.to, d.pi, d.po, d.S, d.lb, nullptr);
        __syncthreads();
        r = fft_rows(o, r, nitem, d.to, d.po, d.S, d.ro, d.nro, d.two, tab, 1.f);
    }
    // store (rows scaled by the output factors when anterpolating)
    {
        const int per_item = d.to * d.po;
        const int total = nitem * per_item;
        const float inv_item = 1.0f / (float)per_item, inv_p = 1.0f / (float)d.po;
        float2 *dst = out + it0 * per_item;
        for (int e = threadIdx.x; e < total; e += blockDim.x) {
            const int t = fdiv(e, per_item, inv_item);
            const int re = e - t * per_item;
            float2 v = r[t * d.S + re];
            if (d.post) {
                const float w = d.post[fdiv(re, d.po, inv_p)];
                v = make_float2(v.x * w, v.y * w);
            }
            dst[e] = v;
        }
    }
}

// radices of n (4s first, then 2, 3, 5, 7); false if n has another factor
bool radix_plan(int n, int *rad, int *nrad)
{
    int m = n, c = 0;
    while (m % 4 == 0 && c < kMaxRadices) rad[c++] = 4, m /= 4;
    for (int r : {2, 3, 5, 7})
        while (m % r == 0 && c < kMaxRadices) rad[c++] = r, m /= r;
    *nrad = c;
    return m == 1;
}

// forward twiddles of every stage of a length-n transform, appended to tab;
// off[s] = offset of stage s (its Ns (R - 1) values, [k][q - 1])
void twiddles(int n, const int *rad, int nrad, int *off, std::vector<float2> &tab)
{
    const double pi = 3.14159265358979323846;
    int Ns = 1;
    for (int s = 0; s < nrad; ++s) {
        const int R = rad[s];
        off[s] = (int)tab.size();
        if (Ns > 1)
            for (int k = 0; k < Ns; ++k)
                for (int q = 1; q < R; ++q) {
                    const double a = -2.0 * pi * q * k / ((double)Ns * R);
                    tab.push_back(make_float2((float)std::cos(a), (float)std::sin(a)));
                }
        Ns *= R;
    }
    (void)n;
}

// Fejer's first rule on theta_i = (i + 1/2) pi / nt, FP64
std::vector<double> fejer(int nt)
{
    std::vector<double> w(nt);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < nt; ++i) {
        const double th = (i + 0.5) * pi / nt;
        double s = 0.0;
        for (int k = 1; k <= nt / 2; ++k) s += std::cos(2.0 * k * th) / (4.0 * k * k - 1.0);
        w[i] = 2.0 / nt * (1.0 - 2.0 * s);
    }
    return w;
}

}  // namespace
}  // namespace dev
}  // namespace mlfma

struct mlfma_fft_s {
    int device = 0;
    mlfma::dev::FftDesc desc{};
    size_t lds_bytes = 0;
    int threads = 256;
    float *d_scale = nullptr;  // [ti] input scales then [to] output scales
    float2 *d_tab = nullptr;   // twiddles and circle phases
};

using mlfma::fail;

extern "C" {

int mlfma_fft_plan(int lband, int nphi_in, int nphi_out, int anterpolate, int device,
                   mlfma_fft_t *out)
{
    using namespace mlfma::dev;
    if (!out) return fail(MLFMA_EINVAL, "fft_plan: out is NULL");
    *out = nullptr;
    if (lband < 0) return fail(MLFMA_EINVAL, "fft_plan: lband %d < 0", lband);
    for (int p : {nphi_in, nphi_out}) {
        if (p < 2 || p % 2 || p > 1024)
            return fail(MLFMA_EINVAL, "fft_plan: phi count %d not even in [2, 1024]", p);
        if (p < 2 * lband + 2)
            return fail(MLFMA_EINVAL, "fft_plan: phi count %d below 2 lband + 2 = %d", p,
                        2 * lband + 2);
    }
    FftDesc d{};
    d.pi = nphi_in;
    d.po = nphi_out;
    d.ti = nphi_in / 2;
    d.to = nphi_out / 2;
    d.lb = lband;
    d.down = anterpolate ? 1 : 0;
    if (!radix_plan(d.pi, d.ri, &d.nri) || !radix_plan(d.po, d.ro, &d.nro))
        return fail(MLFMA_EINVAL, "fft_plan: phi counts %d, %d must have no prime factor "
                    "above 7", nphi_in, nphi_out);
    // largest array of either pipeline
    const int64_t sz[] = {(int64_t)d.ti * d.pi, (int64_t)d.ti * d.po,
                          (int64_t)(d.po / 2) * d.pi, (int64_t)(d.po / 2) * d.po,
                          (int64_t)d.to * d.po, (int64_t)d.to * d.pi,
                          (int64_t)(d.pi / 2) * d.po};
    int64_t S = 0;
    for (int64_t v : sz) S = v > S ? v : S;
    std::vector<float2> tab;
    twiddles(d.pi, d.ri, d.nri, d.twi, tab);
    twiddles(d.po, d.ro, d.nro, d.two, tab);
    d.tab_phase = (int)tab.size();
    {
        // half-sample phase of the circle resampling (P_in -> P_out
        // samples) for output index o, frequency f = o or o - P_out
        const double pi = 3.14159265358979323846;
        for (int o = 0; o < d.po; ++o) {
            const int f = 2 * o <= d.po ? o : o - d.po;
            const double a = pi * f * (1.0 / d.po - 1.0 / d.pi);
            tab.push_back(make_float2((float)std::cos(a), (float)std::sin(a)));
        }
    }
    d.ntab = (int)tab.size();
    const int64_t per_item = 2 * S * (int64_t)sizeof(float2);
    const int64_t tab_bytes = (int64_t)d.ntab * (int64_t)sizeof(float2);
    constexpr int64_t kLdsMax = 160 * 1024, kLdsTarget = 40 * 1024;
    if (per_item + tab_bytes > kLdsMax)
        return fail(MLFMA_EINVAL, "fft_plan: one item needs %lld bytes of LDS (> 160 KiB); "
                    "phi counts %d, %d too large", (long long)(per_item + tab_bytes),
                    nphi_in, nphi_out);
    int ipw = (int)(kLdsTarget / per_item);
    ipw = ipw < 1 ? 1 : (ipw > 16 ? 16 : ipw);
    d.ipw = ipw;
    d.S = (int)S;

    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return fail(MLFMA_EDEVICE, "fft_plan: no HIP device");
    if (cur != device && hipSetDevice(device) != hipSuccess)
        return fail(MLFMA_EDEVICE, "fft_plan: hipSetDevice(%d) failed", device);
    mlfma_fft_s *p = new (std::nothrow) mlfma_fft_s;
    if (!p) {
        if (cur != device) (void)hipSetDevice(cur);
        return fail(MLFMA_ENOMEM, "fft_plan: host allocation");
    }
    p->device = device;
    int rc = MLFMA_OK;
    {
        hipError_t e = hipMalloc(&p->d_tab, tab.size() * sizeof(float2));
        if (e != hipSuccess) {
            p->d_tab = nullptr;
            rc = fail(MLFMA_ENOMEM, "fft_plan: hipMalloc: %s", hipGetErrorString(e));
        } else if ((e = hipMemcpy(p->d_tab, tab.data(), tab.size() * sizeof(float2),
                                  hipMemcpyHostToDevice)) != hipSuccess) {
            rc = fail(MLFMA_EDEVICE, "fft_plan: hipMemcpy: %s", hipGetErrorString(e));
        }
        d.tab = p->d_tab;
    }
    if (rc == MLFMA_OK && d.down) {
        const std::vector<double> wi = fejer(d.ti), wo = fejer(d.to);
        std::vector<float> h(d.ti + d.to);
        for (int i = 0; i < d.ti; ++i) h[i] = (float)wi[i];
        const double ratio = (double)d.pi / (double)d.po;
        for (int i = 0; i < d.to; ++i) h[d.ti + i] = (float)(ratio / wo[i]);
        hipError_t e = hipMalloc(&p->d_scale, h.size() * sizeof(float));
        if (e != hipSuccess) {
            p->d_scale = nullptr;
            rc = fail(MLFMA_ENOMEM, "fft_plan: hipMalloc: %s", hipGetErrorString(e));
        } else if ((e = hipMemcpy(p->d_scale, h.data(), h.size() * sizeof(float),
                                  hipMemcpyHostToDevice)) != hipSuccess) {
            rc = fail(MLFMA_EDEVICE, "fft_plan: hipMemcpy: %s", hipGetErrorString(e));
        }
        d.pre = p->d_scale;
        d.post = p->d_scale ? p->d_scale + d.ti : nullptr;
    }
    if (rc == MLFMA_OK) {
        // (gfx950 launches up to 160 KiB of dynamic LDS without the
        // attribute; it is set for portability of the request only)
        p->lds_bytes = (size_t)((2 * (int64_t)d.ipw * S + d.ntab) * (int64_t)sizeof(float2));
        // one large item per workgroup: more threads share its transforms
        p->threads = (d.ipw == 1 && S >= 4096) ? kMaxThreads : 256;
        if (p->lds_bytes > 64 * 1024)
            (void)hipFuncSetAttribute((const void *)k_fft_resample,
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)p->lds_bytes);
    }
    if (cur != device) (void)hipSetDevice(cur);
    if (rc != MLFMA_OK) {
        if (p->d_scale) (void)hipFree(p->d_scale);
        if (p->d_tab) (void)hipFree(p->d_tab);
        delete p;
        return rc;
    }
    p->desc = d;
    *out = p;
    return MLFMA_OK;
}

int mlfma_fft_execute(mlfma_fft_t p, const void *in, void *out, int64_t nitems, void *stream)
{
    using namespace mlfma::dev;
    if (!p) return fail(MLFMA_EINVAL, "fft_execute: plan is NULL");
    if (nitems < 0) return fail(MLFMA_EINVAL, "fft_execute: nitems %lld < 0", (long long)nitems);
    if (nitems == 0) return MLFMA_OK;
    if (!in || !out) return fail(MLFMA_EINVAL, "fft_execute: null buffer");
    {
        // the batch is read and written by different workgroups: in and out
        // must not overlap
        const uintptr_t i0 = (uintptr_t)in, o0 = (uintptr_t)out;
        const uintptr_t i1 = i0 + (uintptr_t)nitems * p->desc.ti * p->desc.pi * sizeof(float2);
        const uintptr_t o1 = o0 + (uintptr_t)nitems * p->desc.to * p->desc.po * sizeof(float2);
        if (i0 < o1 && o0 < i1) return fail(MLFMA_EINVAL, "fft_execute: in and out overlap");
    }
    const int64_t nblk = (nitems + p->desc.ipw - 1) / p->desc.ipw;
    if (nblk > 0x7fffffffll) return fail(MLFMA_EINVAL, "fft_execute: batch too large");
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return fail(MLFMA_EDEVICE, "fft_execute: no device");
    if (cur != p->device && hipSetDevice(p->device) != hipSuccess)
        return fail(MLFMA_EDEVICE, "fft_execute: hipSetDevice(%d) failed", p->device);
    hipLaunchKernelGGL(k_fft_resample, dim3((unsigned)nblk), dim3(p->threads), p->lds_bytes,
                       (hipStream_t)stream, (const float2 *)in, (float2 *)out, nitems, p->desc);
    hipError_t e = hipGetLastError();
    if (cur != p->device) (void)hipSetDevice(cur);
    if (e != hipSuccess)
        return fail(MLFMA_EDEVICE, "fft_execute: launch: %s", hipGetErrorString(e));
    return MLFMA_OK;
}

int mlfma_fft_info(mlfma_fft_t p, int *items_per_workgroup, int64_t *lds_bytes)
{
    if (!p) return fail(MLFMA_EINVAL, "fft_info: plan is NULL");
    if (items_per_workgroup) *items_per_workgroup = p->desc.ipw;
    if (lds_bytes) *lds_bytes = (int64_t)p->lds_bytes;
    return MLFMA_OK;
}

void mlfma_fft_destroy(mlfma_fft_t p)
{
    if (!p) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != p->device) (void)hipSetDevice(p->device);
    if (p->d_scale) (void)hipFree(p->d_scale);
    if (p->d_tab) (void)hipFree(p->d_tab);
    if (cur != p->device) (void)hipSetDevice(cur);
    delete p;
}

}  // extern "C"
