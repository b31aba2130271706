// Vector kernels of the restarted GMRES solve built on the matvec (the
// iterative solver of the integral equations the potential sum comes from,
// Sec. 1 and Sec. 2).  Krylov vectors are complex64 rows of length n;
// inner products and the Gram-Schmidt coefficients are carried in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace mlfma {
namespace dev {

namespace {

constexpr int kDotThreads = 256;

// partial[i * gridDim.x + blockIdx.x] = sum over this block's share of j of
// conj(V[i][j]) w[j], for row i = blockIdx.y (FP64 accumulation)
__global__ void __launch_bounds__(kDotThreads)
k_gm_dots(const float2 *__restrict__ V, int64_t ldv, const float2 *__restrict__ w, int64_t n,
          double2 *__restrict__ partial)
{
    __shared__ double2 red[kDotThreads];
    const int i = blockIdx.y;
    const float2 *v = V + (int64_t)i * ldv;
    double re = 0.0, im = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * kDotThreads) {
        const float2 a = v[j], b = w[j];
        re += (double)a.x * b.x + (double)a.y * b.y;
        im += (double)a.x * b.y - (double)a.y * b.x;
    }
    red[threadIdx.x] = make_double2(re, im);
    __syncthreads();
    for (int h = kDotThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[threadIdx.x].x += red[threadIdx.x + h].x;
            red[threadIdx.x].y += red[threadIdx.x + h].y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)i * gridDim.x + blockIdx.x] = red[0];
}

// w[j] += sign * sum_{i < m} V[i][j] c[i]
__global__ void __launch_bounds__(256)
k_gm_combine(float2 *__restrict__ w, const float2 *__restrict__ V, int64_t ldv, int m,
             const double2 *__restrict__ c, double sign, int64_t n)
{
    extern __shared__ double2 cs[];
    for (int i = threadIdx.x; i < m; i += blockDim.x) cs[i] = c[i];
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double re = 0.0, im = 0.0;
    for (int i = 0; i < m; ++i) {
        const float2 v = V[(int64_t)i * ldv + j];
        const double2 a = cs[i];
        re += a.x * v.x - a.y * v.y;
        im += a.x * v.y + a.y * v.x;
    }
    const float2 o = w[j];
    w[j] = make_float2((float)(o.x + sign * re), (float)(o.y + sign * im));
}

// y[j] = a x[j] + b y[j]
__global__ void __launch_bounds__(256)
k_gm_axpby(float2 *y, double2 a, const float2 *x, double2 b, int64_t n)  // x may be y
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    // a zero coefficient drops its term (y or x may hold uninitialised data)
    double re = 0.0, im = 0.0;
    if (a.x != 0.0 || a.y != 0.0) {
        const float2 u = x[j];
        re += a.x * u.x - a.y * u.y;
        im += a.x * u.y + a.y * u.x;
    }
    if (b.x != 0.0 || b.y != 0.0) {
        const float2 v = y[j];
        re += b.x * v.x - b.y * v.y;
        im += b.x * v.y + b.y * v.x;
    }
    y[j] = make_float2((float)re, (float)im);
}

}  // namespace

int gm_dot_blocks(int64_t n)
{
    const int64_t nb = (n + 8 * kDotThreads - 1) / (8 * kDotThreads);
    return (int)std::max<int64_t>(1, std::min<int64_t>(512, nb));
}

hipError_t gm_dots(const float2 *V, int64_t ldv, int m, const float2 *w, int64_t n, int nb,
                   double2 *partial, hipStream_t s)
{
    if (m <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gm_dots, dim3((unsigned)nb, (unsigned)m), dim3(kDotThreads), 0, s, V,
                       ldv, w, n, partial);
    return hipGetLastError();
}

hipError_t gm_combine(float2 *w, const float2 *V, int64_t ldv, int m, const double2 *c,
                      double sign, int64_t n, hipStream_t s)
{
    if (m <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gm_combine, dim3((unsigned)((n + 255) / 256)), dim3(256),
                       (size_t)m * sizeof(double2), s, w, V, ldv, m, c, sign, n);
    return hipGetLastError();
}

hipError_t gm_axpby(float2 *y, double2 a, const float2 *x, double2 b, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gm_axpby, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y, a, x,
                       b, n);
    return hipGetLastError();
}

}  // namespace dev
}  // namespace mlfma
