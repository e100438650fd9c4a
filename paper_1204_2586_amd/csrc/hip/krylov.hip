// Vector kernels of the flexible GMRES(m) outer iteration: the Arnoldi step
// orthogonalises A z_j against the basis v_0..v_j by classical Gram-Schmidt
// applied twice, so each pass is a set of dot products with the whole basis
// (one read of every basis vector, the new vector read once per group of
// eight) followed by one combined update, rather than j dependent
// dot/update pairs as modified Gram-Schmidt needs.  Everything is FP64 and
// streams HBM; the sums are in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.hpp"
#include "krylov.hpp"

namespace auxp {

namespace {

constexpr int kGroup = 8;   // basis vectors per workgroup of k_multi_dot

__device__ __forceinline__ double wave_total(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// partials[v * gridDim.x + blockIdx.x]: this workgroup's share of V_v . w
// for the group of vectors blockIdx.y
__global__ __launch_bounds__(kBlock) void k_multi_dot(int n, int nv, const double *__restrict__ V, long long ld,
                                                      const double *w, double *__restrict__ partials)
{
    const int v0 = blockIdx.y * kGroup;
    const int cnt = min(kGroup, nv - v0);
    const double *__restrict__ base = V + (long long)v0 * ld;
    double acc[kGroup];
#pragma unroll
    for (int v = 0; v < kGroup; v++) acc[v] = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const double wi = w[i];
#pragma unroll
        for (int v = 0; v < kGroup; v++)
            if (v < cnt) acc[v] += base[(long long)v * ld + i] * wi;
    }
    __shared__ double red[kGroup][kBlock / 64];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
    for (int v = 0; v < kGroup; v++) {
        const double s = wave_total(acc[v]);
        if (lane == 0) red[v][wave] = s;
    }
    __syncthreads();
    if (threadIdx.x < cnt) {
        double s = 0.0;
        for (int k = 0; k < kBlock / 64; k++) s += red[threadIdx.x][k];
        partials[(long long)(v0 + threadIdx.x) * gridDim.x + blockIdx.x] = s;
    }
}

// out[blockIdx.x] = sum of the nparts partials of vector blockIdx.x
__global__ __launch_bounds__(kBlock) void k_sum_partials(int nparts, const double *__restrict__ partials,
                                                         double *__restrict__ out)
{
    const double *p = partials + (long long)blockIdx.x * nparts;
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kBlock) s += p[i];
    __shared__ double red[kBlock / 64];
    s = wave_total(s);
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kBlock / 64; k++) t += red[k];
        out[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_multi_axpy(int n, int nv, const double *__restrict__ V, long long ld,
                                                       const double *__restrict__ c, double sign,
                                                       double *__restrict__ w, double *__restrict__ partials)
{
    double acc = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        // four independent chains keep four basis loads in flight
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int v = 0;
        for (; v + 4 <= nv; v += 4) {
            s0 += c[v] * V[(long long)v * ld + i];
            s1 += c[v + 1] * V[(long long)(v + 1) * ld + i];
            s2 += c[v + 2] * V[(long long)(v + 2) * ld + i];
            s3 += c[v + 3] * V[(long long)(v + 3) * ld + i];
        }
        for (; v < nv; v++) s0 += c[v] * V[(long long)v * ld + i];
        const double y = w[i] + sign * ((s0 + s1) + (s2 + s3));
        w[i] = y;
        acc += y * y;
    }
    if (!partials) return;
    __shared__ double red[kBlock / 64];
    acc = wave_total(acc);
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kBlock / 64; k++) t += red[k];
        partials[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_scale_unit(int n, const double *w, const double *__restrict__ nrm2,
                                                       double *out)
{
    const double q = *nrm2;
    const double inv = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) out[i] = w[i] * inv;
}

__global__ __launch_bounds__(kBlock) void k_sub_from(int n, const double *__restrict__ a, double *__restrict__ y)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) y[i] = a[i] - y[i];
}

int krylov_grid(int n)
{
    long long g = ((long long)n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > kKrylovBlocks) g = kKrylovBlocks;
    return (int)g;
}

}  // namespace

void multi_dot(hipStream_t s, int n, int nv, const double *V, long long ld, const double *w, double *partials,
               double *out)
{
    if (nv < 1) return;
    const int g = krylov_grid(n);
    hipLaunchKernelGGL(k_multi_dot, dim3(g, (nv + kGroup - 1) / kGroup), dim3(kBlock), 0, s, n, nv, V, ld, w,
                       partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(nv), dim3(kBlock), 0, s, g, (const double *)partials, out);
}

void multi_axpy(hipStream_t s, int n, int nv, const double *V, long long ld, const double *c, double sign, double *w,
                double *partials, double *nrm2)
{
    const int g = krylov_grid(n);
    hipLaunchKernelGGL(k_multi_axpy, dim3(g), dim3(kBlock), 0, s, n, nv, V, ld, c, sign, w,
                       nrm2 ? partials : nullptr);
    if (nrm2) hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, g, (const double *)partials, nrm2);
}

void scale_unit(hipStream_t s, int n, const double *w, const double *nrm2, double *out)
{
    hipLaunchKernelGGL(k_scale_unit, dim3(krylov_grid(n)), dim3(kBlock), 0, s, n, w, nrm2, out);
}

void sub_from(hipStream_t s, int n, const double *a, double *y)
{
    hipLaunchKernelGGL(k_sub_from, dim3(krylov_grid(n)), dim3(kBlock), 0, s, n, a, y);
}

}  // namespace auxp
