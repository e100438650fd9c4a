// Pressure mass-matrix CG of the Stokes preconditioner Q_t (Sec. 5, the
// Schur complement replaced by the pressure mass matrix, solved by
// diagonally preconditioned CG as in the paper's Stokes experiments).  FP64.
// The mass matrix has about 15 entries per row and n_p = n_v rows, a few per
// cent of the velocity work of one Q_t application, so the kernels are plain
// grid-stride passes; their reductions write one partial per workgroup that
// the CG's finish kernel sums in a fixed order.
#include <hip/hip_runtime.h>

#include "stokes.hpp"

namespace auxp {

namespace {

inline int mass_grid(int n)
{
    int g = (n + kBlock - 1) / kBlock;
    return g < 1 ? 1 : (g > kMaxBlocks ? kMaxBlocks : g);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// partials[blockIdx.x] (and partials2[blockIdx.x]) = the workgroup's sums
__device__ __forceinline__ void write_pair(double a, double *pa, double b, double *pb)
{
    __shared__ double red[2][kBlock / 64];
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x / 64;
    if (threadIdx.x % 64 == 0) {
        red[0][w] = a;
        red[1][w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0.0, s1 = 0.0;
        for (int k = 0; k < kBlock / 64; k++) {
            s0 += red[0][k];
            s1 += red[1][k];
        }
        pa[blockIdx.x] = s0;
        if (pb) pb[blockIdx.x] = s1;
    }
}

__global__ __launch_bounds__(kBlock) void k_mass_start(int n, const double *__restrict__ b,
                                                       const double *__restrict__ dinv, double *__restrict__ x,
                                                       double *__restrict__ r, double *__restrict__ z,
                                                       double *__restrict__ partials)
{
    double bb = 0.0, rz = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const double bi = b[i], zi = dinv[i] * bi;
        x[i] = 0.0;
        r[i] = bi;
        z[i] = zi;
        bb += bi * bi;
        rz += bi * zi;
    }
    write_pair(bb, partials, rz, partials + kMaxBlocks);
}

__global__ __launch_bounds__(kBlock) void k_mass_product(int n, const int *__restrict__ ptr,
                                                         const int *__restrict__ col, const double *__restrict__ val,
                                                         const double *__restrict__ p, double *__restrict__ q,
                                                         double *__restrict__ partials, CgState st)
{
    if (*st.done) return;
    double pq = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        double s = 0.0;
        for (int e = ptr[i]; e < ptr[i + 1]; e++) s += val[e] * p[col[e]];
        q[i] = s;
        pq += p[i] * s;
    }
    write_pair(pq, partials, 0.0, nullptr);
}

__global__ __launch_bounds__(kBlock) void k_mass_update(int n, double *__restrict__ x, double *__restrict__ r,
                                                        const double *__restrict__ p, const double *__restrict__ q,
                                                        const double *__restrict__ dinv, double *__restrict__ z,
                                                        double *__restrict__ partials, CgState st)
{
    if (*st.done) return;
    const int k = *st.iter;
    const double alpha = st.rz[k] / st.pq[k];
    double rr = 0.0, rz = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i], zi = dinv[i] * ri;
        r[i] = ri;
        z[i] = zi;
        rr += ri * ri;
        rz += ri * zi;
    }
    write_pair(rr, partials, rz, partials + kMaxBlocks);
}

__global__ __launch_bounds__(kBlock) void k_negate(int n, const double *__restrict__ x, double *__restrict__ y)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) y[i] = -x[i];
}

}  // namespace

int mass_start(hipStream_t s, int n, const double *b, const double *dinv, double *x, double *r, double *z,
               double *partials)
{
    const int g = mass_grid(n);
    hipLaunchKernelGGL(k_mass_start, dim3(g), dim3(kBlock), 0, s, n, b, dinv, x, r, z, partials);
    return g;
}

int mass_product(hipStream_t s, const DevCsrView &M, const double *p, double *q, double *partials,
                 const CgState &st)
{
    const int g = mass_grid(M.n);
    hipLaunchKernelGGL(k_mass_product, dim3(g), dim3(kBlock), 0, s, M.n, M.ptr, M.col, (const double *)M.val, p, q,
                       partials, st);
    return g;
}

int mass_update(hipStream_t s, int n, double *x, double *r, const double *p, const double *q, const double *dinv,
                double *z, double *partials, const CgState &st)
{
    const int g = mass_grid(n);
    hipLaunchKernelGGL(k_mass_update, dim3(g), dim3(kBlock), 0, s, n, x, r, p, q, dinv, z, partials, st);
    return g;
}

void vec_negate(hipStream_t s, int n, const double *x, double *y)
{
    hipLaunchKernelGGL(k_negate, dim3(mass_grid(n)), dim3(kBlock), 0, s, n, x, y);
}

}  // namespace auxp
