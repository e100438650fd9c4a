// Pressure mass-matrix CG of the Stokes preconditioner Q_t (Sec. 5, the
// Schur complement replaced by the pressure mass matrix, solved by
// diagonally preconditioned CG as in the paper's Stokes experiments).  FP64.
// The mass matrix is a few per cent of the velocity work of one Q_t
// application: the product runs a few lanes per row, the vector steps are
// grid-stride passes; their reductions write one partial per workgroup that
// the CG's finish kernel sums in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>

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

// q = M p with LPR lanes per row (rows of M_p hold 15 entries at P1 and
// about 40 at P2 on the benchmark meshes; one lane per row left each lane a
// chain of dependent loads over the whole row, 241 us per product at P2
// 32^3) and the partial sums of p.q.  (Forming p = z + beta p_old inside the
// product, from both vectors gathered, measured slower than the separate
// direction pass: 43.8 against 30.7 + 3.8 us at P2 32^3.)
template <int LPR>
__global__ __launch_bounds__(kBlock) void k_mass_product(int n, const int *__restrict__ ptr,
                                                         const int *__restrict__ col, const double *__restrict__ val,
                                                         const double *__restrict__ p, double *__restrict__ q,
                                                         double *__restrict__ partials, CgState st)
{
    if (*st.done) return;
    double pq = 0.0;
    const int sub = threadIdx.x % LPR;
    for (int base = blockIdx.x * (kBlock / LPR); base < n; base += gridDim.x * (kBlock / LPR)) {
        const int row = base + (int)(threadIdx.x / LPR);
        double s = 0.0;
        if (row < n) {
            const int e1 = ptr[row + 1];
#pragma unroll 4
            for (int e = ptr[row] + sub; e < e1; e += LPR) s += val[e] * p[col[e]];
        }
#pragma unroll
        for (int off = LPR / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, LPR);
        if (row < n && sub == 0) {
            q[row] = s;
            pq += p[row] * s;
        }
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

// One workgroup: the sums of the r.r and r.z partials (each in a fixed
// order), then the two finish steps of a CG iteration: r.r closes iteration
// k (k + 1 recorded, stop on the tolerance, the limit or a non-finite sum),
// r.z is recorded for k + 1 (stop when not positive) unless the solve stopped.
__global__ __launch_bounds__(kBlock) void k_mass_finish(const double *__restrict__ partials, int nparts, CgState st)
{
    if (*st.done) return;
    __shared__ double red[2][kBlock / 64];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kBlock) {
        a += partials[i];
        b += partials[kMaxBlocks + i];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (threadIdx.x % 64 == 0) {
        red[0][threadIdx.x / 64] = a;
        red[1][threadIdx.x / 64] = b;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double rr = 0.0, rz = 0.0;
    for (int w = 0; w < kBlock / 64; w++) {
        rr += red[0][w];
        rz += red[1][w];
    }
    const int k = *st.iter;
    st.rr[k + 1] = rr;
    *st.iter = k + 1;
    int d = 0;
    if (!std::isfinite(rr)) d = 4;
    else if (rr <= st.scal[2]) d = 1;
    else if (k + 1 >= st.maxit) d = 2;
    if (!d) {
        st.rz[k + 1] = rz;
        if (!std::isfinite(rz)) d = 4;
        else if (!(rz > 0.0)) d = 3;
    }
    if (d) *st.done = d;
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
    const int lpr = M.lpr >= 16 ? 16 : (M.lpr >= 8 ? 8 : 4);
    long long g = ((long long)M.n * lpr + kBlock - 1) / kBlock;
    g = g < 1 ? 1 : (g > kMaxBlocks ? kMaxBlocks : g);
    const double *v = (const double *)M.val;
    if (lpr == 16)
        hipLaunchKernelGGL(k_mass_product<16>, dim3(g), dim3(kBlock), 0, s, M.n, M.ptr, M.col, v, p, q, partials, st);
    else if (lpr == 8)
        hipLaunchKernelGGL(k_mass_product<8>, dim3(g), dim3(kBlock), 0, s, M.n, M.ptr, M.col, v, p, q, partials, st);
    else
        hipLaunchKernelGGL(k_mass_product<4>, dim3(g), dim3(kBlock), 0, s, M.n, M.ptr, M.col, v, p, q, partials, st);
    return (int)g;
}

void mass_finish(hipStream_t s, const double *partials, int nparts, const CgState &st)
{
    hipLaunchKernelGGL(k_mass_finish, dim3(1), dim3(kBlock), 0, s, partials, nparts, st);
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
