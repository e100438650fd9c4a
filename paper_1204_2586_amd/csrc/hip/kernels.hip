// Solve-phase kernels of the auxiliary-space preconditioned CG (gfx950).
//
// Memory-bound sparse work: every kernel streams its CSR operator once,
// gathers the vector it multiplies, and fuses the elementwise smoother and
// residual updates into the same pass (l1-Jacobi sweep = one pass over A).
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.hpp"

namespace auxp {

namespace {

__device__ __forceinline__ bool stop(const int *done) { return done != nullptr && *done != 0; }

template <int LPR, typename A>
__device__ __forceinline__ A group_sum(A v)
{
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, LPR);
    return v;
}

// sum_j a_ij x(col_j) over the row, lanes sub, sub+LPR, ...
template <int LPR, typename T, typename XF>
__device__ __forceinline__ T row_dot(const int *__restrict__ ptr, const int *__restrict__ col,
                                     const T *__restrict__ val, int row, int sub, XF x)
{
    T s = T(0);
    const int e1 = ptr[row + 1];
    for (int e = ptr[row] + sub; e < e1; e += LPR) s += val[e] * x(col[e]);
    return group_sum<LPR>(s);
}

__device__ double block_sum(double v)
{
    __shared__ double red[kBlock / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBlock / 64; i++) s += red[i];
    return s;   // valid in thread 0
}

// Deterministic grid reduction: the partial of each workgroup is stored, and
// the last workgroup to arrive sums all partials in index order.
// Returns true in thread 0 of the last workgroup (which then holds *total).
__device__ bool grid_reduce(double v, const Reduce &red, double *total)
{
    __shared__ int is_last;
    double b = block_sum(v);
    if (threadIdx.x == 0) {
        red.partials[blockIdx.x] = b;
        __threadfence();
        unsigned int t = atomicAdd(red.counter, 1u);
        is_last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
    double s = 0.0;
    for (int i = threadIdx.x; i < (int)gridDim.x; i += kBlock)
        s += __hip_atomic_load(&red.partials[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s = block_sum(s);
    if (threadIdx.x == 0) {
        *red.counter = 0u;
        *total = s;
        if (red.out) red.out[red.index ? *red.index : 0] = s;
        return true;
    }
    return false;
}

inline int grid_for(int n, int rows_per_block)
{
    long long g = ((long long)n + rows_per_block - 1) / rows_per_block;
    if (g < 1) g = 1;
    if (g > kMaxBlocks) g = kMaxBlocks;
    return (int)g;
}

#define FOR_ROWS(LPR, n)                                                               \
    const int sub_ = threadIdx.x % (LPR);                                              \
    for (int base_ = blockIdx.x * (kBlock / (LPR)); base_ < (n); base_ += gridDim.x * (kBlock / (LPR))) \
        for (int row = base_ + threadIdx.x / (LPR), once_ = 1; once_; once_ = 0)

// ------------------------------------------------------------- smoothers

template <typename T>
__global__ __launch_bounds__(kBlock) void k_jacobi0(int n, const T *__restrict__ dinv, const double *__restrict__ r,
                                                    T *__restrict__ z, T *__restrict__ rT, const int *done)
{
    if (stop(done)) return;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        T ri = (T)r[i];
        z[i] = dinv[i] * ri;
        if (rT) rT[i] = ri;
    }
}

template <typename T, int LPR>
__global__ __launch_bounds__(kBlock) void k_first2(int n, const int *__restrict__ ptr, const int *__restrict__ col,
                                                   const T *__restrict__ val, const T *__restrict__ dinv,
                                                   const double *__restrict__ r, T *__restrict__ z,
                                                   T *__restrict__ rT, const int *done)
{
    if (stop(done)) return;
    FOR_ROWS(LPR, n)
    {
        if (row < n) {
            // A z1 with z1 = D^{-1} r formed on the fly
            T s = row_dot<LPR>(ptr, col, val, row, sub_, [&](int j) { return dinv[j] * (T)r[j]; });
            if (sub_ == 0) {
                T ri = (T)r[row], di = dinv[row];
                T z1 = di * ri;
                z[row] = z1 + di * (ri - s);
                if (rT) rT[row] = ri;
            }
        }
    }
}

template <typename T, typename TR, typename TZ, int LPR, bool DOT>
__global__ __launch_bounds__(kBlock) void k_sweep(int n, const int *__restrict__ ptr, const int *__restrict__ col,
                                                  const T *__restrict__ val, const T *__restrict__ dinv,
                                                  const TR *__restrict__ rhs, const T *__restrict__ zin,
                                                  TZ *__restrict__ zout, const double *__restrict__ rdot,
                                                  Reduce red, const int *done)
{
    if (stop(done)) return;
    double acc = 0.0;
    FOR_ROWS(LPR, n)
    {
        if (row < n) {
            T s = row_dot<LPR>(ptr, col, val, row, sub_, [&](int j) { return zin[j]; });
            if (sub_ == 0) {
                T zi = zin[row] + dinv[row] * ((T)rhs[row] - s);
                zout[row] = (TZ)zi;
                if (DOT) acc += rdot[row] * (double)(TZ)zi;
            }
        }
    }
    if (DOT) {
        double tot;
        grid_reduce(acc, red, &tot);
    }
}

template <typename T, int LPR>
__global__ __launch_bounds__(kBlock) void k_resid(int n, const int *__restrict__ ptr, const int *__restrict__ col,
                                                  const T *__restrict__ val, const T *__restrict__ rhs,
                                                  const T *__restrict__ z, T *__restrict__ res, const int *done)
{
    if (stop(done)) return;
    FOR_ROWS(LPR, n)
    {
        if (row < n) {
            T s = row_dot<LPR>(ptr, col, val, row, sub_, [&](int j) { return z[j]; });
            if (sub_ == 0) res[row] = rhs[row] - s;
        }
    }
}

template <typename T, int LPR, bool ADD>
__global__ __launch_bounds__(kBlock) void k_matvec(int n, const int *__restrict__ ptr, const int *__restrict__ col,
                                                   const T *__restrict__ val, const T *__restrict__ x,
                                                   T *__restrict__ y, const int *done)
{
    if (stop(done)) return;
    FOR_ROWS(LPR, n)
    {
        if (row < n) {
            T s = row_dot<LPR>(ptr, col, val, row, sub_, [&](int j) { return x[j]; });
            if (sub_ == 0) y[row] = ADD ? y[row] + s : s;
        }
    }
}

template <typename T, int LPR>
__global__ __launch_bounds__(kBlock) void k_vpre(int n, const int *__restrict__ ptr, const int *__restrict__ col,
                                                 const T *__restrict__ val, const T *__restrict__ dinv,
                                                 const T *__restrict__ b, T *__restrict__ x, T *__restrict__ r,
                                                 const int *done)
{
    if (stop(done)) return;
    FOR_ROWS(LPR, n)
    {
        if (row < n) {
            T s = row_dot<LPR>(ptr, col, val, row, sub_, [&](int j) { return dinv[j] * b[j]; });
            if (sub_ == 0) {
                x[row] = dinv[row] * b[row];
                r[row] = b[row] - s;
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dense_gemv(int n, const T *__restrict__ Ainv, const T *__restrict__ b,
                                                       T *__restrict__ x, const int *done)
{
    if (stop(done)) return;
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    for (int i = w; i < n; i += kBlock / 64) {
        T s = T(0);
        for (int j = l; j < n; j += 64) s += Ainv[(size_t)i * n + j] * b[j];
        s = group_sum<64>(s);
        if (l == 0) x[i] = s;
    }
}

// ---------------------------------------------------------------- FP64 CG

template <int LPR, bool DOT>
__global__ __launch_bounds__(kBlock) void k_spmv64(int n, const int *__restrict__ ptr, const int *__restrict__ col,
                                                   const double *__restrict__ val, const double *__restrict__ x,
                                                   double *__restrict__ y, Reduce red, const int *done)
{
    if (stop(done)) return;
    double acc = 0.0;
    FOR_ROWS(LPR, n)
    {
        if (row < n) {
            double s = row_dot<LPR>(ptr, col, val, row, sub_, [&](int j) { return x[j]; });
            if (sub_ == 0) {
                y[row] = s;
                if (DOT) acc += x[row] * s;
            }
        }
    }
    if (DOT) {
        double tot;
        grid_reduce(acc, red, &tot);
    }
}

template <int LPR>
__global__ __launch_bounds__(kBlock) void k_residual64(int n, const int *__restrict__ ptr, const int *__restrict__ col,
                                                       const double *__restrict__ val, const double *__restrict__ f,
                                                       const double *__restrict__ u, double *__restrict__ r)
{
    FOR_ROWS(LPR, n)
    {
        if (row < n) {
            double s = row_dot<LPR>(ptr, col, val, row, sub_, [&](int j) { return u[j]; });
            if (sub_ == 0) r[row] = f[row] - s;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_dot64(int n, const double *__restrict__ a, const double *__restrict__ b,
                                                  Reduce red)
{
    double acc = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) acc += a[i] * b[i];
    double tot;
    grid_reduce(acc, red, &tot);
}

__global__ void k_cg_init(CgState st, double tol2, const double *ff, const double *rr0)
{
    *st.iter = 0;
    double f2 = *ff, r2 = *rr0;
    st.rr[0] = r2;
    *st.tol2bb = tol2 * f2;
    int d = 0;
    if (!std::isfinite(f2) || !std::isfinite(r2)) d = 4;
    else if (r2 <= tol2 * f2) d = 1;          // includes f = 0
    else if (st.maxit <= 0) d = 2;
    *st.done = d;
}

__global__ __launch_bounds__(kBlock) void k_cg_update(int n, double *__restrict__ x, double *__restrict__ r,
                                                      const double *__restrict__ p, const double *__restrict__ q,
                                                      CgState st, Reduce red)
{
    if (*st.done) return;
    const int k = *st.iter;
    const double alpha = st.rz[k] / st.pq[k];
    double acc = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        x[i] += alpha * p[i];
        double ri = r[i] - alpha * q[i];
        r[i] = ri;
        acc += ri * ri;
    }
    double tot;
    if (grid_reduce(acc, red, &tot)) {
        st.rr[k + 1] = tot;
        *st.iter = k + 1;
        if (!std::isfinite(tot)) *st.done = 4;
        else if (tot <= *st.tol2bb) *st.done = 1;
        else if (k + 1 >= st.maxit) *st.done = 2;
    }
}

__global__ __launch_bounds__(kBlock) void k_cg_direction(int n, const double *__restrict__ z, double *__restrict__ p,
                                                         CgState st)
{
    if (*st.done) return;
    const int k = *st.iter;
    if (k == 0) {
        for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) p[i] = z[i];
        return;
    }
    const double beta = st.rz[k] / st.rz[k - 1];
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) p[i] = z[i] + beta * p[i];
}

__global__ void k_cg_check_rz(CgState st)
{
    if (*st.done) return;
    double v = st.rz[*st.iter];
    if (!std::isfinite(v)) *st.done = 4;
    else if (!(v > 0.0)) *st.done = 3;
}

__global__ void k_cg_check_pq(CgState st)
{
    if (*st.done) return;
    double v = st.pq[*st.iter];
    if (!std::isfinite(v)) *st.done = 4;
    else if (!(v > 0.0)) *st.done = 3;
}

// ------------------------------------------------------------- adjoint

__global__ __launch_bounds__(kBlock) void k_kappa_grad(int nt, int nloc, const int *__restrict__ tet_dof,
                                                       const double *__restrict__ G, const double *__restrict__ kappa,
                                                       const double *__restrict__ M, const double *__restrict__ u,
                                                       const double *__restrict__ lam, double *__restrict__ g)
{
    for (int t = blockIdx.x * kBlock + threadIdx.x; t < nt; t += gridDim.x * kBlock) {
        double ue[20], le[20];
        for (int a = 0; a < nloc; a++) {
            int i = tet_dof[(size_t)t * nloc + a];
            ue[a] = i >= 0 ? u[i] : 0.0;
            le[a] = i >= 0 ? lam[i] : 0.0;
        }
        double s = 0.0;
        for (int pq = 0; pq < 16; pq++) {
            const double *Mpq = M + (size_t)pq * nloc * nloc;
            double w = 0.0;
            for (int a = 0; a < nloc; a++) {
                double ra = 0.0;
                for (int b = 0; b < nloc; b++) ra += Mpq[a * nloc + b] * ue[b];
                w += le[a] * ra;
            }
            s += G[(size_t)t * 16 + pq] * w;
        }
        g[t] = -kappa[t] * s;
    }
}

__global__ void k_cast(int64_t n, const double *__restrict__ x, float *__restrict__ y)
{
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        y[i] = (float)x[i];
}

}  // namespace

int pick_lpr(double avg)
{
    if (avg <= 1.5) return 1;
    if (avg <= 3.0) return 2;
    if (avg <= 8.0) return 4;
    if (avg <= 24.0) return 8;
    if (avg <= 64.0) return 16;
    return 32;
}

#define LPR_SWITCH(lpr, CALL)                              \
    switch (lpr) {                                         \
    case 1: { constexpr int L = 1; CALL; } break;          \
    case 2: { constexpr int L = 2; CALL; } break;          \
    case 4: { constexpr int L = 4; CALL; } break;          \
    case 8: { constexpr int L = 8; CALL; } break;          \
    case 16: { constexpr int L = 16; CALL; } break;        \
    default: { constexpr int L = 32; CALL; } break;        \
    }

template <typename T>
void launch_jacobi0(hipStream_t s, int n, const T *dinv, const double *r, T *z, T *rT, const int *done)
{
    hipLaunchKernelGGL(k_jacobi0<T>, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, n, dinv, r, z, rT, done);
}

template <typename T>
void launch_first2(hipStream_t s, const DevCsrView &A, const T *dinv, const double *r, T *z, T *rT, const int *done)
{
    LPR_SWITCH(A.lpr, hipLaunchKernelGGL((k_first2<T, L>), dim3(grid_for(A.n, kBlock / L)), dim3(kBlock), 0, s, A.n,
                                         A.ptr, A.col, (const T *)A.val, dinv, r, z, rT, done));
}

template <typename T, typename TR, typename TZ>
void launch_sweep(hipStream_t s, const DevCsrView &A, const T *dinv, const TR *rhs, const T *zin, TZ *zout,
                  const double *rdot, const Reduce &red, const int *done)
{
    if (red.out) {
        LPR_SWITCH(A.lpr, hipLaunchKernelGGL((k_sweep<T, TR, TZ, L, true>), dim3(grid_for(A.n, kBlock / L)),
                                             dim3(kBlock), 0, s, A.n, A.ptr, A.col, (const T *)A.val, dinv, rhs, zin,
                                             zout, rdot, red, done));
    } else {
        LPR_SWITCH(A.lpr, hipLaunchKernelGGL((k_sweep<T, TR, TZ, L, false>), dim3(grid_for(A.n, kBlock / L)),
                                             dim3(kBlock), 0, s, A.n, A.ptr, A.col, (const T *)A.val, dinv, rhs, zin,
                                             zout, rdot, red, done));
    }
}

template <typename T>
void launch_resid(hipStream_t s, const DevCsrView &A, const T *rhs, const T *z, T *res, const int *done)
{
    LPR_SWITCH(A.lpr, hipLaunchKernelGGL((k_resid<T, L>), dim3(grid_for(A.n, kBlock / L)), dim3(kBlock), 0, s, A.n,
                                         A.ptr, A.col, (const T *)A.val, rhs, z, res, done));
}

template <typename T>
void launch_matvec(hipStream_t s, const DevCsrView &M, const T *x, T *y, const int *done)
{
    LPR_SWITCH(M.lpr, hipLaunchKernelGGL((k_matvec<T, L, false>), dim3(grid_for(M.n, kBlock / L)), dim3(kBlock), 0, s,
                                         M.n, M.ptr, M.col, (const T *)M.val, x, y, done));
}

template <typename T>
void launch_matvec_add(hipStream_t s, const DevCsrView &M, const T *e, T *x, const int *done)
{
    LPR_SWITCH(M.lpr, hipLaunchKernelGGL((k_matvec<T, L, true>), dim3(grid_for(M.n, kBlock / L)), dim3(kBlock), 0, s,
                                         M.n, M.ptr, M.col, (const T *)M.val, e, x, done));
}

template <typename T>
void launch_vpre(hipStream_t s, const DevCsrView &A, const T *dinv, const T *b, T *x, T *r, const int *done)
{
    LPR_SWITCH(A.lpr, hipLaunchKernelGGL((k_vpre<T, L>), dim3(grid_for(A.n, kBlock / L)), dim3(kBlock), 0, s, A.n,
                                         A.ptr, A.col, (const T *)A.val, dinv, b, x, r, done));
}

template <typename T>
void launch_dense_gemv(hipStream_t s, int n, const T *Ainv, const T *b, T *x, const int *done)
{
    hipLaunchKernelGGL(k_dense_gemv<T>, dim3(1), dim3(kBlock), 0, s, n, Ainv, b, x, done);
}

void launch_spmv64(hipStream_t s, const DevCsrView &A, const double *x, double *y, const Reduce &red, const int *done)
{
    if (red.out) {
        LPR_SWITCH(A.lpr, hipLaunchKernelGGL((k_spmv64<L, true>), dim3(grid_for(A.n, kBlock / L)), dim3(kBlock), 0, s,
                                             A.n, A.ptr, A.col, (const double *)A.val, x, y, red, done));
    } else {
        LPR_SWITCH(A.lpr, hipLaunchKernelGGL((k_spmv64<L, false>), dim3(grid_for(A.n, kBlock / L)), dim3(kBlock), 0,
                                             s, A.n, A.ptr, A.col, (const double *)A.val, x, y, red, done));
    }
}

void launch_residual64(hipStream_t s, const DevCsrView &A, const double *f, const double *u, double *r)
{
    LPR_SWITCH(A.lpr, hipLaunchKernelGGL((k_residual64<L>), dim3(grid_for(A.n, kBlock / L)), dim3(kBlock), 0, s, A.n,
                                         A.ptr, A.col, (const double *)A.val, f, u, r));
}

void launch_dot64(hipStream_t s, int n, const double *a, const double *b, const Reduce &red)
{
    hipLaunchKernelGGL(k_dot64, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, n, a, b, red);
}

void launch_cg_init(hipStream_t s, const CgState &st, double tol2, const double *ff, const double *rr0)
{
    hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(1), 0, s, st, tol2, ff, rr0);
}

void launch_cg_update(hipStream_t s, int n, double *x, double *r, const double *p, const double *q, const CgState &st,
                      const Reduce &red)
{
    hipLaunchKernelGGL(k_cg_update, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, n, x, r, p, q, st, red);
}

void launch_cg_direction(hipStream_t s, int n, const double *z, double *p, const CgState &st)
{
    hipLaunchKernelGGL(k_cg_direction, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, n, z, p, st);
}

void launch_cg_check_rz(hipStream_t s, const CgState &st)
{
    hipLaunchKernelGGL(k_cg_check_rz, dim3(1), dim3(1), 0, s, st);
}

void launch_cg_check_pq(hipStream_t s, const CgState &st)
{
    hipLaunchKernelGGL(k_cg_check_pq, dim3(1), dim3(1), 0, s, st);
}

void launch_kappa_grad(hipStream_t s, int nt, int nloc, const int *tet_dof, const double *G, const double *kappa,
                       const double *M, const double *u, const double *lam, double *g)
{
    hipLaunchKernelGGL(k_kappa_grad, dim3(grid_for(nt, kBlock)), dim3(kBlock), 0, s, nt, nloc, tet_dof, G, kappa, M,
                       u, lam, g);
}

void launch_cast(hipStream_t s, int64_t n, const double *x, float *y)
{
    int g = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, kMaxBlocks);
    hipLaunchKernelGGL(k_cast, dim3(g < 1 ? 1 : g), dim3(kBlock), 0, s, n, x, y);
}

#define INST(T)                                                                                              \
    template void launch_jacobi0<T>(hipStream_t, int, const T *, const double *, T *, T *, const int *);     \
    template void launch_first2<T>(hipStream_t, const DevCsrView &, const T *, const double *, T *, T *,     \
                                   const int *);                                                             \
    template void launch_resid<T>(hipStream_t, const DevCsrView &, const T *, const T *, T *, const int *);  \
    template void launch_matvec<T>(hipStream_t, const DevCsrView &, const T *, T *, const int *);            \
    template void launch_matvec_add<T>(hipStream_t, const DevCsrView &, const T *, T *, const int *);        \
    template void launch_vpre<T>(hipStream_t, const DevCsrView &, const T *, const T *, T *, T *, const int *); \
    template void launch_dense_gemv<T>(hipStream_t, int, const T *, const T *, T *, const int *);            \
    template void launch_sweep<T, T, T>(hipStream_t, const DevCsrView &, const T *, const T *, const T *, T *, \
                                        const double *, const Reduce &, const int *);

INST(double)
INST(float)
template void launch_sweep<float, double, double>(hipStream_t, const DevCsrView &, const float *, const double *,
                                                  const float *, double *, const double *, const Reduce &,
                                                  const int *);

}  // namespace auxp
