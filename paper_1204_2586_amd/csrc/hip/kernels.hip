// Solve-phase kernels of the auxiliary-space preconditioned CG (gfx950).
//
// All of this work is memory-bound sparse algebra: every kernel streams its
// operator once, gathers the vector it multiplies, and fuses the elementwise
// smoother / residual / CG updates into the same pass (one l1-Jacobi sweep is
// one pass over A).
#include <hip/hip_runtime.h>

#include <cmath>
#include <stdexcept>

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

// sum over the block (kBlock threads) in a fixed order; valid in thread 0
__device__ double block_sum(double v)
{
    __shared__ double red[kBlock / 64];
    v = group_sum<64>(v);
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBlock / 64; i++) s += red[i];
    return s;
}

__device__ __forceinline__ void write_partial(double *partials, double v)
{
    double b = block_sum(v);
    if (threadIdx.x == 0) partials[blockIdx.x] = b;
}

inline int grid_cap(long long need)
{
    if (need < 1) need = 1;
    if (need > kMaxBlocks) need = kMaxBlocks;
    return (int)need;
}

// ------------------------------------------------------------------ SELL

// One wavefront per 64-row slice (or two, see sell_rows), one lane per row;
// consecutive slices go to consecutive workgroups, which the dispatcher
// spreads round-robin over the dies, so at any moment all dies gather from
// the same neighbourhood of the vector and share it through the last-level
// cache (giving each die its own contiguous range of slices measured twice as
// slow, and no faster when the ranges are balanced by entries).

// MIXED = false: every slice has 32-bit columns, stored in entry order
// (wide[e]); MIXED = true: a 16-bit or 32-bit choice per slice.
template <typename T, bool MIXED, typename XF>
__device__ __forceinline__ T sell_row(const DevSellView &A, int slice, int lane, XF x)
{
    const T *__restrict__ val = (const T *)A.val;
    slice = __builtin_amdgcn_readfirstlane(slice);      // one slice per wavefront
    const int e0 = A.slice_off[slice], e1 = A.slice_off[slice + 1];
    T s = T(0);
    if (!MIXED) {
        const int *__restrict__ col = A.wide;
#pragma unroll 8
        for (int e = e0 + lane; e < e1; e += kSlice) s += val[e] * x(col[e]);
        return s;
    }
    const int mode = A.mode[slice];
    if (mode == 0) {
        // 16-bit offsets: the bases of 64 slots come in one vector load and
        // are broadcast from their lanes
        const int t0 = e0 / kSlice, width = (e1 - e0) / kSlice;
        for (int jc = 0; jc < width; jc += kSlice) {
            const int jn = min(kSlice, width - jc);
            const int bl = lane < jn ? A.base[t0 + jc + lane] : 0;
            const int eb = e0 + jc * kSlice + lane;
#pragma unroll 4
            for (int jj = 0; jj < jn; jj++) {
                const int e = eb + jj * kSlice;
                s += val[e] * x(__builtin_amdgcn_readlane(bl, jj) + (int)A.off[e]);
            }
        }
    } else {
        const int *__restrict__ w = A.wide + ~mode;
#pragma unroll 4
        for (int k = lane; k < e1 - e0; k += kSlice) s += val[e0 + k] * x(w[k]);
    }
    return s;
}


// Slots [half ? ceil(w/2) : 0, half ? w : ceil(w/2)) of a 32-bit slice of
// width w (the split form)
template <typename T, typename XF>
__device__ __forceinline__ T sell_row_half(const DevSellView &A, int slice, int lane, int half, XF x)
{
    const T *__restrict__ val = (const T *)A.val;
    const int *__restrict__ col = A.wide;
    slice = __builtin_amdgcn_readfirstlane(slice);
    const int e0 = A.slice_off[slice], e1 = A.slice_off[slice + 1];
    const int wh = ((e1 - e0) / kSlice + 1) / 2;
    const int b = half ? e0 + wh * kSlice : e0, end = half ? e1 : e0 + wh * kSlice;
    T s = T(0);
#pragma unroll 8
    for (int e = b + lane; e < end; e += kSlice) s += val[e] * x(col[e]);
    return s;
}

// Every row of A: s = (A x)_row, then epi(row, s).  F = 0: one wavefront per
// 32-bit slice; F = 1: the same with per-slice 16/32-bit columns; F = 2 (wide
// 32-bit slices): two wavefronts per slice, each summing half of its slots
// (shorter dependent chains, twice the wavefronts in flight); the second
// half's sums pass through LDS and are added to the first in a fixed order.
// In the split form every thread of the block runs the same number of steps,
// so the barriers are uniform.
template <typename T, int F, typename XF, typename EPI>
__device__ __forceinline__ void sell_rows(const DevSellView &A, XF x, EPI epi)
{
    const int lane = threadIdx.x & 63, w = (int)(threadIdx.x >> 6);
    if constexpr (F != 2) {
        for (int sl = blockIdx.x * (kBlock / 64) + w; sl < A.nslices; sl += gridDim.x * (kBlock / 64)) {
            const T s = sell_row<T, F == 1>(A, sl, lane, x);
            const int row = sl * kSlice + lane;
            if (row < A.n) epi(row, s);
        }
    } else {
        constexpr int kPairs = kBlock / 128;
        __shared__ T part[kPairs][64];
        const int q = w >> 1, h = w & 1;
        const int per_step = kPairs * (int)gridDim.x;
        const int steps = (A.nslices + per_step - 1) / per_step;
        for (int it = 0; it < steps; it++) {
            const int sl = (it * (int)gridDim.x + (int)blockIdx.x) * kPairs + q;
            T s = T(0);
            if (sl < A.nslices) s = sell_row_half<T>(A, sl, lane, h, x);
            if (h == 1) part[q][lane] = s;
            __syncthreads();
            if (h == 0 && sl < A.nslices) {
                s += part[q][lane];
                const int row = sl * kSlice + lane;
                if (row < A.n) epi(row, s);
            }
            __syncthreads();
        }
    }
}

#define FORM_SWITCH(A, CALL)                                \
    do {                                                    \
        if ((A).mixed) {                                    \
            constexpr int F = 1;                            \
            CALL;                                           \
        } else if ((A).split) {                             \
            constexpr int F = 2;                            \
            CALL;                                           \
        } else {                                            \
            constexpr int F = 0;                            \
            CALL;                                           \
        }                                                   \
    } while (0)

inline int sell_grid(const DevSellView &A)
{
    return A.split && !A.mixed ? grid_cap(((long long)A.nslices + 1) / 2) : grid_cap(((long long)A.nslices + 3) / 4);
}

template <typename T, typename TR, typename TZ, bool DOT, int F>
__global__ __launch_bounds__(kBlock) void k_sell_sweep(DevSellView A, const T *__restrict__ dinv,
                                                       const TR *__restrict__ rhs, const T *__restrict__ zin,
                                                       TZ *__restrict__ zout, const double *__restrict__ rdot,
                                                       double *partials, const int *done)
{
    if (stop(done)) return;
    double acc = 0.0;
    sell_rows<T, F>(A, [&](int j) { return zin[j]; }, [&](int row, T s) {
        T zi = zin[row] + dinv[row] * ((T)rhs[row] - s);
        zout[row] = (TZ)zi;
        if (DOT) acc += rdot[row] * (double)(TZ)zi;
    });
    if (DOT) write_partial(partials, acc);
}

template <typename T, int F>
__global__ __launch_bounds__(kBlock) void k_sell_resid(DevSellView A, const T *__restrict__ rhs,
                                                       const T *__restrict__ z, T *__restrict__ res, const int *done)
{
    if (stop(done)) return;
    sell_rows<T, F>(A, [&](int j) { return z[j]; }, [&](int row, T s) { res[row] = rhs[row] - s; });
}

template <bool DOT, int F>
__global__ __launch_bounds__(kBlock) void k_sell_spmv64(DevSellView A, const double *__restrict__ x,
                                                        double *__restrict__ y, double *partials, const int *done)
{
    if (stop(done)) return;
    double acc = 0.0;
    sell_rows<double, F>(A, [&](int j) { return x[j]; }, [&](int row, double s) {
        y[row] = s;
        if (DOT) acc += x[row] * s;
    });
    if (DOT) write_partial(partials, acc);
}

template <int F>
__global__ __launch_bounds__(kBlock) void k_sell_residual64(DevSellView A, const double *__restrict__ f,
                                                            const double *__restrict__ u, double *__restrict__ r)
{
    sell_rows<double, F>(A, [&](int j) { return u[j]; }, [&](int row, double s) { r[row] = f[row] - s; });
}

template <typename T, typename TR>
__global__ __launch_bounds__(kBlock) void k_jacobi0(int n, const T *__restrict__ dinv, const TR *__restrict__ r,
                                                    T *__restrict__ z, T *__restrict__ rT, const int *done)
{
    if (stop(done)) return;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        T ri = (T)r[i];
        z[i] = dinv[i] * ri;
        if (rT) rT[i] = ri;
    }
}

// ------------------------------------------------------------------- CSR

#define FOR_ROWS(LPR, n)                                                                                    \
    const int sub_ = threadIdx.x % (LPR);                                                                   \
    for (int base_ = blockIdx.x * (kBlock / (LPR)); base_ < (n); base_ += gridDim.x * (kBlock / (LPR)))     \
        for (int row = base_ + threadIdx.x / (LPR), once_ = 1; once_; once_ = 0)

template <int LPR, typename T, typename XF>
__device__ __forceinline__ T csr_row(const int *__restrict__ ptr, const int *__restrict__ col,
                                     const T *__restrict__ val, int row, int sub, XF x)
{
    T s = T(0);
    const int e1 = ptr[row + 1];
#pragma unroll 8
    for (int e = ptr[row] + sub; e < e1; e += LPR) s += val[e] * x(col[e]);
    return group_sum<LPR>(s);
}

template <typename T, int LPR, bool ADD>
__global__ __launch_bounds__(kBlock) void k_csr_matvec(int n, const int *__restrict__ ptr, const int *__restrict__ col,
                                                       const T *__restrict__ val, const T *__restrict__ x,
                                                       T *__restrict__ y, const int *done)
{
    if (stop(done)) return;
    FOR_ROWS(LPR, n)
    {
        if (row < n) {
            T s = csr_row<LPR>(ptr, col, val, row, sub_, [&](int j) { return x[j]; });
            if (sub_ == 0) y[row] = ADD ? y[row] + s : s;
        }
    }
}

// Row-split sliced ELL product, one wavefront per slice of 64 / L rows.
// MODE 0: y = M x1; 1: y += M x1; 2: y = M [x1; x2] (columns below split
// index x1).  Every slot is one coalesced load of 64 values and 64 columns;
// the slot count is uniform over the wavefront.
template <typename T, int L, int MODE>
__global__ __launch_bounds__(kBlock) void k_ell_matvec(int n, const int *__restrict__ off, const int *__restrict__ col,
                                                       const T *__restrict__ val, const T *__restrict__ x1,
                                                       const T *__restrict__ x2, int split, T *__restrict__ y,
                                                       const int *done)
{
    if (stop(done)) return;
    constexpr int C = 64 / L;
    const int lane = threadIdx.x % 64;
    const int nsl = (n + C - 1) / C;
    for (int sl = blockIdx.x * (kBlock / 64) + (int)(threadIdx.x / 64); sl < nsl; sl += gridDim.x * (kBlock / 64)) {
        const int e1 = off[sl + 1];
        T acc = T(0);
#pragma unroll 8
        for (int e = off[sl] + lane; e < e1; e += 64) {
            const int j = col[e];
            acc += val[e] * (MODE == 2 ? (j < split ? x1[j] : x2[j - split]) : x1[j]);
        }
        acc = group_sum<L>(acc);
        const int row = sl * C + lane / L;
        if (lane % L == 0 && row < n) {
            if (MODE == 1) y[row] += acc;
            else y[row] = acc;
        }
    }
}

// y = M [x1; x2]: columns below `split` index x1, the others x2
template <typename T, int LPR>
__global__ __launch_bounds__(kBlock) void k_csr_matvec2(int n, const int *__restrict__ ptr, const int *__restrict__ col,
                                                        const T *__restrict__ val, const T *__restrict__ x1,
                                                        const T *__restrict__ x2, int split, T *__restrict__ y,
                                                        const int *done)
{
    if (stop(done)) return;
    FOR_ROWS(LPR, n)
    {
        if (row < n) {
            T s = csr_row<LPR>(ptr, col, val, row, sub_, [&](int j) { return j < split ? x1[j] : x2[j - split]; });
            if (sub_ == 0) y[row] = s;
        }
    }
}

template <typename T, int LPR>
__global__ __launch_bounds__(kBlock) void k_csr_vpre(int n, const int *__restrict__ ptr, const int *__restrict__ col,
                                                     const T *__restrict__ val, const T *__restrict__ dinv,
                                                     const T *__restrict__ b, T *__restrict__ x, T *__restrict__ r,
                                                     const int *done)
{
    if (stop(done)) return;
    FOR_ROWS(LPR, n)
    {
        if (row < n) {
            T s = csr_row<LPR>(ptr, col, val, row, sub_, [&](int j) { return dinv[j] * b[j]; });
            if (sub_ == 0) {
                x[row] = dinv[row] * b[row];
                r[row] = b[row] - s;
            }
        }
    }
}

template <typename T, int LPR>
__global__ __launch_bounds__(kBlock) void k_csr_sweep(int n, const int *__restrict__ ptr, const int *__restrict__ col,
                                                      const T *__restrict__ val, const T *__restrict__ dinv,
                                                      const T *__restrict__ b, const T *__restrict__ x,
                                                      T *__restrict__ y, const int *done)
{
    if (stop(done)) return;
    FOR_ROWS(LPR, n)
    {
        if (row < n) {
            T s = csr_row<LPR>(ptr, col, val, row, sub_, [&](int j) { return x[j]; });
            if (sub_ == 0) y[row] = x[row] + dinv[row] * (b[row] - s);
        }
    }
}

// One workgroup per row: each lane's few loads of the row are all in flight
// at once (at most n / 256 per lane), then a workgroup sum; the rows of the
// dense cycle (at most 8192) are short enough that one wavefront per row
// leaves each lane a chain of dependent load rounds.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dense_gemv(int n, const T *__restrict__ Ainv, const T *__restrict__ b,
                                                       T *__restrict__ x, const int *done)
{
    if (stop(done)) return;
    __shared__ T red[kBlock / 64];
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const T *__restrict__ row = Ainv + (size_t)i * n;
        T s0 = T(0), s1 = T(0);
        int j = threadIdx.x;
        for (; j + kBlock < n; j += 2 * kBlock) {
            s0 += row[j] * b[j];
            s1 += row[j + kBlock] * b[j + kBlock];
        }
        if (j < n) s0 += row[j] * b[j];
        T s = group_sum<64>(s0 + s1);
        __syncthreads();                           // red of the previous row is consumed
        if (l == 0) red[w] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            T t = T(0);
            for (int q = 0; q < kBlock / 64; q++) t += red[q];
            x[i] = t;
        }
    }
}

// ------------------------------------------------------------------ CG

__global__ __launch_bounds__(kBlock) void k_dot(int n, const double *__restrict__ a, const double *__restrict__ b,
                                                double *partials)
{
    double acc = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) acc += a[i] * b[i];
    write_partial(partials, acc);
}

__global__ __launch_bounds__(kBlock) void k_finish(const double *__restrict__ partials, int nparts, int mode,
                                                   double *out, CgState st)
{
    if (mode != FIN_PLAIN && *st.done) return;
    // four accumulators, loads unrolled: all of a thread's partials in flight
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * kBlock < nparts; i += 4 * kBlock) {
        s0 += partials[i];
        s1 += partials[i + kBlock];
        s2 += partials[i + 2 * kBlock];
        s3 += partials[i + 3 * kBlock];
    }
    for (; i < nparts; i += kBlock) s0 += partials[i];
    double s = block_sum((s0 + s1) + (s2 + s3));
    if (threadIdx.x != 0) return;
    if (mode == FIN_PLAIN) {
        *out = s;
        return;
    }
    const int k = *st.iter;
    int d = 0;
    if (mode == FIN_RR) {
        st.rr[k + 1] = s;
        *st.iter = k + 1;
        if (!std::isfinite(s)) d = 4;
        else if (s <= st.scal[2]) d = 1;
        else if (k + 1 >= st.maxit) d = 2;
    } else {
        (mode == FIN_PQ ? st.pq : st.rz)[k] = s;
        if (!std::isfinite(s)) d = 4;
        else if (!(s > 0.0)) d = 3;
    }
    if (d) *st.done = d;
}

__global__ void k_cg_init(CgState st, double tol2)
{
    *st.iter = 0;
    double f2 = st.scal[0], r2 = st.scal[1];
    st.rr[0] = r2;
    st.scal[2] = tol2 * f2;
    int d = 0;
    if (!std::isfinite(f2) || !std::isfinite(r2)) d = 4;
    else if (r2 <= tol2 * f2) d = 1;     // includes f = 0 with u = 0
    else if (st.maxit <= 0) d = 2;
    *st.done = d;
}

__global__ __launch_bounds__(kBlock) void k_cg_update(int n, double *__restrict__ x, double *__restrict__ r,
                                                      const double *__restrict__ p, const double *__restrict__ q,
                                                      CgState st, double *partials)
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
    write_partial(partials, acc);
}

// the update fused with the preconditioner's first sweep from zero:
// z0 = D^-1 r in the preconditioner's type (and its copy of r), with the
// expressions of k_jacobi0
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_update_prep(int n, double *__restrict__ x, double *__restrict__ r,
                                                           const double *__restrict__ p, const double *__restrict__ q,
                                                           CgState st, double *partials, const T *__restrict__ dinv,
                                                           T *__restrict__ z0, T *__restrict__ rT)
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
        T rt = (T)ri;
        z0[i] = dinv[i] * rt;
        if (rT) rT[i] = rt;
    }
    write_partial(partials, acc);
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

__global__ __launch_bounds__(kBlock) void k_gather(int n, const int *__restrict__ idx, const double *__restrict__ x,
                                                   double *__restrict__ y)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) y[i] = x[idx[i]];
}

__global__ __launch_bounds__(kBlock) void k_scatter(int n, const int *__restrict__ idx, const double *__restrict__ x,
                                                    double *__restrict__ y)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) y[idx[i]] = x[i];
}

// ------------------------------------------------------------- adjoint

// One thread per tet; NLOC is a template argument so the element vectors
// stay in registers (the node loops unroll) and the reference tables, read at
// indices uniform over the wavefront, come through scalar loads.
template <int NLOC>
__global__ __launch_bounds__(kBlock) void k_kappa_grad(int nt, const int *__restrict__ tet_dof,
                                                       const double *__restrict__ G, const double *__restrict__ kappa,
                                                       const double *__restrict__ M, const double *__restrict__ u,
                                                       const double *__restrict__ lam, double *__restrict__ g)
{
    for (int t = blockIdx.x * kBlock + threadIdx.x; t < nt; t += gridDim.x * kBlock) {
        double ue[NLOC], le[NLOC];
#pragma unroll
        for (int a = 0; a < NLOC; a++) {
            const int i = tet_dof[(size_t)t * NLOC + a];
            ue[a] = i >= 0 ? u[i] : 0.0;
            le[a] = i >= 0 ? lam[i] : 0.0;
        }
        double s = 0.0;
#pragma unroll 1
        for (int pq = 0; pq < 16; pq++) {
            const double *Mpq = M + (size_t)pq * NLOC * NLOC;
            double w = 0.0;
#pragma unroll
            for (int a = 0; a < NLOC; a++) {
                double ra = 0.0;
#pragma unroll
                for (int b = 0; b < NLOC; b++) ra += Mpq[a * NLOC + b] * ue[b];
                w += le[a] * ra;
            }
            s += G[(size_t)t * 16 + pq] * w;
        }
        g[t] = -kappa[t] * s;
    }
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

#define LPR_SWITCH(lpr, CALL)                         \
    switch (lpr) {                                    \
    case 1: { constexpr int L = 1; CALL; } break;     \
    case 2: { constexpr int L = 2; CALL; } break;     \
    case 4: { constexpr int L = 4; CALL; } break;     \
    case 8: { constexpr int L = 8; CALL; } break;     \
    case 16: { constexpr int L = 16; CALL; } break;   \
    default: { constexpr int L = 32; CALL; } break;   \
    }

static int vec_grid(long long n) { return grid_cap((n + kBlock - 1) / kBlock); }
static int rows_grid(int n, int lpr) { return grid_cap(((long long)n * lpr + kBlock - 1) / kBlock); }

template <typename T>
int vec_jacobi0(hipStream_t s, int n, const T *dinv, const double *r, T *z, T *rT, const int *done)
{
    int g = vec_grid(n);
    hipLaunchKernelGGL((k_jacobi0<T, double>), dim3(g), dim3(kBlock), 0, s, n, dinv, r, z, rT, done);
    return g;
}

template <typename T>
void vec_jacobi0_t(hipStream_t s, int n, const T *dinv, const T *r, T *z, const int *done)
{
    hipLaunchKernelGGL((k_jacobi0<T, T>), dim3(vec_grid(n)), dim3(kBlock), 0, s, n, dinv, r, z, nullptr, done);
}

template <typename T, typename TR, typename TZ>
int sell_sweep(hipStream_t s, const DevSellView &A, const T *dinv, const TR *rhs, const T *zin, TZ *zout,
               const double *rdot, double *partials, const int *done)
{
    int g = sell_grid(A);
    FORM_SWITCH(A, if (partials) hipLaunchKernelGGL((k_sell_sweep<T, TR, TZ, true, F>), dim3(g), dim3(kBlock), 0, s, A,
                                                     dinv, rhs, zin, zout, rdot, partials, done);
                 else hipLaunchKernelGGL((k_sell_sweep<T, TR, TZ, false, F>), dim3(g), dim3(kBlock), 0, s, A, dinv,
                                         rhs, zin, zout, rdot, partials, done));
    return g;
}

template <typename T>
int sell_resid(hipStream_t s, const DevSellView &A, const T *rhs, const T *z, T *res, const int *done)
{
    int g = sell_grid(A);
    FORM_SWITCH(A, hipLaunchKernelGGL((k_sell_resid<T, F>), dim3(g), dim3(kBlock), 0, s, A, rhs, z, res, done));
    return g;
}

int sell_spmv64(hipStream_t s, const DevSellView &A, const double *x, double *y, double *partials, const int *done)
{
    int g = sell_grid(A);
    if (partials)
        FORM_SWITCH(A, hipLaunchKernelGGL((k_sell_spmv64<true, F>), dim3(g), dim3(kBlock), 0, s, A, x, y, partials,
                                           done));
    else
        FORM_SWITCH(A, hipLaunchKernelGGL((k_sell_spmv64<false, F>), dim3(g), dim3(kBlock), 0, s, A, x, y, partials,
                                           done));
    return g;
}

int sell_residual64(hipStream_t s, const DevSellView &A, const double *f, const double *u, double *r)
{
    int g = sell_grid(A);
    FORM_SWITCH(A, hipLaunchKernelGGL((k_sell_residual64<F>), dim3(g), dim3(kBlock), 0, s, A, f, u, r));
    return g;
}

static int ell_grid(int n, int lanes)
{
    const long long slices = ((long long)n * lanes + 63) / 64;
    return grid_cap((slices + kBlock / 64 - 1) / (kBlock / 64));
}

template <typename T, int MODE>
void ell_matvec(hipStream_t s, const DevCsrView &M, const T *x1, const T *x2, int split, T *y, const int *done)
{
    LPR_SWITCH(M.ell_lanes, hipLaunchKernelGGL((k_ell_matvec<T, L, MODE>), dim3(ell_grid(M.n, L)), dim3(kBlock), 0, s,
                                               M.n, M.ell_off, M.ell_col, (const T *)M.ell_val, x1, x2, split, y,
                                               done));
}

template <typename T>
void csr_matvec(hipStream_t s, const DevCsrView &M, const T *x, T *y, const int *done)
{
    if (M.ell_lanes > 0) return ell_matvec<T, 0>(s, M, x, nullptr, 0, y, done);
    LPR_SWITCH(M.lpr, hipLaunchKernelGGL((k_csr_matvec<T, L, false>), dim3(rows_grid(M.n, L)), dim3(kBlock), 0, s,
                                         M.n, M.ptr, M.col, (const T *)M.val, x, y, done));
}

template <typename T>
void csr_matvec_add(hipStream_t s, const DevCsrView &M, const T *e, T *x, const int *done)
{
    if (M.ell_lanes > 0) return ell_matvec<T, 1>(s, M, e, nullptr, 0, x, done);
    LPR_SWITCH(M.lpr, hipLaunchKernelGGL((k_csr_matvec<T, L, true>), dim3(rows_grid(M.n, L)), dim3(kBlock), 0, s,
                                         M.n, M.ptr, M.col, (const T *)M.val, e, x, done));
}

template <typename T>
void csr_matvec2(hipStream_t s, const DevCsrView &M, const T *x1, const T *x2, int split, T *y, const int *done)
{
    if (M.ell_lanes > 0) return ell_matvec<T, 2>(s, M, x1, x2, split, y, done);
    LPR_SWITCH(M.lpr, hipLaunchKernelGGL((k_csr_matvec2<T, L>), dim3(rows_grid(M.n, L)), dim3(kBlock), 0, s, M.n,
                                         M.ptr, M.col, (const T *)M.val, x1, x2, split, y, done));
}

template <typename T>
void csr_vpre(hipStream_t s, const DevCsrView &A, const T *dinv, const T *b, T *x, T *r, const int *done)
{
    LPR_SWITCH(A.lpr, hipLaunchKernelGGL((k_csr_vpre<T, L>), dim3(rows_grid(A.n, L)), dim3(kBlock), 0, s, A.n, A.ptr,
                                         A.col, (const T *)A.val, dinv, b, x, r, done));
}

template <typename T>
void csr_sweep(hipStream_t s, const DevCsrView &A, const T *dinv, const T *b, const T *x, T *y, const int *done)
{
    LPR_SWITCH(A.lpr, hipLaunchKernelGGL((k_csr_sweep<T, L>), dim3(rows_grid(A.n, L)), dim3(kBlock), 0, s, A.n,
                                         A.ptr, A.col, (const T *)A.val, dinv, b, x, y, done));
}

template <typename T>
void dense_gemv(hipStream_t s, int n, const T *Ainv, const T *b, T *x, const int *done)
{
    // one workgroup per row
    hipLaunchKernelGGL(k_dense_gemv<T>, dim3(grid_cap(n)), dim3(kBlock), 0, s, n, Ainv, b, x, done);
}

int vec_dot(hipStream_t s, int n, const double *a, const double *b, double *partials)
{
    int g = vec_grid(n);
    hipLaunchKernelGGL(k_dot, dim3(g), dim3(kBlock), 0, s, n, a, b, partials);
    return g;
}

void finish(hipStream_t s, const double *partials, int nparts, FinishMode mode, double *out, const CgState &st)
{
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kBlock), 0, s, partials, nparts, (int)mode, out, st);
}

void cg_init(hipStream_t s, const CgState &st, double tol2)
{
    hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(1), 0, s, st, tol2);
}

int cg_update(hipStream_t s, int n, double *x, double *r, const double *p, const double *q, const CgState &st,
              double *partials)
{
    int g = vec_grid(n);
    hipLaunchKernelGGL(k_cg_update, dim3(g), dim3(kBlock), 0, s, n, x, r, p, q, st, partials);
    return g;
}

template <typename T>
int cg_update_prep(hipStream_t s, int n, double *x, double *r, const double *p, const double *q, const CgState &st,
                   double *partials, const T *dinv, T *z0, T *rT)
{
    int g = vec_grid(n);
    hipLaunchKernelGGL(k_cg_update_prep<T>, dim3(g), dim3(kBlock), 0, s, n, x, r, p, q, st, partials, dinv, z0, rT);
    return g;
}
template int cg_update_prep<float>(hipStream_t, int, double *, double *, const double *, const double *,
                                   const CgState &, double *, const float *, float *, float *);
template int cg_update_prep<double>(hipStream_t, int, double *, double *, const double *, const double *,
                                    const CgState &, double *, const double *, double *, double *);

void cg_direction(hipStream_t s, int n, const double *z, double *p, const CgState &st)
{
    hipLaunchKernelGGL(k_cg_direction, dim3(vec_grid(n)), dim3(kBlock), 0, s, n, z, p, st);
}

void vec_gather(hipStream_t s, int n, const int *idx, const double *x, double *y)
{
    hipLaunchKernelGGL(k_gather, dim3(vec_grid(n)), dim3(kBlock), 0, s, n, idx, x, y);
}

void vec_scatter(hipStream_t s, int n, const int *idx, const double *x, double *y)
{
    hipLaunchKernelGGL(k_scatter, dim3(vec_grid(n)), dim3(kBlock), 0, s, n, idx, x, y);
}

void kappa_grad(hipStream_t s, int nt, int nloc, const int *tet_dof, const double *G, const double *kappa,
                const double *M, const double *u, const double *lam, double *g)
{
    switch (nloc) {
    case 10:
        hipLaunchKernelGGL(k_kappa_grad<10>, dim3(vec_grid(nt)), dim3(kBlock), 0, s, nt, tet_dof, G, kappa, M, u, lam, g);
        break;
    case 20:
        hipLaunchKernelGGL(k_kappa_grad<20>, dim3(vec_grid(nt)), dim3(kBlock), 0, s, nt, tet_dof, G, kappa, M, u, lam, g);
        break;
    case 35:
        hipLaunchKernelGGL(k_kappa_grad<35>, dim3(vec_grid(nt)), dim3(kBlock), 0, s, nt, tet_dof, G, kappa, M, u, lam, g);
        break;
    default:
        throw std::invalid_argument("kappa gradient: nodes per tet must be 10, 20 or 35");
    }
}

#define INST(T)                                                                                              \
    template int vec_jacobi0<T>(hipStream_t, int, const T *, const double *, T *, T *, const int *);         \
    template void vec_jacobi0_t<T>(hipStream_t, int, const T *, const T *, T *, const int *);               \
    template int sell_resid<T>(hipStream_t, const DevSellView &, const T *, const T *, T *, const int *);    \
    template int sell_sweep<T, T, T>(hipStream_t, const DevSellView &, const T *, const T *, const T *, T *, \
                                     const double *, double *, const int *);                                 \
    template void csr_matvec<T>(hipStream_t, const DevCsrView &, const T *, T *, const int *);               \
    template void csr_matvec_add<T>(hipStream_t, const DevCsrView &, const T *, T *, const int *);           \
    template void csr_matvec2<T>(hipStream_t, const DevCsrView &, const T *, const T *, int, T *, const int *); \
    template void csr_vpre<T>(hipStream_t, const DevCsrView &, const T *, const T *, T *, T *, const int *); \
    template void csr_sweep<T>(hipStream_t, const DevCsrView &, const T *, const T *, const T *, T *,        \
                               const int *);                                                                 \
    template void dense_gemv<T>(hipStream_t, int, const T *, const T *, T *, const int *);

INST(double)
INST(float)
template int sell_sweep<float, double, double>(hipStream_t, const DevSellView &, const float *, const double *,
                                               const float *, double *, const double *, double *, const int *);

}  // namespace auxp
