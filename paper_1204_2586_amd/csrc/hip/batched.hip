// Batched solve phase: NR right-hand sides in lock-step.
//
// Block vectors are row-major [n][NR] (NR in {8, 16, 32, 64}); a row of a
// sparse operator is handled by NR consecutive lanes, one per right-hand
// side, so each matrix entry is read once per row and applied to all
// columns (sparse matrix times dense block).  The gathered rows of the block
// are NR contiguous words.  Every column follows the single right-hand-side
// CG exactly: its own alpha, beta and stopping test; converged columns are
// frozen while the others continue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "batched.hpp"

namespace auxp {

namespace {

__device__ __forceinline__ bool stop_all(const int *all_done) { return all_done != nullptr && *all_done != 0; }

inline int grid_cap(long long need)
{
    if (need < 1) need = 1;
    if (need > kMaxBlocks) need = kMaxBlocks;
    return (int)need;
}

// rows handled by a block: kBlock / NR
#define FOR_BROWS(NR, nrows)                                                                                 \
    const int c_ = threadIdx.x % (NR);                                                                       \
    for (int row = blockIdx.x * (kBlock / (NR)) + (int)threadIdx.x / (NR); row < (nrows);                    \
         row += gridDim.x * (kBlock / (NR)))

inline int brows_grid(int n, int NR) { return grid_cap(((long long)n * NR + kBlock - 1) / kBlock); }

// per-column partial sums of a block of BS threads: partials[blockIdx.x * NR + c]
template <int NR, int BS = kBlock>
__device__ void write_col_partials(double *partials, double v)
{
    __shared__ double red[BS];
    red[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x < NR) {
        double s = 0.0;
        for (int i = threadIdx.x; i < BS; i += NR) s += red[i];
        partials[(size_t)blockIdx.x * NR + threadIdx.x] = s;
    }
}

// ------------------------------------------------------------------ SELL

// One block per 64-row slice.  The slice's values and decoded columns are
// staged in LDS in chunks of kChunk slots (coalesced, once per block), then
// every (row, column) pair of the slice is accumulated by the lane that owns
// it: kBlock / NR rows per pass, kSlice / (kBlock / NR) passes.  Blocks never
// share a slice, so no two XCDs fetch the same matrix lines.
constexpr int kChunk = 32;

// Element idx of a block vector addressed by a 32-bit byte offset from the
// (uniform) base: the load takes the scalar-base form, one address register
// per gather instead of two.  The caller guarantees blocks below 4 GiB.
template <typename T>
__device__ __forceinline__ T gather32(const T *__restrict__ base, unsigned idx)
{
    return *(const T *)((const char *)base + idx * (unsigned)sizeof(T));
}


// U: slots unrolled in the accumulation (more gathers in flight per lane;
// 4 for A_h and for level operators with long rows or few slices, 1 for the
// large prolongations)
template <typename T, int NR, int U, typename XL, typename BODY>
__device__ __forceinline__ void bsell_slices(const DevSellView &A, XL xload, BODY body)
{
    constexpr int RP = kBlock / NR, NP = kSlice / RP;
    __shared__ T vs[kChunk * kSlice];
    __shared__ int cs[kChunk * kSlice];
    const T *__restrict__ val = (const T *)A.val;
    const int c = threadIdx.x % NR, rl0 = threadIdx.x / NR;
    // Slices go round-robin over the workgroups (and so over the dies), or,
    // with die ranges (A_h in the spatially ordered batched layout), die d =
    // b % 8 walks its own contiguous range so its gathers stay in one region
    // (for operators in the length-sorted single-vector order, contiguous die
    // shares measured slower: the sweeps by 9%, I_P by 38%)
    int sl = blockIdx.x, sl_end = A.nslices, sl_step = gridDim.x;
    if (A.die_off) {
        const int d = blockIdx.x % 8;
        sl = A.die_off[d] + (int)blockIdx.x / 8;
        sl_end = A.die_off[d + 1];
        sl_step = ((int)gridDim.x - d + 7) / 8;
    }
    for (; sl < sl_end; sl += sl_step) {
        const int e0 = A.slice_off[sl], width = (A.slice_off[sl + 1] - e0) / kSlice;
        const int mode = A.mode[sl];
        T acc[NP];
#pragma unroll
        for (int p = 0; p < NP; p++) acc[p] = T(0);
        for (int j0 = 0; j0 < width; j0 += kChunk) {
            const int jn = min(kChunk, width - j0);
            const int cnt = jn * kSlice, eb = e0 + j0 * kSlice;
            // every load of the chunk is issued before any is waited on
            // (indices clamped into the chunk, stores predicated)
            constexpr int PER = kChunk * kSlice / kBlock;
            T vt[PER];
            int ct[PER];
            if (mode == 0) {
#pragma unroll
                for (int i = 0; i < PER; i++) {
                    const int e = eb + min(threadIdx.x + i * kBlock, cnt - 1);
                    vt[i] = val[e];
                    ct[i] = A.base[e / kSlice] + (int)A.off[e];
                }
            } else {
                const int *__restrict__ w = A.wide + (~mode) + (eb - e0);
#pragma unroll
                for (int i = 0; i < PER; i++) {
                    const int k = min(threadIdx.x + i * kBlock, cnt - 1);
                    vt[i] = val[eb + k];
                    ct[i] = w[k];
                }
            }
            __syncthreads();                           // the previous chunk is consumed
#pragma unroll
            for (int i = 0; i < PER; i++) {
                const int k = threadIdx.x + i * kBlock;
                if (k < cnt) {
                    vs[k] = vt[i];
                    cs[k] = ct[i];
                }
            }
            __syncthreads();
            // the NP rows of a lane are independent: their gathers (for U
            // slots) are in flight together
#pragma unroll U
            for (int jj = 0; jj < jn; jj++) {
                T xv[NP], vv[NP];
#pragma unroll
                for (int p = 0; p < NP; p++) {
                    const int k = jj * kSlice + p * RP + rl0;
                    vv[p] = vs[k];
                    xv[p] = xload(cs[k], c);
                }
#pragma unroll
                for (int p = 0; p < NP; p++) acc[p] += vv[p] * xv[p];
            }
        }
#pragma unroll
        for (int p = 0; p < NP; p++) {
            const int row = sl * kSlice + p * RP + rl0;
            if (row < A.n) body(row, c, acc[p]);
        }
    }
}

// with die ranges every die needs a workgroup: at least 8
inline int bsell_grid(const DevSellView &A) { return A.die_off ? std::max(8, grid_cap(A.nslices)) : grid_cap(A.nslices); }

template <typename T, int NR>
__global__ __launch_bounds__(kBlock) void kb_jacobi0(int n, const T *__restrict__ dinv, const double *__restrict__ R,
                                                     T *__restrict__ Z, T *__restrict__ RT, const int *all_done)
{
    if (stop_all(all_done)) return;
    FOR_BROWS(NR, n)
    {
        size_t o = (size_t)row * NR + c_;
        T ri = (T)R[o];
        Z[o] = dinv[row] * ri;
        if (RT) RT[o] = ri;
    }
}

template <typename T, typename TR, typename TZ, int NR, bool DOT>
__global__ __launch_bounds__(kBlock) void kb_sweep(DevSellView A, const T *__restrict__ dinv,
                                                   const TR *__restrict__ RHS, const T *__restrict__ Zin,
                                                   TZ *__restrict__ Zout, const double *__restrict__ Rdot,
                                                   double *partials, const int *all_done)
{
    if (stop_all(all_done)) return;
    double acc = 0.0;
    bsell_slices<T, NR, 4>(A, [&](int j, int c) { return gather32(Zin, (unsigned)j * NR + c); }, [&](int row, int c, T s) {
        size_t o = (size_t)row * NR + c;
        T zi = Zin[o] + dinv[row] * ((T)RHS[o] - s);
        Zout[o] = (TZ)zi;
        if (DOT) acc += Rdot[o] * (double)(TZ)zi;
    });
    if (DOT) write_col_partials<NR>(partials, acc);
}

template <typename T, int NR>
__global__ __launch_bounds__(kBlock) void kb_resid(DevSellView A, const T *__restrict__ RHS, const T *__restrict__ Z,
                                                   T *__restrict__ Res, const int *all_done)
{
    if (stop_all(all_done)) return;
    bsell_slices<T, NR, 4>(A, [&](int j, int c) { return gather32(Z, (unsigned)j * NR + c); }, [&](int row, int c, T s) {
        size_t o = (size_t)row * NR + c;
        Res[o] = RHS[o] - s;
    });
}

template <int NR, bool DOT, bool RESID>
__global__ __launch_bounds__(kBlock) void kb_spmv64(DevSellView A, const double *__restrict__ X,
                                                    double *__restrict__ Y, const double *__restrict__ F,
                                                    double *partials, const int *all_done)
{
    if (stop_all(all_done)) return;
    double acc = 0.0;
    bsell_slices<double, NR, 4>(A, [&](int j, int c) { return gather32(X, (unsigned)j * NR + c); }, [&](int row, int c, double s) {
        size_t o = (size_t)row * NR + c;
        if (RESID) {
            Y[o] = F[o] - s;
        } else {
            Y[o] = s;
            if (DOT) acc += X[o] * s;
        }
    });
    if (DOT) write_col_partials<NR>(partials, acc);
}

// ------------------------------------------------------------------ tiles
// One workgroup per tile of consecutive (original-order) rows: the tile's
// distinct gathered block rows (NR words each), its values, column
// positions and row offsets are staged in LDS with coalesced loads, then
// each group of NR lanes accumulates its rows from LDS.  A gathered block
// row crosses L2 once per tile instead of once per entry (5x fewer for P2,
// 8x for P3 at 64-row tiles).

constexpr int kTileBlock = 512;

template <typename T>
__host__ __device__ inline size_t tile_lds_bytes(int max_cols, int max_entries, int tile, int nr)
{
    size_t b = (size_t)max_cols * nr * sizeof(T) + (size_t)max_entries * sizeof(T);
    b += (size_t)(tile + 1) * sizeof(int) + (size_t)max_cols * sizeof(int);
    b += (size_t)max_entries * sizeof(unsigned short);
    return (b + 15) & ~(size_t)15;
}

// Staging happens in two steps so that no load waits on another global
// load: the tile's column list, values, positions and row offsets first
// (coalesced), then the gathered block rows, whose addresses now come from
// LDS, unrolled so that many rows are in flight per thread.
template <typename T, int NR, typename XT, typename BODY>
__device__ __forceinline__ void btile_rows(const DevTilesView &A, const XT *__restrict__ X, BODY body)
{
    constexpr int BS = kTileBlock, RG = BS / NR;   // row groups of NR lanes
    extern __shared__ __align__(16) unsigned char lds_[];
    T *Xs = (T *)lds_;
    T *Vs = Xs + (size_t)A.max_cols * NR;
    int *Rp = (int *)(Vs + A.max_entries);
    int *Us = Rp + A.tile + 1;
    unsigned short *Ls = (unsigned short *)(Us + A.max_cols);
    const T *__restrict__ val = (const T *)A.val;
    const int c = threadIdx.x % NR, g = threadIdx.x / NR;
    for (int t = blockIdx.x; t < A.ntiles; t += gridDim.x) {
        const int c0 = A.col_off[t], nc = A.col_off[t + 1] - c0;
        const int e0 = A.row_ptr[(size_t)t * A.tile], ne = A.row_ptr[(size_t)(t + 1) * A.tile] - e0;
        __syncthreads();                               // the previous tile is consumed
        for (int k = threadIdx.x; k < nc; k += BS) Us[k] = A.ucols[c0 + k];
        for (int k = threadIdx.x; k < ne; k += BS) {
            Vs[k] = val[e0 + k];
            Ls[k] = A.lidx[e0 + k];
        }
        for (int k = threadIdx.x; k <= A.tile; k += BS) Rp[k] = A.row_ptr[(size_t)t * A.tile + k] - e0;
        __syncthreads();
#pragma unroll 8
        for (int u = g; u < nc; u += RG) Xs[u * NR + c] = (T)X[(size_t)Us[u] * NR + c];
        __syncthreads();
        for (int i = g; i < A.tile; i += RG) {
            const int row = A.rows[(size_t)t * A.tile + i];
            if (row < 0) continue;
            T s = T(0);
            const int k1 = Rp[i + 1];
#pragma unroll 4
            for (int k = Rp[i]; k < k1; k++) s += Vs[k] * Xs[(int)Ls[k] * NR + c];
            body(row, c, s);
        }
    }
}

template <typename T, typename TR, typename TZ, int NR, bool DOT>
__global__ __launch_bounds__(kTileBlock) void kt_sweep(DevTilesView A, const T *__restrict__ dinv,
                                                       const TR *__restrict__ RHS, const T *__restrict__ Zin,
                                                       TZ *__restrict__ Zout, const double *__restrict__ Rdot,
                                                       double *partials, const int *all_done)
{
    if (stop_all(all_done)) return;
    double acc = 0.0;
    btile_rows<T, NR>(A, Zin, [&](int row, int c, T s) {
        size_t o = (size_t)row * NR + c;
        T zi = Zin[o] + dinv[row] * ((T)RHS[o] - s);
        Zout[o] = (TZ)zi;
        if (DOT) acc += Rdot[o] * (double)(TZ)zi;
    });
    if (DOT) write_col_partials<NR, kTileBlock>(partials, acc);
}

template <typename T, int NR>
__global__ __launch_bounds__(kTileBlock) void kt_resid(DevTilesView A, const T *__restrict__ RHS,
                                                       const T *__restrict__ Z, T *__restrict__ Res,
                                                       const int *all_done)
{
    if (stop_all(all_done)) return;
    btile_rows<T, NR>(A, Z, [&](int row, int c, T s) {
        size_t o = (size_t)row * NR + c;
        Res[o] = RHS[o] - s;
    });
}

template <int NR, bool DOT, bool RESID>
__global__ __launch_bounds__(kTileBlock) void kt_spmv64(DevTilesView A, const double *__restrict__ X,
                                                        double *__restrict__ Y, const double *__restrict__ F,
                                                        double *partials, const int *all_done)
{
    if (stop_all(all_done)) return;
    double acc = 0.0;
    btile_rows<double, NR>(A, X, [&](int row, int c, double s) {
        size_t o = (size_t)row * NR + c;
        if (RESID) {
            Y[o] = F[o] - s;
        } else {
            Y[o] = s;
            if (DOT) acc += X[o] * s;
        }
    });
    if (DOT) write_col_partials<NR, kTileBlock>(partials, acc);
}

// ------------------------------------------------------- AMG levels, transfers
// Row-permuted sliced ELL: internal row r of M is row perm[r] of the
// operator; columns are not renumbered.

template <typename T, int NR, int MODE, int U>   // MODE 0: Y = M X, 1: Y += M X
__global__ __launch_bounds__(kBlock) void kb_lmatvec(DevSellView M, const int *__restrict__ perm,
                                                     const T *__restrict__ X, T *__restrict__ Y, const int *all_done)
{
    if (stop_all(all_done)) return;
    bsell_slices<T, NR, U>(M, [&](int j, int c) { return gather32(X, (unsigned)j * NR + c); }, [&](int r, int c, T s) {
        size_t o = (size_t)perm[r] * NR + c;
        if (MODE) Y[o] += s;
        else Y[o] = s;
    });
}

// Y = M [X1; X2] (columns below split index X1, the others X2)
template <typename T, int NR, int U>
__global__ __launch_bounds__(kBlock) void kb_lmatvec2(DevSellView M, const int *__restrict__ perm,
                                                      const T *__restrict__ X1, const T *__restrict__ X2, int split,
                                                      T *__restrict__ Y, const int *all_done)
{
    if (stop_all(all_done)) return;
    bsell_slices<T, NR, U>(
        M, [&](int j, int c) { return j < split ? gather32(X1, (unsigned)j * NR + c) : gather32(X2, (unsigned)(j - split) * NR + c); },
        [&](int r, int c, T s) { Y[(size_t)perm[r] * NR + c] = s; });
}

// X = D^-1 B, R = B - A X, with AD the values of A D^-1: the product
// gathers B alone (one load per slot keeps the unrolled gathers in flight)
template <typename T, int NR, int U>
__global__ __launch_bounds__(kBlock) void kb_lvpre(DevSellView AD, const int *__restrict__ perm,
                                                   const T *__restrict__ dinv, const T *__restrict__ B,
                                                   T *__restrict__ X, T *__restrict__ R, const int *all_done)
{
    if (stop_all(all_done)) return;
    bsell_slices<T, NR, U>(AD, [&](int j, int c) { return gather32(B, (unsigned)j * NR + c); }, [&](int r, int c, T s) {
        const int i = perm[r];
        size_t o = (size_t)i * NR + c;
        T b = B[o];
        X[o] = dinv[i] * b;
        R[o] = b - s;
    });
}

// Y = X + D^-1 (B - A X)
template <typename T, int NR, int U>
__global__ __launch_bounds__(kBlock) void kb_lsweep(DevSellView A, const int *__restrict__ perm,
                                                    const T *__restrict__ dinv, const T *__restrict__ B,
                                                    const T *__restrict__ X, T *__restrict__ Y, const int *all_done)
{
    if (stop_all(all_done)) return;
    bsell_slices<T, NR, U>(A, [&](int j, int c) { return gather32(X, (unsigned)j * NR + c); }, [&](int r, int c, T s) {
        const int i = perm[r];
        size_t o = (size_t)i * NR + c;
        Y[o] = X[o] + dinv[i] * (B[o] - s);
    });
}

// X = M B for a dense row-major n x n matrix M (the coarsest inverse or the
// dense sub-cycle).  A workgroup takes kDenseRows rows; its KG = kBlock / NR
// lane groups split the inner index j (group g takes j = g, g + KG, ...), so
// each lane keeps kDenseRows independent chains of n / KG terms, and the
// groups' partial sums are added in LDS in a fixed order.
constexpr int kDenseRows = 4;

template <typename T, int NR>
__global__ __launch_bounds__(kBlock) void kb_dense(int n, const T *__restrict__ M, const T *__restrict__ B,
                                                   T *__restrict__ X, const int *all_done)
{
    if (stop_all(all_done)) return;
    constexpr int KG = kBlock / NR;
    __shared__ T red[KG][kDenseRows][NR];
    const int c = threadIdx.x % NR, g = threadIdx.x / NR;
    for (int r0 = blockIdx.x * kDenseRows; r0 < n; r0 += gridDim.x * kDenseRows) {
        T acc[kDenseRows];
#pragma unroll
        for (int r = 0; r < kDenseRows; r++) acc[r] = T(0);
        const T *m[kDenseRows];
#pragma unroll
        for (int r = 0; r < kDenseRows; r++) m[r] = M + (size_t)min(r0 + r, n - 1) * n;   // clamped rows unused
#pragma unroll 4
        for (int j = g; j < n; j += KG) {
            const T b = B[(size_t)j * NR + c];
#pragma unroll
            for (int r = 0; r < kDenseRows; r++) acc[r] += m[r][j] * b;
        }
#pragma unroll
        for (int r = 0; r < kDenseRows; r++) red[g][r][c] = acc[r];
        __syncthreads();
        if (threadIdx.x < kDenseRows * NR) {
            const int r = threadIdx.x / NR, cc = threadIdx.x % NR;
            T s = T(0);
            for (int k = 0; k < KG; k++) s += red[k][r][cc];
            if (r0 + r < n) X[(size_t)(r0 + r) * NR + cc] = s;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------- CG

template <int NR>
__global__ __launch_bounds__(kBlock) void kb_dot(int n, const double *__restrict__ a, const double *__restrict__ b,
                                                 double *partials)
{
    double acc = 0.0;
    FOR_BROWS(NR, n)
    {
        size_t o = (size_t)row * NR + c_;
        acc += a[o] * b[o];
    }
    write_col_partials<NR>(partials, acc);
}

// sum the per-column partials and update the per-column CG state
constexpr int kFinishBlock = 1024;

template <int NR>
__global__ __launch_bounds__(kFinishBlock) void kb_finish(const double *__restrict__ partials, int nparts, int mode,
                                                          double *out, BCgState st)
{
    if (mode != FIN_PLAIN && *st.all_done) return;
    __shared__ double red[kFinishBlock];
    constexpr int G = kFinishBlock / NR;           // partial rows summed side by side
    const int c = threadIdx.x % NR, g = threadIdx.x / NR;
    // four independent accumulators keep several loads in flight
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int b = g;
    for (; b + 3 * G < nparts; b += 4 * G) {
        s0 += partials[(size_t)b * NR + c];
        s1 += partials[(size_t)(b + G) * NR + c];
        s2 += partials[(size_t)(b + 2 * G) * NR + c];
        s3 += partials[(size_t)(b + 3 * G) * NR + c];
    }
    for (; b < nparts; b += G) s0 += partials[(size_t)b * NR + c];
    red[threadIdx.x] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    __shared__ int active_left;
    if (threadIdx.x == 0) active_left = 0;
    __syncthreads();
    if (threadIdx.x < NR) {
        double t = 0.0;
        for (int i = threadIdx.x; i < kFinishBlock; i += NR) t += red[i];
        const int k = *st.k;
        if (mode == FIN_PLAIN) {
            out[c] = t;
        } else if (st.done[c] == 0) {
            int d = 0;
            if (mode == FIN_RR) {
                st.rr[(size_t)(k + 1) * NR + c] = t;
                st.iter[c] = k + 1;
                if (!std::isfinite(t)) d = 4;
                else if (t <= st.tol2ff[c]) d = 1;
                else if (k + 1 >= st.maxit) d = 2;
            } else {
                (mode == FIN_PQ ? st.pq : st.rz)[(size_t)k * NR + c] = t;
                if (!std::isfinite(t)) d = 4;
                else if (!(t > 0.0)) d = 3;
            }
            if (d) st.done[c] = d;
            else atomicAdd(&active_left, 1);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && mode != FIN_PLAIN) {
        if (mode == FIN_RR) *st.k += 1;
        if (active_left == 0) *st.all_done = 1;
    }
}

template <int NR>
__global__ void kb_cg_init(BCgState st, double tol2, const double *ff, const double *rr0)
{
    const int c = threadIdx.x;
    if (c >= NR) return;
    double f2 = ff[c], r2 = rr0[c];
    st.rr[c] = r2;
    st.tol2ff[c] = tol2 * f2;
    st.iter[c] = 0;
    int d = 0;
    if (!std::isfinite(f2) || !std::isfinite(r2)) d = 4;
    else if (r2 <= tol2 * f2) d = 1;
    else if (st.maxit <= 0) d = 2;
    st.done[c] = d;
    __shared__ int any;
    if (c == 0) any = 0;
    __syncthreads();
    if (d == 0) atomicAdd(&any, 1);
    __syncthreads();
    if (c == 0) {
        *st.k = 0;
        *st.all_done = any == 0;
    }
}

template <int NR>
__global__ __launch_bounds__(kBlock) void kb_cg_update(int n, double *__restrict__ X, double *__restrict__ R,
                                                       const double *__restrict__ P, const double *__restrict__ Q,
                                                       BCgState st, double *partials)
{
    if (*st.all_done) return;
    const int k = *st.k;
    const int c = threadIdx.x % NR;
    const bool active = st.done[c] == 0;
    const double alpha = active ? st.rz[(size_t)k * NR + c] / st.pq[(size_t)k * NR + c] : 0.0;
    double acc = 0.0;
    FOR_BROWS(NR, n)
    {
        size_t o = (size_t)row * NR + c_;
        double ri = R[o];
        if (active) {
            X[o] += alpha * P[o];
            ri -= alpha * Q[o];
            R[o] = ri;
        }
        acc += ri * ri;
    }
    write_col_partials<NR>(partials, acc);
}

// the update fused with the preconditioner's first sweep from zero (the
// expressions of kb_jacobi0): Z0 = D^-1 R and RT = R in the type T
template <typename T, int NR>
__global__ __launch_bounds__(kBlock) void kb_cg_update_prep(int n, double *__restrict__ X, double *__restrict__ R,
                                                            const double *__restrict__ P,
                                                            const double *__restrict__ Q, BCgState st,
                                                            double *partials, const T *__restrict__ dinv,
                                                            T *__restrict__ Z0, T *__restrict__ RT)
{
    if (*st.all_done) return;
    const int k = *st.k;
    const int c = threadIdx.x % NR;
    const bool active = st.done[c] == 0;
    const double alpha = active ? st.rz[(size_t)k * NR + c] / st.pq[(size_t)k * NR + c] : 0.0;
    double acc = 0.0;
    FOR_BROWS(NR, n)
    {
        size_t o = (size_t)row * NR + c_;
        double ri = R[o];
        if (active) {
            X[o] += alpha * P[o];
            ri -= alpha * Q[o];
            R[o] = ri;
        }
        acc += ri * ri;
        T rt = (T)ri;
        Z0[o] = dinv[row] * rt;
        if (RT) RT[o] = rt;
    }
    write_col_partials<NR>(partials, acc);
}

template <int NR, typename TZ>
__global__ __launch_bounds__(kBlock) void kb_cg_direction(int n, const TZ *__restrict__ Z, double *__restrict__ P,
                                                          BCgState st)
{
    if (*st.all_done) return;
    const int k = *st.k;
    const int c = threadIdx.x % NR;
    if (st.done[c] != 0) return;
    const double beta = k == 0 ? 0.0 : st.rz[(size_t)k * NR + c] / st.rz[(size_t)(k - 1) * NR + c];
    FOR_BROWS(NR, n)
    {
        size_t o = (size_t)row * NR + c_;
        const double z = Z[o];
        P[o] = k == 0 ? z : z + beta * P[o];
    }
}

// internal block row i = external row perm[i]; external leading dimension ld
template <int NR>
__global__ __launch_bounds__(kBlock) void kb_gather(int n, int ld, const int *__restrict__ perm,
                                                    const double *__restrict__ x, double *__restrict__ y)
{
    FOR_BROWS(NR, n)
    {
        y[(size_t)row * NR + c_] = c_ < ld ? x[(size_t)perm[row] * ld + c_] : 0.0;
    }
}

template <int NR>
__global__ __launch_bounds__(kBlock) void kb_scatter(int n, int ld, const int *__restrict__ perm,
                                                     const double *__restrict__ x, double *__restrict__ y)
{
    FOR_BROWS(NR, n)
    {
        if (c_ < ld) y[(size_t)perm[row] * ld + c_] = x[(size_t)row * NR + c_];
    }
}

}  // namespace

#define NR_SWITCH(nr, CALL)                            \
    switch (nr) {                                      \
    case 8: { constexpr int NR = 8; CALL; } break;     \
    case 16: { constexpr int NR = 16; CALL; } break;   \
    case 32: { constexpr int NR = 32; CALL; } break;   \
    default: { constexpr int NR = 64; CALL; } break;   \
    }

constexpr size_t kTileLdsMax = 40 * 1024;   // leaves room for several workgroups per CU

size_t btile_lds(const DevTilesView &A, int nr, int s)
{
    size_t b = s == 8 ? tile_lds_bytes<double>(A.max_cols, A.max_entries, A.tile, nr)
                      : tile_lds_bytes<float>(A.max_cols, A.max_entries, A.tile, nr);
    return b <= kTileLdsMax ? b : 0;
}

inline int btile_grid(const DevTilesView &A) { return grid_cap(A.ntiles); }

template <typename T, typename TR, typename TZ>
int btile_sweep(hipStream_t s, int nr, const DevTilesView &A, const T *dinv, const TR *RHS, const T *Zin, TZ *Zout,
                const double *Rdot, double *partials, const int *all_done)
{
    const int g = btile_grid(A);
    const size_t lds = btile_lds(A, nr, sizeof(T));
    if (partials) {
        NR_SWITCH(nr, hipLaunchKernelGGL((kt_sweep<T, TR, TZ, NR, true>), dim3(g), dim3(kTileBlock), lds, s, A, dinv, RHS,
                                         Zin, Zout, Rdot, partials, all_done));
    } else {
        NR_SWITCH(nr, hipLaunchKernelGGL((kt_sweep<T, TR, TZ, NR, false>), dim3(g), dim3(kTileBlock), lds, s, A, dinv,
                                         RHS, Zin, Zout, Rdot, partials, all_done));
    }
    return g;
}

template <typename T>
int btile_resid(hipStream_t s, int nr, const DevTilesView &A, const T *RHS, const T *Z, T *Res, const int *all_done)
{
    const int g = btile_grid(A);
    const size_t lds = btile_lds(A, nr, sizeof(T));
    NR_SWITCH(nr, hipLaunchKernelGGL((kt_resid<T, NR>), dim3(g), dim3(kTileBlock), lds, s, A, RHS, Z, Res, all_done));
    return g;
}

int btile_spmv64(hipStream_t s, int nr, const DevTilesView &A, const double *X, double *Y, double *partials,
                 const int *all_done)
{
    const int g = btile_grid(A);
    const size_t lds = btile_lds(A, nr, 8);
    if (partials) {
        NR_SWITCH(nr, hipLaunchKernelGGL((kt_spmv64<NR, true, false>), dim3(g), dim3(kTileBlock), lds, s, A, X, Y,
                                         (const double *)nullptr, partials, all_done));
    } else {
        NR_SWITCH(nr, hipLaunchKernelGGL((kt_spmv64<NR, false, false>), dim3(g), dim3(kTileBlock), lds, s, A, X, Y,
                                         (const double *)nullptr, partials, all_done));
    }
    return g;
}

int btile_residual64(hipStream_t s, int nr, const DevTilesView &A, const double *F, const double *U, double *R)
{
    const int g = btile_grid(A);
    const size_t lds = btile_lds(A, nr, 8);
    NR_SWITCH(nr, hipLaunchKernelGGL((kt_spmv64<NR, false, true>), dim3(g), dim3(kTileBlock), lds, s, A, U, R, F,
                                     (double *)nullptr, (const int *)nullptr));
    return g;
}

template <typename T>
void bjacobi0(hipStream_t s, int nr, int n, const T *dinv, const double *R, T *Z, T *RT, const int *all_done)
{
    int g = brows_grid(n, nr);
    NR_SWITCH(nr, hipLaunchKernelGGL((kb_jacobi0<T, NR>), dim3(g), dim3(kBlock), 0, s, n, dinv, R, Z, RT, all_done));
}

template <typename T, typename TR, typename TZ>
int bsell_sweep(hipStream_t s, int nr, const DevSellView &A, const T *dinv, const TR *RHS, const T *Zin, TZ *Zout,
                const double *Rdot, double *partials, const int *all_done)
{
    int g = bsell_grid(A);
    if (partials) {
        NR_SWITCH(nr, hipLaunchKernelGGL((kb_sweep<T, TR, TZ, NR, true>), dim3(g), dim3(kBlock), 0, s, A, dinv, RHS,
                                         Zin, Zout, Rdot, partials, all_done));
    } else {
        NR_SWITCH(nr, hipLaunchKernelGGL((kb_sweep<T, TR, TZ, NR, false>), dim3(g), dim3(kBlock), 0, s, A, dinv, RHS,
                                         Zin, Zout, Rdot, partials, all_done));
    }
    return g;
}

template <typename T>
int bsell_resid(hipStream_t s, int nr, const DevSellView &A, const T *RHS, const T *Z, T *Res, const int *all_done)
{
    int g = bsell_grid(A);
    NR_SWITCH(nr, hipLaunchKernelGGL((kb_resid<T, NR>), dim3(g), dim3(kBlock), 0, s, A, RHS, Z, Res, all_done));
    return g;
}

int bsell_spmv64(hipStream_t s, int nr, const DevSellView &A, const double *X, double *Y, double *partials,
                 const int *all_done)
{
    int g = bsell_grid(A);
    if (partials) {
        NR_SWITCH(nr, hipLaunchKernelGGL((kb_spmv64<NR, true, false>), dim3(g), dim3(kBlock), 0, s, A, X, Y,
                                         (const double *)nullptr, partials, all_done));
    } else {
        NR_SWITCH(nr, hipLaunchKernelGGL((kb_spmv64<NR, false, false>), dim3(g), dim3(kBlock), 0, s, A, X, Y,
                                         (const double *)nullptr, partials, all_done));
    }
    return g;
}

int bsell_residual64(hipStream_t s, int nr, const DevSellView &A, const double *F, const double *U, double *R)
{
    int g = bsell_grid(A);
    NR_SWITCH(nr, hipLaunchKernelGGL((kb_spmv64<NR, false, true>), dim3(g), dim3(kBlock), 0, s, A, U, R, F,
                                     (double *)nullptr, (const int *)nullptr));
    return g;
}

// unroll: slots per lane whose gathers are in flight together (1 or 4).
// Four pays off on operators with long rows (the level matrices, the
// restrictions); on the short rows of the prolongations the extra registers
// cost more occupancy than the overlap gains.
#define U_SWITCH(unroll, CALL)             \
    do {                                   \
        if ((unroll) >= 4) {               \
            constexpr int U = 4;           \
            CALL;                          \
        } else {                           \
            constexpr int U = 1;           \
            CALL;                          \
        }                                  \
    } while (0)

template <typename T>
void blevel_matvec(hipStream_t s, int nr, const DevSellView &M, int unroll, const int *perm, const T *X, T *Y,
                   bool add, const int *all_done)
{
    int g = bsell_grid(M);
    if (add) {
        U_SWITCH(unroll, NR_SWITCH(nr, hipLaunchKernelGGL((kb_lmatvec<T, NR, 1, U>), dim3(g), dim3(kBlock), 0, s, M, perm,
                                                     X, Y, all_done)));
    } else {
        U_SWITCH(unroll, NR_SWITCH(nr, hipLaunchKernelGGL((kb_lmatvec<T, NR, 0, U>), dim3(g), dim3(kBlock), 0, s, M, perm,
                                                     X, Y, all_done)));
    }
}

template <typename T>
void blevel_matvec2(hipStream_t s, int nr, const DevSellView &M, int unroll, const int *perm, const T *X1, const T *X2, int split,
                    T *Y, const int *all_done)
{
    int g = bsell_grid(M);
    U_SWITCH(unroll, NR_SWITCH(nr, hipLaunchKernelGGL((kb_lmatvec2<T, NR, U>), dim3(g), dim3(kBlock), 0, s, M, perm, X1,
                                                 X2, split, Y, all_done)));
}

template <typename T>
void blevel_vpre(hipStream_t s, int nr, const DevSellView &AD, int unroll, const int *perm, const T *dinv, const T *B, T *X, T *R,
                 const int *all_done)
{
    int g = bsell_grid(AD);
    U_SWITCH(unroll, NR_SWITCH(nr, hipLaunchKernelGGL((kb_lvpre<T, NR, U>), dim3(g), dim3(kBlock), 0, s, AD, perm, dinv,
                                                 B, X, R, all_done)));
}

template <typename T>
void blevel_sweep(hipStream_t s, int nr, const DevSellView &A, int unroll, const int *perm, const T *dinv, const T *B, const T *X,
                  T *Y, const int *all_done)
{
    int g = bsell_grid(A);
    U_SWITCH(unroll, NR_SWITCH(nr, hipLaunchKernelGGL((kb_lsweep<T, NR, U>), dim3(g), dim3(kBlock), 0, s, A, perm, dinv,
                                                 B, X, Y, all_done)));
}




template <typename T>
void bdense(hipStream_t s, int nr, int n, const T *Ainv, const T *B, T *X, const int *all_done)
{
    int g = grid_cap((n + kDenseRows - 1) / kDenseRows);
    NR_SWITCH(nr, hipLaunchKernelGGL((kb_dense<T, NR>), dim3(g), dim3(kBlock), 0, s, n, Ainv, B, X, all_done));
}

int bvec_dot(hipStream_t s, int nr, int n, const double *a, const double *b, double *partials)
{
    int g = brows_grid(n, nr);
    NR_SWITCH(nr, hipLaunchKernelGGL((kb_dot<NR>), dim3(g), dim3(kBlock), 0, s, n, a, b, partials));
    return g;
}

void bfinish(hipStream_t s, int nr, const double *partials, int nparts, FinishMode mode, double *out,
             const BCgState &st)
{
    NR_SWITCH(nr, hipLaunchKernelGGL((kb_finish<NR>), dim3(1), dim3(kFinishBlock), 0, s, partials, nparts, (int)mode,
                                     out, st));
}

void bcg_init(hipStream_t s, int nr, const BCgState &st, double tol2, const double *ff, const double *rr0)
{
    NR_SWITCH(nr, hipLaunchKernelGGL((kb_cg_init<NR>), dim3(1), dim3(64), 0, s, st, tol2, ff, rr0));
}

int bcg_update(hipStream_t s, int nr, int n, double *X, double *R, const double *P, const double *Q,
               const BCgState &st, double *partials)
{
    int g = brows_grid(n, nr);
    NR_SWITCH(nr, hipLaunchKernelGGL((kb_cg_update<NR>), dim3(g), dim3(kBlock), 0, s, n, X, R, P, Q, st, partials));
    return g;
}

template <typename T>
int bcg_update_prep(hipStream_t s, int nr, int n, double *X, double *R, const double *P, const double *Q,
                    const BCgState &st, double *partials, const T *dinv, T *Z0, T *RT)
{
    int g = brows_grid(n, nr);
    NR_SWITCH(nr, hipLaunchKernelGGL((kb_cg_update_prep<T, NR>), dim3(g), dim3(kBlock), 0, s, n, X, R, P, Q, st,
                                     partials, dinv, Z0, RT));
    return g;
}
template int bcg_update_prep<float>(hipStream_t, int, int, double *, double *, const double *, const double *,
                                    const BCgState &, double *, const float *, float *, float *);
template int bcg_update_prep<double>(hipStream_t, int, int, double *, double *, const double *, const double *,
                                     const BCgState &, double *, const double *, double *, double *);

template <typename TZ>
void bcg_direction(hipStream_t s, int nr, int n, const TZ *Z, double *P, const BCgState &st)
{
    int g = brows_grid(n, nr);
    NR_SWITCH(nr, hipLaunchKernelGGL((kb_cg_direction<NR, TZ>), dim3(g), dim3(kBlock), 0, s, n, Z, P, st));
}

void bgather(hipStream_t s, int nr, int n, int ld, const int *perm, const double *x, double *y)
{
    int g = brows_grid(n, nr);
    NR_SWITCH(nr, hipLaunchKernelGGL((kb_gather<NR>), dim3(g), dim3(kBlock), 0, s, n, ld, perm, x, y));
}

void bscatter(hipStream_t s, int nr, int n, int ld, const int *perm, const double *x, double *y)
{
    int g = brows_grid(n, nr);
    NR_SWITCH(nr, hipLaunchKernelGGL((kb_scatter<NR>), dim3(g), dim3(kBlock), 0, s, n, ld, perm, x, y));
}

#define BINST(T)                                                                                                   \
    template int btile_sweep<T, T, T>(hipStream_t, int, const DevTilesView &, const T *, const T *, const T *, T *, \
                                      const double *, double *, const int *);                                      \
    template int btile_resid<T>(hipStream_t, int, const DevTilesView &, const T *, const T *, T *, const int *);    \
    template void bjacobi0<T>(hipStream_t, int, int, const T *, const double *, T *, T *, const int *);            \
    template int bsell_sweep<T, T, T>(hipStream_t, int, const DevSellView &, const T *, const T *, const T *, T *, \
                                      const double *, double *, const int *);                                      \
    template int bsell_resid<T>(hipStream_t, int, const DevSellView &, const T *, const T *, T *, const int *);    \
    template void blevel_matvec<T>(hipStream_t, int, const DevSellView &, int, const int *, const T *, T *, bool,      \
                                   const int *);                                                                   \
    template void blevel_matvec2<T>(hipStream_t, int, const DevSellView &, int, const int *, const T *, const T *, int, \
                                    T *, const int *);                                                             \
    template void blevel_vpre<T>(hipStream_t, int, const DevSellView &, int, const int *, const T *, const T *, T *,     \
                                 T *, const int *);                                                                \
    template void blevel_sweep<T>(hipStream_t, int, const DevSellView &, int, const int *, const T *, const T *,         \
                                  const T *, T *, const int *);                                                    \
    template void bdense<T>(hipStream_t, int, int, const T *, const T *, T *, const int *);

BINST(double)
BINST(float)
template void bcg_direction<double>(hipStream_t, int, int, const double *, double *, const BCgState &);
template void bcg_direction<float>(hipStream_t, int, int, const float *, double *, const BCgState &);
template int bsell_sweep<float, double, float>(hipStream_t, int, const DevSellView &, const float *, const double *,
                                               const float *, float *, const double *, double *, const int *);
template int btile_sweep<float, double, float>(hipStream_t, int, const DevTilesView &, const float *, const double *,
                                               const float *, float *, const double *, double *, const int *);

}  // namespace auxp
