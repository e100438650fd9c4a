// Batched (multi right-hand side) solve-phase kernels; see batched.hip.
#pragma once

#include "kernels.hpp"

namespace auxp {

// Per-column CG state of a lock-step batched solve (NR columns).
struct BCgState {
    int *k;              // lock-step iteration index
    int *iter;           // [NR] iterations performed by each column
    int *done;           // [NR] 0 running, 1 converged, 2 maxit, 3 breakdown, 4 non-finite
    int *all_done;       // 1 when no column is running
    double *rz, *pq, *rr;  // [(maxit+2)][NR]
    double *tol2ff;      // [NR] tol^2 f_c . f_c
    int maxit;
};

// Row tiles of the P^k operator for block products (see Tiles in the host
// setup): per tile the distinct gathered block rows are staged in LDS.
struct DevTilesView {
    int n, tile, ntiles, max_cols, max_entries;
    const int *rows, *row_ptr, *col_off, *ucols;
    const unsigned short *lidx;
    const void *val;     // double or float
};
// LDS bytes a tile kernel needs for nr columns of type size s (0 if the
// tiles cannot be used: more than 64 KiB)
size_t btile_lds(const DevTilesView &A, int nr, int s);

template <typename T, typename TR, typename TZ>
int btile_sweep(hipStream_t s, int nr, const DevTilesView &A, const T *dinv, const TR *RHS, const T *Zin, TZ *Zout,
                const double *Rdot, double *partials, const int *all_done);
template <typename T>
int btile_resid(hipStream_t s, int nr, const DevTilesView &A, const T *RHS, const T *Z, T *Res, const int *all_done);
int btile_spmv64(hipStream_t s, int nr, const DevTilesView &A, const double *X, double *Y, double *partials,
                 const int *all_done);
int btile_residual64(hipStream_t s, int nr, const DevTilesView &A, const double *F, const double *U, double *R);

template <typename T>
void bjacobi0(hipStream_t s, int nr, int n, const T *dinv, const double *R, T *Z, T *RT, const int *all_done);
template <typename T, typename TR, typename TZ>
int bsell_sweep(hipStream_t s, int nr, const DevSellView &A, const T *dinv, const TR *RHS, const T *Zin, TZ *Zout,
                const double *Rdot, double *partials, const int *all_done);
template <typename T>
int bsell_resid(hipStream_t s, int nr, const DevSellView &A, const T *RHS, const T *Z, T *Res, const int *all_done);
int bsell_spmv64(hipStream_t s, int nr, const DevSellView &A, const double *X, double *Y, double *partials,
                 const int *all_done);
int bsell_residual64(hipStream_t s, int nr, const DevSellView &A, const double *F, const double *U, double *R);

// AMG levels and transfers as row-permuted sliced ELL (row r of M is row
// perm[r] of the operator, columns not renumbered)
template <typename T>
void blevel_matvec(hipStream_t s, int nr, const DevSellView &M, int unroll, const int *perm, const T *X, T *Y, bool add,
                   const int *all_done);
// Y = M [X1; X2] (columns below split index X1, the others X2)
template <typename T>
void blevel_matvec2(hipStream_t s, int nr, const DevSellView &M, int unroll, const int *perm, const T *X1, const T *X2, int split,
                    T *Y, const int *all_done);
// X = D^-1 B, R = B - (A D^-1) B; AD holds the values of A D^-1
template <typename T>
void blevel_vpre(hipStream_t s, int nr, const DevSellView &AD, int unroll, const int *perm, const T *dinv, const T *B, T *X, T *R,
                 const int *all_done);
// Y = X + D^-1 (B - A X)
template <typename T>
void blevel_sweep(hipStream_t s, int nr, const DevSellView &A, int unroll, const int *perm, const T *dinv, const T *B, const T *X,
                  T *Y, const int *all_done);
// X = M B, M dense row-major n x n (coarsest inverse or dense sub-cycle)
template <typename T>
void bdense(hipStream_t s, int nr, int n, const T *Ainv, const T *B, T *X, const int *all_done);

int bvec_dot(hipStream_t s, int nr, int n, const double *a, const double *b, double *partials);
void bfinish(hipStream_t s, int nr, const double *partials, int nparts, FinishMode mode, double *out,
             const BCgState &st);
void bcg_init(hipStream_t s, int nr, const BCgState &st, double tol2, const double *ff, const double *rr0);
int bcg_update(hipStream_t s, int nr, int n, double *X, double *R, const double *P, const double *Q,
               const BCgState &st, double *partials);
// the same, also writing the preconditioner's first sweep from zero
// (Z0 = D^-1 R) and, with RT non-null, R in the preconditioner's type
template <typename T>
int bcg_update_prep(hipStream_t s, int nr, int n, double *X, double *R, const double *P, const double *Q,
                    const BCgState &st, double *partials, const T *dinv, T *Z0, T *RT);
// Z: the preconditioned block, FP64 or (mixed mode, whose last sweep rounds
// it to FP32 anyway) FP32
template <typename TZ>
void bcg_direction(hipStream_t s, int nr, int n, const TZ *Z, double *P, const BCgState &st);
void bgather(hipStream_t s, int nr, int n, int ld, const int *perm, const double *x, double *y);
void bscatter(hipStream_t s, int nr, int n, int ld, const int *perm, const double *x, double *y);

}  // namespace auxp
