// Solve-phase kernels for gfx950 (CDNA4, wave64).
//
// The P^k operator A_h is stored as sliced ELLPACK with 64-row slices
// (one wavefront per slice, one lane per row, entries of a slice stored
// column-major so every load of a wavefront is 64 consecutive words).  Its
// rows are numbered in an internal order, sorted by length so the padding of
// each slice stays small: either over the whole operator (a stable sort,
// which on structured meshes groups nodes of one kind and keeps a slice's
// gathers nearly contiguous) or within windows of consecutive dofs; the setup
// times both on the device and keeps the faster (the global sort wins on the
// benchmark meshes).  The AMG operators and the transfers are CSR with LPR
// lanes per row or row-split sliced ELL, whichever the setup times faster.
//
// Dot products are reduced deterministically without atomics: every
// workgroup writes one partial, and a one-workgroup "finish" kernel that
// follows in the stream sums them in a fixed order.  Kernels that belong to a
// CG iteration return at once when the device "done" flag is set, so
// iterations can be enqueued ahead of the convergence test.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace auxp {

constexpr int kBlock = 256;
constexpr int kMaxBlocks = 4096;       // partial sums per reduction at most
constexpr int kSlice = 64;             // rows per ELL slice (one wavefront)

struct DevCsrView {
    int n;
    const int *ptr;
    const int *col;
    const void *val;     // double or float
    int lpr;
    // Row-split sliced ELL copy of the same operator (ell_lanes > 0: the
    // products use it): slices of 64 / ell_lanes rows, one wavefront each,
    // entry k of the slice's row q in slot k / ell_lanes at lane
    // q * ell_lanes + k % ell_lanes; ell_off[s] is the first entry of slice s
    // (a multiple of 64), padding entries have column 0 and value 0.
    int ell_lanes;
    const int *ell_off;
    const int *ell_col;
    const void *ell_val;
};

struct DevSellView {
    int n;               // rows
    int nslices;
    int max_width;       // longest slice, in slots of 64 entries
    int mixed;           // 0: every slice 32-bit with wide[e] the column of entry e
    const int *slice_off;  // [nslices+1] first entry of each slice (multiple of 64)
    // Columns.  mode[s] == 0: entry e of slot t = e / 64 has column
    // base[t] + off[e]; mode[s] = ~w < 0: column wide[w + e - slice_off[s]].
    const int *mode;
    const int *base;
    const unsigned short *off;
    const int *wide;
    const void *val;     // double or float, padding entries are 0
    int split;           // with mixed == 0: two wavefronts per slice (wide slices)
    // block kernels only: when set, die d (the workgroups b with b % 8 == d,
    // which the dispatcher places on die d) takes slices [die_off[d],
    // die_off[d + 1]) (9 entries); otherwise slices go round-robin
    const int *die_off = nullptr;
};

// State of a CG solve in device memory.
struct CgState {
    int *iter;           // completed iterations
    int *done;           // 0 running, 1 converged, 2 maxit, 3 breakdown, 4 non-finite
    double *rz;          // rz[k] = r_k . z_k
    double *pq;          // pq[k] = p_k . A p_k
    double *rr;          // rr[k] = r_k . r_k
    double *scal;        // [0] f.f, [1] r_0.r_0, [2] tol^2 f.f
    int maxit;
};

enum FinishMode { FIN_PLAIN = 0, FIN_PQ = 1, FIN_RZ = 2, FIN_RR = 3 };

// ---- P^k level (SELL).  Kernels that reduce write one partial per
// workgroup to `partials` (if non-null) and return the grid size used.

// z = D^{-1} r (one sweep from zero); rT = (T) r if rT
template <typename T>
int vec_jacobi0(hipStream_t s, int n, const T *dinv, const double *r, T *z, T *rT, const int *done);
// z = D^{-1} r for r in the working precision
template <typename T>
void vec_jacobi0_t(hipStream_t s, int n, const T *dinv, const T *r, T *z, const int *done);
// zout = zin + D^{-1} (rhs - A zin); with partials, also sum_i rdot_i zout_i
template <typename T, typename TR, typename TZ>
int sell_sweep(hipStream_t s, const DevSellView &A, const T *dinv, const TR *rhs, const T *zin, TZ *zout,
               const double *rdot, double *partials, const int *done);
// res = rhs - A z
template <typename T>
int sell_resid(hipStream_t s, const DevSellView &A, const T *rhs, const T *z, T *res, const int *done);
// y = A x (FP64); with partials also x.y
int sell_spmv64(hipStream_t s, const DevSellView &A, const double *x, double *y, double *partials, const int *done);
// r = f - A u (FP64)
int sell_residual64(hipStream_t s, const DevSellView &A, const double *f, const double *u, double *r);

// ---- CSR (AMG levels, transfers)
template <typename T>
void csr_matvec(hipStream_t s, const DevCsrView &M, const T *x, T *y, const int *done);
template <typename T>
void csr_matvec_add(hipStream_t s, const DevCsrView &M, const T *e, T *x, const int *done);
// z += M e for M with at most w (1..4) entries per row in w column-major
// slots (slot k of row i at k n + i, padding value 0 at column 0)
template <typename T>
void fixed_matvec_add(hipStream_t s, int n, int w, const int *col, const T *val, const T *e, T *z, const int *done);
// y = M [x1; x2] (columns below split index x1, the rest x2)
template <typename T>
void csr_matvec2(hipStream_t s, const DevCsrView &M, const T *x1, const T *x2, int split, T *y, const int *done);

// x = D^{-1} b, r = b - A x (V-cycle presmoothing from zero fused with the residual)
template <typename T>
void csr_vpre(hipStream_t s, const DevCsrView &A, const T *dinv, const T *b, T *x, T *r, const int *done);
// y = x + D^{-1} (b - A x)
template <typename T>
void csr_sweep(hipStream_t s, const DevCsrView &A, const T *dinv, const T *b, const T *x, T *y, const int *done);
// x = Ainv b, dense row-major n x n (one workgroup)
template <typename T>
void dense_gemv(hipStream_t s, int n, const T *Ainv, const T *b, T *x, const int *done);

// ---- vectors and CG bookkeeping (FP64)
int vec_dot(hipStream_t s, int n, const double *a, const double *b, double *partials);
// sum nparts partials; FIN_PLAIN writes out[0]; the others write the CG slot of
// the current iteration and update the state (see kernels.hip)
void finish(hipStream_t s, const double *partials, int nparts, FinishMode mode, double *out, const CgState &st);
void cg_init(hipStream_t s, const CgState &st, double tol2);
// x += alpha p ; r -= alpha q ; partial r.r
int cg_update(hipStream_t s, int n, double *x, double *r, const double *p, const double *q, const CgState &st,
              double *partials);
// the same, also writing the preconditioner's first sweep from zero,
// z0 = D^-1 r, and (rT non-null) r in the preconditioner's type
template <typename T>
int cg_update_prep(hipStream_t s, int n, double *x, double *r, const double *p, const double *q, const CgState &st,
                   double *partials, const T *dinv, T *z0, T *rT);
// p = z + beta p, beta = rz[k]/rz[k-1] (p = z at k = 0)
void cg_direction(hipStream_t s, int n, const double *z, double *p, const CgState &st);
// y[i] = x[idx[i]]
void vec_gather(hipStream_t s, int n, const int *idx, const double *x, double *y);
// y[idx[i]] = x[i]
void vec_scatter(hipStream_t s, int n, const int *idx, const double *x, double *y);

// g_t = -kappa_t sum_pq G_pq lam_t^T M^pq u_t per tet (FP64); tet_dof holds
// internal dof numbers (-1 on the boundary)
void kappa_grad(hipStream_t s, int nt, int nloc, const int *tet_dof, const double *G, const double *kappa,
                const double *M, const double *u, const double *lam, double *g);

int pick_lpr(double avg_row_nnz);

}  // namespace auxp
