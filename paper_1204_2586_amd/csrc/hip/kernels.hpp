// Solve-phase kernels for gfx950 (CDNA4, wave64).  All sparse operators are
// CSR with int32 indices; each row is handled by LPR consecutive lanes of a
// wavefront (LPR in {1,2,4,8,16,32,64}) that stride over the row and combine
// with cross-lane shuffles.  Dot products are reduced deterministically: one
// partial per workgroup, and the last workgroup to finish sums the partials
// in a fixed order.  Kernels that belong to a CG iteration return at once when
// the device "done" flag is set, so iterations can be enqueued ahead of the
// convergence test.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace auxp {

constexpr int kBlock = 256;
constexpr int kMaxBlocks = 2048;

struct DevCsrView {
    int n;
    const int *ptr;
    const int *col;
    const void *val;     // double or float
    int lpr;
};

// Reduction target: partials[kMaxBlocks], an arrival counter, and the
// output slot.
struct Reduce {
    double *partials;
    unsigned int *counter;
    double *out;         // result slot base (null: no reduction)
    const int *index;    // if set, the result goes to out[*index] (the CG iteration)
};

// State of a CG solve in device memory.
struct CgState {
    int *iter;           // completed iterations
    int *done;           // 0 running, 1 converged, 2 maxit, 3 breakdown, 4 non-finite
    double *rz;          // rz[k] = r_k . z_k
    double *pq;          // pq[k] = p_k . A p_k
    double *rr;          // rr[k] = r_k . r_k
    double *tol2bb;      // tol^2 ||f||^2
    int maxit;
};

// ---- launchers (T = double or float is the preconditioner precision)

// z = D^{-1} r  (one sweep from zero); optionally writes rT = (T) r
template <typename T>
void launch_jacobi0(hipStream_t s, int n, const T *dinv, const double *r, T *z, T *rT, const int *done);

// z = D^{-1} r + D^{-1} (r - A D^{-1} r)   (two sweeps from zero); optionally rT = (T) r
template <typename T>
void launch_first2(hipStream_t s, const DevCsrView &A, const T *dinv, const double *r, T *z, T *rT,
                   const int *done);

// zout = zin + D^{-1} (rhs - A zin); RHS type TR, output type TZ.  With red.out,
// also reduces dot(rdot, zout) in double (rdot: double rhs of the dot).
template <typename T, typename TR, typename TZ>
void launch_sweep(hipStream_t s, const DevCsrView &A, const T *dinv, const TR *rhs, const T *zin, TZ *zout,
                  const double *rdot, const Reduce &red, const int *done);

// res = rhs - A z
template <typename T>
void launch_resid(hipStream_t s, const DevCsrView &A, const T *rhs, const T *z, T *res, const int *done);

// y = M x (rectangular CSR)
template <typename T>
void launch_matvec(hipStream_t s, const DevCsrView &M, const T *x, T *y, const int *done);

// x += M e
template <typename T>
void launch_matvec_add(hipStream_t s, const DevCsrView &M, const T *e, T *x, const int *done);

// V-cycle presmoothing from zero fused with the residual: x = D^{-1} b, r = b - A x
template <typename T>
void launch_vpre(hipStream_t s, const DevCsrView &A, const T *dinv, const T *b, T *x, T *r, const int *done);

// x = Ainv b for a dense row-major n x n inverse (one workgroup)
template <typename T>
void launch_dense_gemv(hipStream_t s, int n, const T *Ainv, const T *b, T *x, const int *done);

// ---- FP64 CG kernels

// y = A x; with red.out also dot(x, y)
void launch_spmv64(hipStream_t s, const DevCsrView &A, const double *x, double *y, const Reduce &red,
                   const int *done);
// r = f - A u, rr[0] = r.r, tol2bb = tol^2 f.f ; two reductions, host-ordered
void launch_dot64(hipStream_t s, int n, const double *a, const double *b, const Reduce &red);
// the CG "init" bookkeeping kernel (single thread)
void launch_cg_init(hipStream_t s, const CgState &st, double tol2, const double *ff, const double *rr0);
// x += alpha p ; r -= alpha q ; rr[k+1] = r.r ; convergence test ; iter++
void launch_cg_update(hipStream_t s, int n, double *x, double *r, const double *p, const double *q,
                      const CgState &st, const Reduce &red);
// p = z + beta p  (beta = rz[k]/rz[k-1]); with first = true, p = z
void launch_cg_direction(hipStream_t s, int n, const double *z, double *p, const CgState &st);
// check r.z > 0 after the preconditioner: sets done = 3/4 (single thread)
void launch_cg_check_rz(hipStream_t s, const CgState &st);
// check p.Ap > 0 (single thread)
void launch_cg_check_pq(hipStream_t s, const CgState &st);

// r = f - A u (FP64)
void launch_residual64(hipStream_t s, const DevCsrView &A, const double *f, const double *u, double *r);

// g_t = -lam_t^T K_t u_t for every tet (FP64): K_t = kappa_t sum_pq G_pq M^pq,
// G per tet [nt][16], M^pq tables [16][nloc][nloc], tet_dof [nt][nloc]
void launch_kappa_grad(hipStream_t s, int nt, int nloc, const int *tet_dof, const double *G,
                       const double *kappa, const double *M, const double *u, const double *lam, double *g);

void launch_cast(hipStream_t s, int64_t n, const double *x, float *y);

int pick_lpr(double avg_row_nnz);

}  // namespace auxp
