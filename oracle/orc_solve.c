/*
 * Test infrastructure (CPU oracle): the GAMG preconditioner and CG.
 *
 * The preconditioner B is the two-level method of Algorithm 2.1 made
 * symmetric with a presmoothing step (Remark 2.1): smooth on the P^k system,
 * restrict the residual with I_R, solve the P^1 problem approximately by one
 * AMG V-cycle (Remark 2.1 allows "an AMG method or a few AMG cycles" for Step
 * 1), prolong with I_P (Step 2) and postsmooth (Step 3).  The smoother G_h,
 * which the paper leaves open, is l1-Jacobi: G_h = D_l1^{-1} with
 * D_l1 = diag(sum_j |a_ij|).  The outer iteration is preconditioned CG, or
 * flexible GMRES(m), the method of the paper's experiments (Sec. 6.1).
 *
 * The "fp32" mode runs B in single precision: every stored operand of B is
 * rounded to float once, the input residual is rounded to float, and every
 * arithmetic result inside B is rounded to float (double rounding of a float
 * sum or product through double is exact).  CG itself stays in double.
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double (*rfun)(double);
static double r64(double x) { return x; }
static double r32(double x) { return (double)(float)x; }

/* operands of B, either the double originals or float-rounded copies */
typedef struct {
    const double *Aval, *dinv;
    const double *IPval, *IRval;
    const double *lAval[ORC_MAX_LEVELS], *ldinv[ORC_MAX_LEVELS];
    const double *lPval[ORC_MAX_LEVELS], *lRval[ORC_MAX_LEVELS];
    const double *chol;
    double *own[4 * ORC_MAX_LEVELS + 8];
    int nown;
    rfun R;
} bops;

static const double *keep(bops *b, const double *src, size_t n, rfun R, int inv)
{
    double *d = malloc((n ? n : 1) * sizeof(double));
    for (size_t i = 0; i < n; i++) d[i] = R(inv ? 1.0 / src[i] : src[i]);
    b->own[b->nown++] = d;
    return d;
}

static void bops_init(const orc *o, int fp32, bops *b)
{
    memset(b, 0, sizeof(*b));
    rfun R = fp32 ? r32 : r64;
    b->R = R;
    b->Aval = keep(b, o->A.val, (size_t)o->A.ptr[o->A.n], R, 0);
    b->dinv = keep(b, o->dl1, (size_t)o->ndof, R, 1);
    if (o->omega != 1.0) {
        double *d = (double *)b->dinv;
        for (int i = 0; i < o->ndof; i++) d[i] = R(o->omega / o->dl1[i]);
    }
    b->IPval = keep(b, o->IP.val, (size_t)o->IP.ptr[o->IP.n], R, 0);
    b->IRval = keep(b, o->IR.val, (size_t)o->IR.ptr[o->IR.n], R, 0);
    for (int l = 0; l < o->nlev; l++) {
        const olevel *lv = &o->lev[l];
        b->lAval[l] = keep(b, lv->A.val, (size_t)lv->A.ptr[lv->A.n], R, 0);
        b->ldinv[l] = keep(b, lv->dl1, (size_t)lv->A.n, R, 1);
        if (l + 1 < o->nlev) {
            b->lPval[l] = keep(b, lv->P.val, (size_t)lv->P.ptr[lv->P.n], R, 0);
            b->lRval[l] = keep(b, lv->R.val, (size_t)lv->R.ptr[lv->R.n], R, 0);
        }
    }
    b->chol = keep(b, o->chol, (size_t)o->ncoarse * o->ncoarse, R, 0);
}

static void bops_free(bops *b)
{
    for (int i = 0; i < b->nown; i++) free(b->own[i]);
}

/* xout = xin + D^{-1} (rhs - A xin)   (one l1-Jacobi sweep) */
static void sweep(const ocsr *A, const double *av, const double *dinv, const double *rhs,
                  const double *xin, double *xout, rfun R)
{
    for (int i = 0; i < A->n; i++) {
        double s = 0.0;
        for (int e = A->ptr[i]; e < A->ptr[i + 1]; e++) s = R(s + R(av[e] * xin[A->col[e]]));
        xout[i] = R(xin[i] + R(dinv[i] * R(rhs[i] - s)));
    }
}

/* res = rhs - A x */
static void residual(const ocsr *A, const double *av, const double *rhs, const double *x,
                     double *res, rfun R)
{
    for (int i = 0; i < A->n; i++) {
        double s = 0.0;
        for (int e = A->ptr[i]; e < A->ptr[i + 1]; e++) s = R(s + R(av[e] * x[A->col[e]]));
        res[i] = R(rhs[i] - s);
    }
}

/* y = M x for a rectangular CSR operator (restriction) */
static void matvec(const ocsr *M, const double *mv, const double *x, double *y, rfun R)
{
    for (int i = 0; i < M->n; i++) {
        double s = 0.0;
        for (int e = M->ptr[i]; e < M->ptr[i + 1]; e++) s = R(s + R(mv[e] * x[M->col[e]]));
        y[i] = s;
    }
}

/* x += M e (prolongation and correction) */
static void matvec_add(const ocsr *M, const double *mv, const double *e, double *x, rfun R)
{
    for (int i = 0; i < M->n; i++) {
        double s = 0.0;
        for (int f = M->ptr[i]; f < M->ptr[i + 1]; f++) s = R(s + R(mv[f] * e[M->col[f]]));
        x[i] = R(x[i] + s);
    }
}

/* exact coarsest solve by the Cholesky factor L L^T */
static void chol_solve(int n, const double *L, const double *b, double *x, rfun R)
{
    for (int i = 0; i < n; i++) {
        double s = b[i];
        for (int p = 0; p < i; p++) s = R(s - R(L[(size_t)i * n + p] * x[p]));
        x[i] = R(s / L[(size_t)i * n + i]);
    }
    for (int i = n - 1; i >= 0; i--) {
        double s = x[i];
        for (int p = i + 1; p < n; p++) s = R(s - R(L[(size_t)p * n + i] * x[p]));
        x[i] = R(s / L[(size_t)i * n + i]);
    }
}

/* V(1,1) cycle from a zero initial guess: x = V_l b */
static void vcycle(const orc *o, const bops *B, int l, const double *b, double *x)
{
    const olevel *lv = &o->lev[l];
    rfun R = B->R;
    int n = lv->A.n;
    if (l == o->nlev - 1) {
        chol_solve(n, B->chol, b, x, R);
        return;
    }
    int nc = lv->nc;
    double *r = malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *t = malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *bc = malloc((size_t)(nc > 0 ? nc : 1) * sizeof(double));
    double *ec = malloc((size_t)(nc > 0 ? nc : 1) * sizeof(double));
    for (int i = 0; i < n; i++) x[i] = R(B->ldinv[l][i] * b[i]);           /* presmooth */
    residual(&lv->A, B->lAval[l], b, x, r, R);
    matvec(&lv->R, B->lRval[l], r, bc, R);                                  /* restrict */
    vcycle(o, B, l + 1, bc, ec);
    matvec_add(&lv->P, B->lPval[l], ec, x, R);                              /* correct */
    sweep(&lv->A, B->lAval[l], B->ldinv[l], b, x, t, R);                    /* postsmooth */
    memcpy(x, t, (size_t)n * sizeof(double));
    free(r); free(t); free(bc); free(ec);
}

/* x = V b for the P^1 problem: the AMG V(1,1) cycle of Step 1 on its own */
int orc_apply_vcycle(const orc *o, int fp32, const double *b, double *x)
{
    if (o->nlev < 1 || o->nH < 1) return -1;
    bops B;
    bops_init(o, fp32, &B);
    double *bb = malloc((size_t)o->nH * sizeof(double));
    for (int i = 0; i < o->nH; i++) bb[i] = B.R(b[i]);
    vcycle(o, &B, 0, bb, x);
    free(bb);
    bops_free(&B);
    return 0;
}

/* z = B r */
static void apply_B(const orc *o, const bops *B, const double *rin, double *z)
{
    rfun R = B->R;
    int n = o->ndof, nH = o->nH;
    double *r = calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *t = malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *bH = malloc((size_t)(nH > 0 ? nH : 1) * sizeof(double));
    double *eH = malloc((size_t)(nH > 0 ? nH : 1) * sizeof(double));
    for (int i = 0; i < n; i++) r[i] = R(rin[i]);
    /* presmoothing: nu l1-Jacobi sweeps from z = 0 */
    for (int i = 0; i < n; i++) z[i] = R(B->dinv[i] * r[i]);
    for (int s = 1; s < o->nu; s++) {
        sweep(&o->A, B->Aval, B->dinv, r, z, t, R);
        memcpy(z, t, (size_t)n * sizeof(double));
    }
    /* Step 1: coarse equation A_H w_H = I_R (f - A_h u), by one V-cycle */
    residual(&o->A, B->Aval, r, z, t, R);
    matvec(&o->IR, B->IRval, t, bH, R);
    if (nH > 0) vcycle(o, B, 0, bH, eH);
    /* Step 2: correction u += I_P w_H */
    matvec_add(&o->IP, B->IPval, eH, z, R);
    /* Step 3: postsmoothing */
    for (int s = 0; s < o->nu; s++) {
        sweep(&o->A, B->Aval, B->dinv, r, z, t, R);
        memcpy(z, t, (size_t)n * sizeof(double));
    }
    free(r); free(t); free(bH); free(eH);
}

int orc_apply_precond(const orc *o, int fp32, const double *r, double *z)
{
    bops B;
    bops_init(o, fp32, &B);
    apply_B(o, &B, r, z);
    bops_free(&B);
    return 0;
}

static double dot(int n, const double *a, const double *b)
{
    double s = 0.0;
    for (int i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

static void spmv(const ocsr *A, const double *x, double *y)
{
    for (int i = 0; i < A->n; i++) {
        double s = 0.0;
        for (int e = A->ptr[i]; e < A->ptr[i + 1]; e++) s += A->val[e] * x[A->col[e]];
        y[i] = s;
    }
}

/* Preconditioned CG on A_h x = b from the given x.  Stops when
   ||r_k||_2 <= tol ||b||_2 (recursive residual).  Returns 0 converged,
   1 not converged in maxit, 2 breakdown (p.Ap <= 0 or r.z <= 0), 3 NaN. */
typedef void (*precfn)(void *ctx, const double *r, double *z);

static int pcg_core(const orc *o, precfn prec, void *ctx, const double *b, double *x, double tol, int maxit,
                    int *iters, double *relres)
{
    int n = o->ndof, status = 1, it = 0;
    double *r = malloc((size_t)n * sizeof(double)), *z = malloc((size_t)n * sizeof(double));
    double *p = malloc((size_t)n * sizeof(double)), *q = malloc((size_t)n * sizeof(double));
    spmv(&o->A, x, q);
    for (int i = 0; i < n; i++) r[i] = b[i] - q[i];
    double bn = sqrt(dot(n, b, b)), rn = sqrt(dot(n, r, r));
    if (bn == 0.0) {
        for (int i = 0; i < n; i++) x[i] = 0.0;
        rn = 0.0;
        bn = 1.0;
        status = 0;
        goto done;
    }
    if (rn <= tol * bn) { status = 0; goto done; }
    prec(ctx, r, z);
    double rho = dot(n, r, z);
    if (!(rho > 0.0)) { status = isnan(rho) ? 3 : 2; goto done; }
    memcpy(p, z, (size_t)n * sizeof(double));
    while (it < maxit) {
        spmv(&o->A, p, q);
        double pq = dot(n, p, q);
        if (!(pq > 0.0)) { status = isnan(pq) ? 3 : 2; break; }
        double alpha = rho / pq;
        for (int i = 0; i < n; i++) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        it++;
        rn = sqrt(dot(n, r, r));
        if (isnan(rn)) { status = 3; break; }
        if (rn <= tol * bn) { status = 0; break; }
        prec(ctx, r, z);
        double rho_new = dot(n, r, z);
        if (!(rho_new > 0.0)) { status = isnan(rho_new) ? 3 : 2; break; }
        double beta = rho_new / rho;
        rho = rho_new;
        for (int i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
    }
done:
    if (iters) *iters = it;
    if (relres) *relres = rn / bn;
    free(r); free(z); free(p); free(q);
    return status;
}

struct bctx { const orc *o; const bops *B; };
static void prec_B(void *c, const double *r, double *z)
{
    const struct bctx *b = c;
    apply_B(b->o, b->B, r, z);
}

int orc_pcg(const orc *o, int fp32, const double *b, double *x, double tol, int maxit,
            int *iters, double *relres)
{
    bops B;
    bops_init(o, fp32, &B);
    struct bctx c = {o, &B};
    int status = pcg_core(o, prec_B, &c, b, x, tol, maxit, iters, relres);
    bops_free(&B);
    return status;
}

/* ------------------------------------------------------------------------
 * Intermediate auxiliary space (Remark 6.2): the two-level method of
 * Algorithm 2.1 on P^k with the P^2 space of the same mesh in place of P^1,
 * made symmetric as above -- presmoothing, the residual restricted by I_2^T,
 * the P^2 problem solved approximately by one application of its own
 * auxiliary-space preconditioner B_2 (P^2 smoothing around the P^1 AMG
 * cycle), the correction prolonged by I_2 (Step 2), postsmoothing (Step 3).
 * B_2 is symmetric positive definite, so B stays symmetric; in the fp32 mode
 * B_2 runs in single precision too.
 * ------------------------------------------------------------------------ */
typedef struct {
    const double *I2val, *I2Tval;
    double *own[2];
} nops;

static void nops_init(const orc *o, rfun R, nops *N)
{
    size_t a = (size_t)o->I2.ptr[o->I2.n], b = (size_t)o->I2T.ptr[o->I2T.n];
    N->own[0] = malloc((a ? a : 1) * sizeof(double));
    N->own[1] = malloc((b ? b : 1) * sizeof(double));
    for (size_t e = 0; e < a; e++) N->own[0][e] = R(o->I2.val[e]);
    for (size_t e = 0; e < b; e++) N->own[1][e] = R(o->I2T.val[e]);
    N->I2val = N->own[0];
    N->I2Tval = N->own[1];
}

static void apply_B_nested(const orc *o, const bops *B, const bops *B2, const nops *N, const double *rin,
                           double *z)
{
    rfun R = B->R;
    const orc *o2 = o->aux2;
    int n = o->ndof, n2 = o2->ndof;
    double *r = calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *t = malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *b2 = malloc((size_t)(n2 > 0 ? n2 : 1) * sizeof(double));
    double *e2 = malloc((size_t)(n2 > 0 ? n2 : 1) * sizeof(double));
    for (int i = 0; i < n; i++) r[i] = R(rin[i]);
    /* presmoothing: nu l1-Jacobi sweeps from z = 0 */
    for (int i = 0; i < n; i++) z[i] = R(B->dinv[i] * r[i]);
    for (int s = 1; s < o->nu; s++) {
        sweep(&o->A, B->Aval, B->dinv, r, z, t, R);
        memcpy(z, t, (size_t)n * sizeof(double));
    }
    /* the P^2 equation A_2 w = I_2^T (f - A_h u), by one application of B_2 */
    residual(&o->A, B->Aval, r, z, t, R);
    matvec(&o->I2T, N->I2Tval, t, b2, R);
    if (n2 > 0) apply_B(o2, B2, b2, e2);
    /* correction u += I_2 w */
    matvec_add(&o->I2, N->I2val, e2, z, R);
    /* postsmoothing */
    for (int s = 0; s < o->nu; s++) {
        sweep(&o->A, B->Aval, B->dinv, r, z, t, R);
        memcpy(z, t, (size_t)n * sizeof(double));
    }
    free(r); free(t); free(b2); free(e2);
}

struct nctx { const orc *o; const bops *B, *B2; const nops *N; };
static void prec_nested(void *c, const double *r, double *z)
{
    const struct nctx *x = c;
    apply_B_nested(x->o, x->B, x->B2, x->N, r, z);
}

int orc_apply_nested(const orc *o, int fp32, const double *r, double *z)
{
    if (!o->aux2) return -1;
    bops B, B2;
    nops N;
    bops_init(o, fp32, &B);
    bops_init(o->aux2, fp32, &B2);
    nops_init(o, B.R, &N);
    apply_B_nested(o, &B, &B2, &N, r, z);
    bops_free(&B);
    bops_free(&B2);
    free(N.own[0]); free(N.own[1]);
    return 0;
}

int orc_pcg_nested(const orc *o, int fp32, const double *b, double *x, double tol, int maxit, int *iters,
                   double *relres)
{
    if (!o->aux2) return -1;
    bops B, B2;
    nops N;
    bops_init(o, fp32, &B);
    bops_init(o->aux2, fp32, &B2);
    nops_init(o, B.R, &N);
    struct nctx c = {o, &B, &B2, &N};
    int status = pcg_core(o, prec_nested, &c, b, x, tol, maxit, iters, relres);
    bops_free(&B);
    bops_free(&B2);
    free(N.own[0]); free(N.own[1]);
    return status;
}

/* Cholesky factor of a small dense SPD matrix (s x s, row-major) in place
   (lower triangle); returns 0, or -1 if a pivot is not positive. */
static int small_cholesky(int s, double *M)
{
    for (int j = 0; j < s; j++) {
        double d = M[j * s + j];
        for (int p = 0; p < j; p++) d -= M[j * s + p] * M[j * s + p];
        if (!(d > 0.0)) return -1;
        d = sqrt(d);
        M[j * s + j] = d;
        for (int i = j + 1; i < s; i++) {
            double t = M[i * s + j];
            for (int p = 0; p < j; p++) t -= M[i * s + p] * M[j * s + p];
            M[i * s + j] = t / d;
        }
    }
    return 0;
}

/* Y = M^{-1} Y for the Cholesky factor L of M (L L^T Y = Y), Y s x s row-major */
static void small_cholesky_solve(int s, const double *L, double *Y)
{
    for (int c = 0; c < s; c++) {
        for (int i = 0; i < s; i++) {
            double t = Y[i * s + c];
            for (int p = 0; p < i; p++) t -= L[i * s + p] * Y[p * s + c];
            Y[i * s + c] = t / L[i * s + i];
        }
        for (int i = s - 1; i >= 0; i--) {
            double t = Y[i * s + c];
            for (int p = i + 1; p < s; p++) t -= L[p * s + i] * Y[p * s + c];
            Y[i * s + c] = t / L[i * s + i];
        }
    }
}

/* G = U^T V for blocks U, V of n rows and s columns (row-major [n][s]) */
static void block_gram(int n, int s, const double *U, const double *V, double *G)
{
    for (int a = 0; a < s; a++)
        for (int b = 0; b < s; b++) {
            double t = 0.0;
            for (int i = 0; i < n; i++) t += U[(size_t)i * s + a] * V[(size_t)i * s + b];
            G[a * s + b] = t;
        }
}

/* Per-column relative residuals ||r_j|| / ||f_j|| of a block R; returns 3 on
   a NaN, 0 when every column with f_j != 0 meets tol, 1 otherwise. */
static int block_status(int n, int s, const double *R, const double *fn, double tol, double *relres)
{
    int ok = 1, bad = 0;
    for (int j = 0; j < s; j++) {
        double r2 = 0.0;
        for (int i = 0; i < n; i++) r2 += R[(size_t)i * s + j] * R[(size_t)i * s + j];
        relres[j] = fn[j] > 0.0 ? sqrt(r2) / fn[j] : 0.0;
        if (isnan(r2)) bad = 1;
        if (fn[j] > 0.0 && !(sqrt(r2) <= tol * fn[j])) ok = 0;
    }
    return bad ? 3 : (ok ? 0 : 1);
}

/* Block preconditioned CG (O'Leary 1980) on A_h X = F with s right-hand
   sides, blocks row-major [n][s], the preconditioner B applied column by
   column.  With gamma = Z^T R and delta = P^T A P (s x s):
       alpha = delta^{-1} gamma,  X += P alpha,  R -= A P alpha,
       Z = B R,  beta = gamma^{-1} gamma_new,  P = Z + P beta.
   Every column's iterate lies in the sum of the block Krylov spaces of all
   columns.  Stops when every column has ||r_j|| <= tol ||f_j|| (columns with
   f_j = 0 count as converged), after maxit iterations (status 1), on a
   non-positive pivot of delta or gamma (status 2, breakdown) or a NaN (3).
   relres[j] receives each column's final relative residual. */
int orc_block_pcg(const orc *o, int fp32, int s, const double *F, double *X, double tol, int maxit,
                  int *iters, double *relres)
{
    int n = o->ndof, status = 1, it = 0;
    if (s < 1) return -1;
    bops B;
    bops_init(o, fp32, &B);
    size_t ns = (size_t)n * s;
    double *R = malloc(ns * sizeof(double)), *Z = malloc(ns * sizeof(double));
    double *P = malloc(ns * sizeof(double)), *Q = malloc(ns * sizeof(double));
    double *col = malloc((size_t)n * sizeof(double)), *out = malloc((size_t)n * sizeof(double));
    double *gam = malloc((size_t)s * s * sizeof(double)), *gnew = malloc((size_t)s * s * sizeof(double));
    double *del = malloc((size_t)s * s * sizeof(double)), *coef = malloc((size_t)s * s * sizeof(double));
    double *fn = malloc((size_t)s * sizeof(double)), *Lg = malloc((size_t)s * s * sizeof(double));
    double *tmp = malloc((size_t)s * sizeof(double));

    /* R = F - A X, column by column */
    for (int j = 0; j < s; j++) {
        for (int i = 0; i < n; i++) col[i] = X[(size_t)i * s + j];
        spmv(&o->A, col, out);
        double f2 = 0.0;
        for (int i = 0; i < n; i++) {
            R[(size_t)i * s + j] = F[(size_t)i * s + j] - out[i];
            f2 += F[(size_t)i * s + j] * F[(size_t)i * s + j];
        }
        fn[j] = sqrt(f2);
    }
    int c = block_status(n, s, R, fn, tol, relres);
    if (c != 1) { status = c; goto done; }
    /* Z = B R; gamma = Z^T R; P = Z */
    for (int j = 0; j < s; j++) {
        for (int i = 0; i < n; i++) col[i] = R[(size_t)i * s + j];
        apply_B(o, &B, col, out);
        for (int i = 0; i < n; i++) Z[(size_t)i * s + j] = out[i];
    }
    block_gram(n, s, Z, R, gam);
    memcpy(P, Z, ns * sizeof(double));
    while (it < maxit) {
        /* Q = A P; delta = P^T Q; alpha = delta^{-1} gamma */
        for (int j = 0; j < s; j++) {
            for (int i = 0; i < n; i++) col[i] = P[(size_t)i * s + j];
            spmv(&o->A, col, out);
            for (int i = 0; i < n; i++) Q[(size_t)i * s + j] = out[i];
        }
        block_gram(n, s, P, Q, del);
        if (small_cholesky(s, del)) { status = 2; break; }
        memcpy(coef, gam, (size_t)s * s * sizeof(double));
        small_cholesky_solve(s, del, coef);
        /* X += P alpha; R -= Q alpha */
        for (int i = 0; i < n; i++)
            for (int b = 0; b < s; b++) {
                double px = 0.0, qx = 0.0;
                for (int a = 0; a < s; a++) {
                    px += P[(size_t)i * s + a] * coef[a * s + b];
                    qx += Q[(size_t)i * s + a] * coef[a * s + b];
                }
                X[(size_t)i * s + b] += px;
                R[(size_t)i * s + b] -= qx;
            }
        it++;
        c = block_status(n, s, R, fn, tol, relres);
        if (c != 1) { status = c; break; }
        /* Z = B R; beta = gamma^{-1} gamma_new; P = Z + P beta */
        for (int j = 0; j < s; j++) {
            for (int i = 0; i < n; i++) col[i] = R[(size_t)i * s + j];
            apply_B(o, &B, col, out);
            for (int i = 0; i < n; i++) Z[(size_t)i * s + j] = out[i];
        }
        block_gram(n, s, Z, R, gnew);
        memcpy(Lg, gam, (size_t)s * s * sizeof(double));
        if (small_cholesky(s, Lg)) { status = 2; break; }
        memcpy(coef, gnew, (size_t)s * s * sizeof(double));
        small_cholesky_solve(s, Lg, coef);
        for (int i = 0; i < n; i++) {
            for (int b = 0; b < s; b++) {
                double t = 0.0;
                for (int a = 0; a < s; a++) t += P[(size_t)i * s + a] * coef[a * s + b];
                tmp[b] = t;
            }
            for (int b = 0; b < s; b++) P[(size_t)i * s + b] = Z[(size_t)i * s + b] + tmp[b];
        }
        memcpy(gam, gnew, (size_t)s * s * sizeof(double));
    }
done:
    if (iters) *iters = it;
    free(R); free(Z); free(P); free(Q); free(col); free(out); free(gam); free(gnew); free(del);
    free(coef); free(fn); free(Lg); free(tmp);
    bops_free(&B);
    return status;
}

int orc_element_matrix(const orc *o, int t, double *K);

/* dL/dlog(kappa_t) = -lam_t^T K_t u_t for L(u) with A u = f and
   A lam = dL/du (K_t includes kappa_t; Dirichlet entries are zero) */
int orc_kappa_grad(const orc *o, const double *u, const double *lam, double *g)
{
    int nloc = o->nloc;
    double *K = malloc((size_t)nloc * nloc * sizeof(double));
    double ue[35], le[35];
    for (int t = 0; t < o->nt; t++) {
        for (int a = 0; a < nloc; a++) {
            int i = o->node_dof[o->tet_node[(size_t)t * nloc + a]];
            ue[a] = i >= 0 ? u[i] : 0.0;
            le[a] = i >= 0 ? lam[i] : 0.0;
        }
        orc_element_matrix(o, t, K);
        double s = 0.0;
        for (int a = 0; a < nloc; a++)
            for (int c = 0; c < nloc; c++) s += le[a] * K[a * nloc + c] * ue[c];
        g[t] = -s;
    }
    free(K);
    return 0;
}

/* Flexible GMRES(m), the Krylov method of the paper's Sec. 6.1 (Saad's
   flexible variant, right preconditioning): each Arnoldi step stores the
   preconditioned vector z_j = B v_j, orthogonalises w = A z_j against
   v_0..v_j by modified Gram-Schmidt, and the least-squares problem
   min ||beta e_1 - Hbar y|| is kept triangular by Givens rotations; at the
   end of a cycle x += Z y.  prec: 0 B in FP64, 1 B in FP32, 2 none (B = I).
   Stops when the rotated residual norm |g_{j+1}| <= tol ||r_0||_2, r_0 the
   residual of the initial x.  hist (optional, [maxit+1]) receives ||r_0||
   and the rotated residual norm after every Arnoldi step.  Returns 0
   converged, 1 not converged in maxit steps, 3 NaN; *relres is the true
   ||b - A x|| / ||r_0|| at exit. */
int orc_fgmres_core(const orc *o, int n, orc_vecop op, orc_vecop prec, void *ctx, const double *b, double *x,
                    double tol, int m, int maxit, int *iters, double *relres, double *hist)
{
    int status = 1, it = 0;
    if (m < 1) return -1;
    double *V = malloc((size_t)(m + 1) * n * sizeof(double));
    double *Z = malloc((size_t)m * n * sizeof(double));
    double *w = malloc((size_t)n * sizeof(double));
    double *H = calloc((size_t)(m + 1) * m, sizeof(double));   /* H[i*m + j] */
    double *cs = malloc((size_t)m * sizeof(double)), *sn = malloc((size_t)m * sizeof(double));
    double *g = malloc((size_t)(m + 1) * sizeof(double)), *y = malloc((size_t)m * sizeof(double));

    op(o, ctx, x, w);
    for (int i = 0; i < n; i++) w[i] = b[i] - w[i];
    double beta = sqrt(dot(n, w, w)), r0 = beta;
    if (hist) hist[0] = beta;
    if (beta == 0.0) { status = 0; goto done; }
    if (isnan(beta)) { status = 3; goto done; }
    while (it < maxit) {
        for (int i = 0; i < n; i++) V[i] = w[i] / beta;
        memset(g, 0, (size_t)(m + 1) * sizeof(double));
        g[0] = beta;
        int jend = 0, stop = 0;
        for (int j = 0; j < m && it < maxit; j++) {
            double *vj = V + (size_t)j * n, *zj = Z + (size_t)j * n;
            prec(o, ctx, vj, zj);
            op(o, ctx, zj, w);
            for (int i = 0; i <= j; i++) {
                const double *vi = V + (size_t)i * n;
                double h = dot(n, w, vi);
                H[(size_t)i * m + j] = h;
                for (int k = 0; k < n; k++) w[k] -= h * vi[k];
            }
            double hn = sqrt(dot(n, w, w));
            H[(size_t)(j + 1) * m + j] = hn;
            if (hn > 0.0)
                for (int k = 0; k < n; k++) V[(size_t)(j + 1) * n + k] = w[k] / hn;
            /* earlier rotations on the new column, then the rotation that
               zeroes its subdiagonal entry */
            for (int i = 0; i < j; i++) {
                double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            double a = H[(size_t)j * m + j], c = H[(size_t)(j + 1) * m + j];
            double d = sqrt(a * a + c * c);
            cs[j] = d > 0.0 ? a / d : 1.0;
            sn[j] = d > 0.0 ? c / d : 0.0;
            H[(size_t)j * m + j] = d;
            H[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            it++;
            jend = j + 1;
            double est = fabs(g[j + 1]);
            if (hist) hist[it] = est;
            if (isnan(est)) { status = 3; stop = 1; break; }
            if (est <= tol * r0) { status = 0; stop = 1; break; }
            if (hn == 0.0) break;   /* exact solution in this space */
        }
        if (status == 3) break;
        /* back substitution R y = g, then x += Z y */
        for (int i = jend - 1; i >= 0; i--) {
            double s = g[i];
            for (int k = i + 1; k < jend; k++) s -= H[(size_t)i * m + k] * y[k];
            y[i] = s / H[(size_t)i * m + i];
        }
        for (int j = 0; j < jend; j++)
            for (int k = 0; k < n; k++) x[k] += y[j] * Z[(size_t)j * n + k];
        op(o, ctx, x, w);
        for (int i = 0; i < n; i++) w[i] = b[i] - w[i];
        beta = sqrt(dot(n, w, w));
        if (stop) break;
        if (beta == 0.0) { status = 0; break; }
    }
done:
    op(o, ctx, x, w);
    for (int i = 0; i < n; i++) w[i] = b[i] - w[i];
    if (iters) *iters = it;
    if (relres) *relres = r0 > 0.0 ? sqrt(dot(n, w, w)) / r0 : 0.0;
    free(V); free(Z); free(w); free(H); free(cs); free(sn); free(g); free(y);
    return status;
}

/* the Poisson system: A_h and B in FP64 (mode 0), B in FP32 (1) or none (2) */
typedef struct {
    const bops *B;
    int mode;
} poisson_ctx;

static void poisson_op(const orc *o, void *ctx, const double *in, double *out)
{
    (void)ctx;
    spmv(&o->A, in, out);
}

static void poisson_prec(const orc *o, void *ctx, const double *in, double *out)
{
    const poisson_ctx *c = ctx;
    if (c->mode == 2) memcpy(out, in, (size_t)o->ndof * sizeof(double));
    else apply_B(o, c->B, in, out);
}

int orc_fgmres(const orc *o, int prec, const double *b, double *x, double tol, int m, int maxit,
               int *iters, double *relres, double *hist)
{
    bops B;
    bops_init(o, prec == 1, &B);
    poisson_ctx c = {&B, prec};
    int st = orc_fgmres_core(o, o->ndof, poisson_op, poisson_prec, &c, b, x, tol, m, maxit, iters, relres, hist);
    bops_free(&B);
    return st;
}

/* ------------------------------------------------------------------ Stokes
   The saddle-point system of Sec. 5,
       F [u; p] = [A B^T; B 0] [u; p] = [f; g],
   A = diag(A_h, A_h, A_h) (one P^2 Laplacian per velocity component),
   B = discrete -div, unknowns [u_x; u_y; u_z; p] (3 n_h + n_p), and the block
   upper triangular preconditioner Q_t of eq. (precond_t): for a residual
   [r_u; r_p],
       y_p = -M_p^{-1} r_p     (the Schur complement S = B A^{-1} B^T replaced
                                by the pressure mass matrix M_p, solved by
                                diagonally preconditioned CG),
       y_u = B_aux (r_u - B^T y_p) per component (one application of the
                                auxiliary-space preconditioner for A).
   Reading where the paper is silent: the M_p solve stops at a relative
   residual of 1e-6 (at most 200 steps). */
typedef struct {
    const bops *B;
    double *t, *c1, *c2;          /* work vectors */
    int mass_steps;               /* CG steps of the last pressure mass solve */
} stokes_ctx;

static void stokes_op(const orc *o, void *ctx, const double *in, double *out)
{
    stokes_ctx *c = ctx;
    int n = o->ndof, np = o->np;
    for (int k = 0; k < 3; k++) spmv(&o->A, in + (size_t)k * n, out + (size_t)k * n);
    spmv(&o->BdivT, in + 3 * (size_t)n, c->t);
    for (int i = 0; i < 3 * n; i++) out[i] += c->t[i];
    spmv(&o->Bdiv, in, out + 3 * (size_t)n);
    (void)np;
}

/* x = M_p^{-1} b by CG with the diagonal preconditioner, from x = 0 */
static int mass_pcg(const orc *o, const double *b, double *x, double rtol, int maxit)
{
    int np = o->np, it = 0;
    double *r = malloc((size_t)np * sizeof(double)), *z = malloc((size_t)np * sizeof(double));
    double *p = malloc((size_t)np * sizeof(double)), *q = malloc((size_t)np * sizeof(double));
    double *dg = malloc((size_t)np * sizeof(double));
    for (int i = 0; i < np; i++) {
        dg[i] = 0.0;
        for (int e = o->Mp.ptr[i]; e < o->Mp.ptr[i + 1]; e++)
            if (o->Mp.col[e] == i) dg[i] = o->Mp.val[e];
        x[i] = 0.0;
        r[i] = b[i];
        z[i] = r[i] / dg[i];
        p[i] = z[i];
    }
    double bn = sqrt(dot(np, b, b)), rho = dot(np, r, z);
    while (it < maxit && sqrt(dot(np, r, r)) > rtol * bn) {
        spmv(&o->Mp, p, q);
        double alpha = rho / dot(np, p, q);
        for (int i = 0; i < np; i++) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        for (int i = 0; i < np; i++) z[i] = r[i] / dg[i];
        double rho_new = dot(np, r, z);
        for (int i = 0; i < np; i++) p[i] = z[i] + (rho_new / rho) * p[i];
        rho = rho_new;
        it++;
    }
    free(r); free(z); free(p); free(q); free(dg);
    return it;
}

static void stokes_qt(const orc *o, void *ctx, const double *in, double *out)
{
    stokes_ctx *c = ctx;
    int n = o->ndof, np = o->np;
    double *yp = out + 3 * (size_t)n;
    c->mass_steps = mass_pcg(o, in + 3 * (size_t)n, yp, 1e-6, 200);
    for (int i = 0; i < np; i++) yp[i] = -yp[i];
    spmv(&o->BdivT, yp, c->t);
    for (int k = 0; k < 3; k++) {
        for (int i = 0; i < n; i++) c->c1[i] = in[(size_t)k * n + i] - c->t[(size_t)k * n + i];
        apply_B(o, c->B, c->c1, out + (size_t)k * n);
    }
}

int orc_stokes_fgmres(const orc *o, int fp32, const double *b, double *x, double tol, int m, int maxit,
                      int *iters, double *relres, double *hist)
{
    if (!o->np) return -1;
    bops B;
    bops_init(o, fp32, &B);
    int n = o->ndof;
    stokes_ctx c = {&B, malloc(3 * (size_t)n * sizeof(double)), malloc((size_t)n * sizeof(double)), NULL};
    int st = orc_fgmres_core(o, 3 * n + o->np, stokes_op, stokes_qt, &c, b, x, tol, m, maxit, iters, relres, hist);
    free(c.t);
    free(c.c1);
    bops_free(&B);
    return st;
}

/* out = F in (the saddle-point operator), for tests */
int orc_stokes_apply_operator(const orc *o, const double *in, double *out)
{
    if (!o->np) return -1;
    stokes_ctx c = {NULL, malloc(3 * (size_t)o->ndof * sizeof(double)), NULL, NULL};
    stokes_op(o, &c, in, out);
    free(c.t);
    return 0;
}

/* out = Q_t in with B in FP64 (fp32 = 0) or FP32, for tests; returns the
   pressure mass solve's CG step count (-1 before orc_stokes_setup) */
int orc_stokes_apply_qt(const orc *o, int fp32, const double *in, double *out)
{
    if (!o->np) return -1;
    bops B;
    bops_init(o, fp32, &B);
    stokes_ctx c = {&B, malloc(3 * (size_t)o->ndof * sizeof(double)), malloc((size_t)o->ndof * sizeof(double)), NULL, 0};
    stokes_qt(o, &c, in, out);
    free(c.t);
    free(c.c1);
    bops_free(&B);
    return c.mass_steps;
}
