/*
 * Test infrastructure (CPU oracle): the GAMG preconditioner and CG.
 *
 * The preconditioner B is the two-level method of Algorithm 2.1 made
 * symmetric with a presmoothing step (Remark 2.1): smooth on the P^k system,
 * restrict the residual with I_R, solve the P^1 problem approximately by one
 * AMG V-cycle (Remark 2.1 allows "an AMG method or a few AMG cycles" for Step
 * 1), prolong with I_P (Step 2) and postsmooth (Step 3).  The smoother G_h,
 * which the paper leaves open, is l1-Jacobi: G_h = D_l1^{-1} with
 * D_l1 = diag(sum_j |a_ij|).  The outer iteration is preconditioned CG.
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
int orc_pcg(const orc *o, int fp32, const double *b, double *x, double tol, int maxit,
            int *iters, double *relres)
{
    int n = o->ndof, status = 1, it = 0;
    bops B;
    bops_init(o, fp32, &B);
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
    apply_B(o, &B, r, z);
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
        apply_B(o, &B, r, z);
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
