/*
 * Test infrastructure (CPU oracle): entry points called from Python (ctypes).
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

int orc_element_matrix(const orc *o, int t, double *K);
int orc_qpoints(const orc *o, int m, double *out);
int orc_load(const orc *o, int m, const double *fq, double *b);
double orc_l2_error(const orc *o, int m, const double *uq, const double *u);
double orc_h1_error(const orc *o, int m, const double *gq, const double *u);
int orc_apply_precond(const orc *o, int fp32, const double *r, double *z);
int orc_pcg(const orc *o, int fp32, const double *b, double *x, double tol, int maxit,
            int *iters, double *relres);
int orc_fgmres(const orc *o, int prec, const double *b, double *x, double tol, int m, int maxit,
               int *iters, double *relres, double *hist);
int orc_kappa_grad(const orc *o, const double *u, const double *lam, double *g);
int orc_block_pcg(const orc *o, int fp32, int s, const double *F, double *X, double tol, int maxit,
                  int *iters, double *relres);
int orc_stokes_fgmres(const orc *o, int fp32, const double *b, double *x, double tol, int m, int maxit,
                      int *iters, double *relres, double *hist);
int orc_stokes_apply_operator(const orc *o, const double *in, double *out);
int orc_stokes_apply_qt(const orc *o, int fp32, const double *in, double *out);

void orc_free(orc *o)
{
    if (!o) return;
    free(o->xyz); free(o->tets); free(o->kappa);
    free(o->node_key); free(o->tet_node); free(o->node_dof); free(o->vert_dof);
    ocsr_free(&o->A); free(o->dl1); ocsr_free(&o->AH); ocsr_free(&o->IP); ocsr_free(&o->IR);
    for (int l = 0; l < o->nlev; l++) {
        ocsr_free(&o->lev[l].A); free(o->lev[l].dl1); free(o->lev[l].cf); free(o->lev[l].round);
        ocsr_free(&o->lev[l].P); ocsr_free(&o->lev[l].R);
    }
    free(o->chol);
    ocsr_free(&o->Bdiv); ocsr_free(&o->BdivT); ocsr_free(&o->Mp);
    free(o->pnode_key); free(o->ptet_node);
    ocsr_free(&o->I2); ocsr_free(&o->I2T);
    free(o);
}

/* Discretise on the mesh (no AMG yet).  kappa may be NULL (= 1). */
orc *orc_create(int nv, const double *xyz, int nt, const int *tets, int k, const double *kappa)
{
    if (k < 1 || k > 4 || nv < 4 || nt < 1) return NULL;
    orc *o = calloc(1, sizeof(orc));
    o->k = k;
    o->nloc = (k + 1) * (k + 2) * (k + 3) / 6;
    o->nv = nv;
    o->nt = nt;
    o->xyz = malloc((size_t)nv * 3 * sizeof(double));
    memcpy(o->xyz, xyz, (size_t)nv * 3 * sizeof(double));
    o->tets = malloc((size_t)nt * 4 * sizeof(int));
    memcpy(o->tets, tets, (size_t)nt * 4 * sizeof(int));
    o->kappa = malloc((size_t)nt * sizeof(double));
    for (int t = 0; t < nt; t++) o->kappa[t] = kappa ? kappa[t] : 1.0;
    o->omega = 1.0;
    if (orc_build_mesh_dofs(o) || orc_assemble(o)) { orc_free(o); return NULL; }
    return o;
}

int orc_setup_amg(orc *o, double theta, int nu, int coarse_max, int max_levels, uint64_t seed)
{
    o->theta = theta;
    o->nu = nu;
    o->coarse_max = coarse_max;
    o->max_levels = max_levels;
    o->seed = seed;
    return orc_amg_setup(o);
}

int orc_stokes_setup(orc *o) { return o->np ? 0 : orc_stokes_assemble(o); }

/* weight of the P^k smoother: G_h = omega D_l1^{-1} */
void orc_set_smoother_weight(orc *o, double omega) { o->omega = omega; }

/* intermediate auxiliary space (Remark 6.2): o2 is the P^2 problem on the same
   mesh with its AMG set up (kept alive by the caller); nu sweeps on P^k */
int orc_setup_nested(orc *o, const orc *o2, int nu)
{
    if (!o2 || !o2->nlev) return -1;
    o->nu = nu;
    return orc_nested_transfer(o, o2);
}

/* pressure count and node keys [np][k-1] (after orc_stokes_setup) */
int orc_stokes_np(const orc *o) { return o->np; }
int orc_pressure_keys(const orc *o, int *keys)
{
    if (!o->np) return -1;
    memcpy(keys, o->pnode_key, (size_t)o->np * (o->k - 1) * sizeof(int));
    return 0;
}

/* sizes: [n_h, n_H, nnode, nlev, nnz(A_h), nnz(A_H), nnz(I_P), ncoarse, nloc] */
void orc_sizes(const orc *o, long long *s)
{
    s[0] = o->ndof; s[1] = o->nH; s[2] = o->nnode; s[3] = o->nlev;
    s[4] = o->A.ptr[o->A.n]; s[5] = o->AH.ptr[o->AH.n]; s[6] = o->IP.ptr[o->IP.n];
    s[7] = o->ncoarse; s[8] = o->nloc;
}

static const ocsr *pick(const orc *o, int which, int level)
{
    switch (which) {
    case 0: return &o->A;
    case 1: return &o->AH;
    case 2: return &o->IP;
    case 3: return level < o->nlev ? &o->lev[level].A : NULL;
    case 4: return level + 1 < o->nlev ? &o->lev[level].P : NULL;
    case 5: return o->np ? &o->Bdiv : NULL;
    case 6: return o->np ? &o->Mp : NULL;
    case 7: return o->aux2 ? &o->I2 : NULL;
    default: return NULL;
    }
}

/* shape of a matrix: out = [n, m, nnz] */
int orc_csr_shape(const orc *o, int which, int level, long long *out)
{
    const ocsr *a = pick(o, which, level);
    if (!a) return -1;
    out[0] = a->n; out[1] = a->m; out[2] = a->ptr[a->n];
    return 0;
}

int orc_csr_copy(const orc *o, int which, int level, int *ptr, int *col, double *val)
{
    const ocsr *a = pick(o, which, level);
    if (!a) return -1;
    memcpy(ptr, a->ptr, ((size_t)a->n + 1) * sizeof(int));
    memcpy(col, a->col, (size_t)a->ptr[a->n] * sizeof(int));
    memcpy(val, a->val, (size_t)a->ptr[a->n] * sizeof(double));
    return 0;
}

int orc_level_cf(const orc *o, int level, int *cf)
{
    if (level + 1 >= o->nlev) return -1;
    memcpy(cf, o->lev[level].cf, (size_t)o->lev[level].A.n * sizeof(int));
    return 0;
}

int orc_level_round(const orc *o, int level, int *round)
{
    if (level + 1 >= o->nlev) return -1;
    memcpy(round, o->lev[level].round, (size_t)o->lev[level].A.n * sizeof(int));
    return 0;
}

void orc_dof_keys(const orc *o, int *keys)
{
    for (int g = 0; g < o->nnode; g++) {
        int i = o->node_dof[g];
        if (i >= 0) memcpy(keys + (size_t)i * o->k, o->node_key + (size_t)g * o->k, o->k * sizeof(int));
    }
}

void orc_tet_dofs(const orc *o, int *out)
{
    for (size_t s = 0; s < (size_t)o->nt * o->nloc; s++) out[s] = o->node_dof[o->tet_node[s]];
}

void orc_l1(const orc *o, double *d) { memcpy(d, o->dl1, (size_t)o->ndof * sizeof(double)); }

void orc_coarse_chol(const orc *o, double *L)
{
    memcpy(L, o->chol, (size_t)o->ncoarse * o->ncoarse * sizeof(double));
}
