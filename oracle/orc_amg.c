/*
 * Test infrastructure (CPU oracle): classical AMG setup on the auxiliary
 * P^1 stiffness matrix A_H.
 *
 * The paper (Sec. 1 and Sec. 6.1) runs the auxiliary-space solve with
 * BoomerAMG using PMIS coarsening (De Sterck, Yang, Heys 2006) and extended+i
 * distance-two interpolation (De Sterck, Falgout, Nolting, Yang 2008), with
 * the strength-of-connection rule of Sec. 6.2: i depends strongly on j if
 * -a_ij > theta * max_{k != i}(-a_ik).  This file states those published
 * methods directly, one level at a time, followed by the Galerkin product
 * A_{l+1} = P_l^T A_l P_l.
 *
 * Readings where the paper is silent:
 *  - strict '>' in the strength test; a ratio equal to theta up to a relative
 *    1e-12 of the row maximum counts as a tie and is therefore not strong;
 *  - PMIS measure (|S_i^T|, rho_i, -i) compared lexicographically, with
 *    rho_i = splitmix64 output of (splitmix64(seed) + level*2^32 + i);
 *  - extended+i without the "+cc" restriction and without truncation;
 *  - coarsening stops when a level has <= coarse_max rows, when it does not
 *    shrink, or at max_levels; the coarsest level is solved exactly.
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* splitmix64 output function (Steele, Lea, Flood 2014) */
static uint64_t splitmix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static uint64_t pmis_rho(uint64_t seed, int level, int i)
{
    return splitmix64(splitmix64(seed) + ((uint64_t)level << 32) + (uint64_t)i);
}

/* S_i: the j != i that i strongly depends on */
static void strength(const ocsr *A, double theta, ocsr *S)
{
    int n = A->n;
    S->n = S->m = n;
    S->ptr = calloc((size_t)n + 1, sizeof(int));
    S->col = malloc((size_t)(A->ptr[n] ? A->ptr[n] : 1) * sizeof(int));
    S->val = NULL;
    int c = 0;
    for (int i = 0; i < n; i++) {
        double mx = -INFINITY;
        for (int e = A->ptr[i]; e < A->ptr[i + 1]; e++)
            if (A->col[e] != i && -A->val[e] > mx) mx = -A->val[e];
        if (mx > 0.0) {
            double thr = theta * mx + 1e-12 * mx;
            for (int e = A->ptr[i]; e < A->ptr[i + 1]; e++)
                if (A->col[e] != i && -A->val[e] > thr) S->col[c++] = A->col[e];
        }
        S->ptr[i + 1] = c;
    }
}

static int pattern_transpose(const ocsr *S, ocsr *T)
{
    ocsr tmp = *S;
    int nnz = S->ptr[S->n];
    double *dummy = calloc((size_t)(nnz ? nnz : 1), sizeof(double));
    tmp.val = dummy;
    ocsr_transpose(&tmp, T);
    free(dummy);
    return 0;
}

/* is i's measure larger than j's? */
static int beats(const int *nst, const uint64_t *rho, int i, int j)
{
    if (nst[i] != nst[j]) return nst[i] > nst[j];
    if (rho[i] != rho[j]) return rho[i] > rho[j];
    return i < j;
}

/* PMIS coarse/fine splitting: cf[i] = +1 (C) or -1 (F).  round[i] records
   when i was decided: 0 for points that influence nobody (F before the
   first round), r >= 1 for points that joined D or became F in round r. */
static void pmis(const ocsr *S, const ocsr *ST, uint64_t seed, int level, int *cf, int *round)
{
    int n = S->n;
    int *nst = malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    uint64_t *rho = malloc((size_t)(n > 0 ? n : 1) * sizeof(uint64_t));
    char *inD = calloc((size_t)(n > 0 ? n : 1), 1);
    for (int i = 0; i < n; i++) {
        nst[i] = ST->ptr[i + 1] - ST->ptr[i];
        rho[i] = pmis_rho(seed, level, i);
        cf[i] = nst[i] == 0 ? -1 : 0;       /* influences nobody: F */
        round[i] = 0;
    }
    for (int r = 1;; r++) {
        int left = 0;
        for (int i = 0; i < n; i++) left += cf[i] == 0;
        if (!left) break;
        /* D: undecided points whose measure beats every undecided neighbour */
        for (int i = 0; i < n; i++) {
            inD[i] = 0;
            if (cf[i] != 0) continue;
            int best = 1;
            for (int e = S->ptr[i]; e < S->ptr[i + 1] && best; e++) {
                int j = S->col[e];
                if (cf[j] == 0 && !beats(nst, rho, i, j)) best = 0;
            }
            for (int e = ST->ptr[i]; e < ST->ptr[i + 1] && best; e++) {
                int j = ST->col[e];
                if (cf[j] == 0 && !beats(nst, rho, i, j)) best = 0;
            }
            inD[i] = (char)best;
        }
        for (int i = 0; i < n; i++)
            if (inD[i]) { cf[i] = 1; round[i] = r; }
        /* undecided points that strongly depend on a new C point become F */
        for (int i = 0; i < n; i++) {
            if (cf[i] != 0) continue;
            for (int e = S->ptr[i]; e < S->ptr[i + 1]; e++)
                if (inD[S->col[e]]) { cf[i] = -1; round[i] = r; break; }
        }
    }
    free(nst); free(rho); free(inD);
}

/* extended+i interpolation */
static void ext_i_interp(const ocsr *A, const ocsr *S, const int *cf, ocsr *P, int *ncout)
{
    int n = A->n;
    int *cidx = malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    int nc = 0;
    for (int i = 0; i < n; i++) cidx[i] = cf[i] > 0 ? nc++ : -1;
    *ncout = nc;

    /* strong-neighbour marker per row, reset lazily */
    int *strong_of = malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    int *inC = malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    double *num = malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    int *list = malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    for (int i = 0; i < n; i++) { strong_of[i] = -1; inC[i] = -1; }

    size_t cap = (size_t)n * 8 + 16, nnz = 0;
    int *col = malloc(cap * sizeof(int));
    double *val = malloc(cap * sizeof(double));
    P->n = n;
    P->m = nc;
    P->ptr = calloc((size_t)n + 1, sizeof(int));
    for (int i = 0; i < n; i++) {
        int cnt = 0;
        if (cf[i] > 0) {
            list[cnt] = cidx[i];
            num[0] = 1.0;
            if (nnz + 1 > cap) { cap *= 2; col = realloc(col, cap * sizeof(int)); val = realloc(val, cap * sizeof(double)); }
            col[nnz] = cidx[i];
            val[nnz] = 1.0;
            nnz++;
            P->ptr[i + 1] = (int)nnz;
            continue;
        }
        /* hat C_i = (S_i cap C) cup union_{k in S_i cap F} (S_k cap C) */
        for (int e = S->ptr[i]; e < S->ptr[i + 1]; e++) strong_of[S->col[e]] = i;
        for (int e = S->ptr[i]; e < S->ptr[i + 1]; e++) {
            int j = S->col[e];
            if (cf[j] > 0) {
                if (inC[j] != i) { inC[j] = i; list[cnt++] = j; }
            } else {
                for (int f = S->ptr[j]; f < S->ptr[j + 1]; f++) {
                    int l = S->col[f];
                    if (cf[l] > 0 && inC[l] != i) { inC[l] = i; list[cnt++] = l; }
                }
            }
        }
        for (int x = 0; x < cnt; x++) num[list[x]] = 0.0;

        double aii = 0.0;
        for (int e = A->ptr[i]; e < A->ptr[i + 1]; e++)
            if (A->col[e] == i) aii += A->val[e];
        double diag = aii;
        for (int e = A->ptr[i]; e < A->ptr[i + 1]; e++) {
            int j = A->col[e];
            double aij = A->val[e];
            if (j == i) continue;
            if (inC[j] == i) {
                num[j] += aij;                         /* direct interpolatory */
            } else if (strong_of[j] == i && cf[j] < 0) {
                /* strong F neighbour k = j: distribute a_ik over hat C_i and i */
                int kk = j;
                double akk = 0.0;
                for (int f = A->ptr[kk]; f < A->ptr[kk + 1]; f++)
                    if (A->col[f] == kk) akk += A->val[f];
                double d = 0.0;
                for (int f = A->ptr[kk]; f < A->ptr[kk + 1]; f++) {
                    int l = A->col[f];
                    double akl = A->val[f];
                    double abar = (akl * akk < 0.0) ? akl : 0.0;
                    if (l == i || inC[l] == i) d += abar;
                }
                if (d == 0.0) {
                    diag += aij;
                } else {
                    for (int f = A->ptr[kk]; f < A->ptr[kk + 1]; f++) {
                        int l = A->col[f];
                        double akl = A->val[f];
                        double abar = (akl * akk < 0.0) ? akl : 0.0;
                        if (l == i) diag += aij * abar / d;
                        else if (inC[l] == i) num[l] += aij * abar / d;
                    }
                }
            } else {
                diag += aij;                           /* weak: lumped */
            }
        }
        /* emit sorted by coarse index (= fine index order) */
        for (int x = 1; x < cnt; x++)
            for (int y = x; y > 0 && list[y] < list[y - 1]; y--) {
                int t = list[y]; list[y] = list[y - 1]; list[y - 1] = t;
            }
        if (nnz + cnt > cap) {
            while (nnz + cnt > cap) cap *= 2;
            col = realloc(col, cap * sizeof(int));
            val = realloc(val, cap * sizeof(double));
        }
        for (int x = 0; x < cnt; x++) {
            col[nnz] = cidx[list[x]];
            val[nnz] = -num[list[x]] / diag;
            nnz++;
        }
        P->ptr[i + 1] = (int)nnz;
    }
    P->col = col;
    P->val = val;
    free(cidx); free(strong_of); free(inC); free(num); free(list);
}

static double *l1_norms(const ocsr *A)
{
    double *d = malloc((size_t)(A->n ? A->n : 1) * sizeof(double));
    for (int i = 0; i < A->n; i++) {
        double s = 0.0;
        for (int e = A->ptr[i]; e < A->ptr[i + 1]; e++) s += fabs(A->val[e]);
        d[i] = s;
    }
    return d;
}

/* dense lower Cholesky factor of an SPD matrix given in CSR */
static double *dense_cholesky(const ocsr *A)
{
    int n = A->n;
    double *L = calloc((size_t)n * n + 1, sizeof(double));
    for (int i = 0; i < n; i++)
        for (int e = A->ptr[i]; e < A->ptr[i + 1]; e++) L[(size_t)i * n + A->col[e]] = A->val[e];
    for (int j = 0; j < n; j++) {
        double s = L[(size_t)j * n + j];
        for (int p = 0; p < j; p++) s -= L[(size_t)j * n + p] * L[(size_t)j * n + p];
        if (!(s > 0.0)) { free(L); return NULL; }
        double d = sqrt(s);
        L[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; i++) {
            double t = L[(size_t)i * n + j];
            for (int p = 0; p < j; p++) t -= L[(size_t)i * n + p] * L[(size_t)j * n + p];
            L[(size_t)i * n + j] = t / d;
        }
    }
    for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++) L[(size_t)i * n + j] = 0.0;
    return L;
}

int orc_amg_setup(orc *o)
{
    /* level 0 operator: the P^1 stiffness itself */
    olevel *L0 = &o->lev[0];
    L0->A.n = o->AH.n;
    L0->A.m = o->AH.m;
    int nnz = o->AH.ptr[o->AH.n];
    L0->A.ptr = malloc(((size_t)o->AH.n + 1) * sizeof(int));
    L0->A.col = malloc((size_t)(nnz ? nnz : 1) * sizeof(int));
    L0->A.val = malloc((size_t)(nnz ? nnz : 1) * sizeof(double));
    memcpy(L0->A.ptr, o->AH.ptr, ((size_t)o->AH.n + 1) * sizeof(int));
    memcpy(L0->A.col, o->AH.col, (size_t)nnz * sizeof(int));
    memcpy(L0->A.val, o->AH.val, (size_t)nnz * sizeof(double));

    int maxl = o->max_levels < ORC_MAX_LEVELS ? o->max_levels : ORC_MAX_LEVELS;
    int l = 0;
    for (;;) {
        olevel *lv = &o->lev[l];
        lv->dl1 = l1_norms(&lv->A);
        int n = lv->A.n;
        if (n <= o->coarse_max || l + 1 >= maxl) break;
        ocsr S, ST;
        strength(&lv->A, o->theta, &S);
        pattern_transpose(&S, &ST);
        lv->cf = malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
        lv->round = malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
        pmis(&S, &ST, o->seed, l, lv->cf, lv->round);
        int nc;
        ext_i_interp(&lv->A, &S, lv->cf, &lv->P, &nc);
        free(S.ptr); free(S.col); free(ST.ptr); free(ST.col); free(ST.val);
        if (nc == 0 || nc >= n) {                  /* no coarsening possible */
            ocsr_free(&lv->P);
            free(lv->cf);
            free(lv->round);
            lv->cf = NULL;
            lv->round = NULL;
            break;
        }
        lv->nc = nc;
        ocsr_transpose(&lv->P, &lv->R);
        ocsr AP;
        ocsr_matmul(&lv->A, &lv->P, &AP);
        ocsr_matmul(&lv->R, &AP, &o->lev[l + 1].A);
        ocsr_free(&AP);
        l++;
    }
    o->nlev = l + 1;
    o->ncoarse = o->lev[l].A.n;
    if (o->ncoarse > 8192) return -4;
    o->chol = dense_cholesky(&o->lev[l].A);
    return o->chol ? 0 : -5;
}

/* exported for the hash test vector */
uint64_t orc_splitmix64(uint64_t z) { return splitmix64(z); }
uint64_t orc_pmis_rho(uint64_t seed, int level, int i) { return pmis_rho(seed, level, i); }

/* Extended+i interpolation of a caller-given matrix (CSR, sorted columns)
   and C/F splitting (cf[i] = +1 C, -1 F), with the strength sets of the
   Sec. 6.2 rule at threshold theta; for checking the interpolation step on
   its own.  Writes at most cap entries of P (n rows, CSR) and returns its
   number of entries, or -1 if cap is too small. */
int orc_interp_given(int n, const int *ptr, const int *col, const double *val, double theta,
                     const int *cf, int cap, int *pptr, int *pcol, double *pval)
{
    ocsr A = {n, n, (int *)ptr, (int *)col, (double *)val};
    ocsr S, P;
    int nc;
    strength(&A, theta, &S);
    ext_i_interp(&A, &S, cf, &P, &nc);
    int nnz = P.ptr[n];
    if (nnz <= cap) {
        memcpy(pptr, P.ptr, ((size_t)n + 1) * sizeof(int));
        memcpy(pcol, P.col, (size_t)nnz * sizeof(int));
        memcpy(pval, P.val, (size_t)nnz * sizeof(double));
    }
    free(S.ptr); free(S.col);
    ocsr_free(&P);
    return nnz <= cap ? nnz : -1;
}
