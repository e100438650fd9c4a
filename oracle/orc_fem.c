/*
 * Test infrastructure (CPU oracle): Lagrange P^k finite elements on
 * tetrahedra, the P^1 auxiliary space and the transfer between them.
 *
 * Follows Sec. 2 of Lee-Leng-Zhang: the P^k space V_h with evenly spaced
 * nodes (Sec. 2, definition of V_h and the node sets x_i^h), the stiffness
 * matrix (A_h)_ij = a(phi_j, phi_i) (eq. (2.5), "mat:eq"), the hat-function
 * space V_H and the transfer coefficients c_j^i = psi_j(x_i^h) that form
 * I_P, with I_R = I_P^T (eq. "Prol").
 *
 * Element integrals are computed by numerical quadrature of the gradients of
 * the nodal basis (a conical-product Gauss-Jacobi rule, exact for the
 * polynomial degrees involved).
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- basis */

/* multi-indices alpha in N^4 with |alpha| = k, lexicographic order */
int orc_local_multi_indices(int k, int *alpha)
{
    int c = 0;
    for (int a0 = 0; a0 <= k; a0++)
        for (int a1 = 0; a1 <= k - a0; a1++)
            for (int a2 = 0; a2 <= k - a0 - a1; a2++) {
                alpha[4 * c + 0] = a0;
                alpha[4 * c + 1] = a1;
                alpha[4 * c + 2] = a2;
                alpha[4 * c + 3] = k - a0 - a1 - a2;
                c++;
            }
    return c;
}

/* one factor prod_{j<a} (k t - j)/(j+1) of the nodal basis */
static double factor(int k, int a, double t)
{
    double f = 1.0;
    for (int j = 0; j < a; j++) f *= (k * t - j) / (j + 1);
    return f;
}

static double dfactor(int k, int a, double t)
{
    double d = 0.0;
    for (int m = 0; m < a; m++) {
        double g = (double)k / (m + 1);
        for (int j = 0; j < a; j++)
            if (j != m) g *= (k * t - j) / (j + 1);
        d += g;
    }
    return d;
}

/* nodal basis function of the node with barycentric index alpha/k:
   phi_alpha(lam) = prod_p prod_{j<alpha_p} (k lam_p - j)/(j+1) */
double orc_basis(int k, const int *alpha, const double *lam)
{
    double f = 1.0;
    for (int p = 0; p < 4; p++) f *= factor(k, alpha[p], lam[p]);
    return f;
}

/* partial derivatives d phi_alpha / d lam_p, treating the four
   barycentric coordinates as independent variables */
void orc_basis_dlam(int k, const int *alpha, const double *lam, double *d)
{
    for (int p = 0; p < 4; p++) {
        double g = dfactor(k, alpha[p], lam[p]);
        for (int q = 0; q < 4; q++)
            if (q != p) g *= factor(k, alpha[q], lam[q]);
        d[p] = g;
    }
}

/* ----------------------------------------------------------- quadrature */

/* Jacobi polynomial P_n^{(a,b)}(x) by its three-term recurrence */
static double jacobi(int n, double a, double b, double x)
{
    if (n == 0) return 1.0;
    double p0 = 1.0, p1 = 0.5 * (a - b + (a + b + 2.0) * x);
    for (int i = 2; i <= n; i++) {
        double c = 2.0 * i + a + b;
        double a1 = 2.0 * i * (i + a + b) * (c - 2.0);
        double a2 = (c - 1.0) * (a * a - b * b);
        double a3 = (c - 2.0) * (c - 1.0) * c;
        double a4 = 2.0 * (i + a - 1.0) * (i + b - 1.0) * c;
        double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

static double djacobi(int n, double a, double b, double x)
{
    if (n == 0) return 0.0;
    return 0.5 * (n + a + b + 1.0) * jacobi(n - 1, a + 1.0, b + 1.0, x);
}

/* m-point Gauss-Jacobi rule for int_0^1 (1-x)^a g(x) dx.
   Roots of P_m^{(a,0)} by Newton's method with deflation; for b = 0 the
   Gauss-Jacobi weight on [-1,1] is 2^{a+1} / ((1-x^2) P_m'(x)^2). */
int orc_gauss_jacobi(int m, int a, double *x, double *w)
{
    const double pi = 3.14159265358979323846;
    double r[32];
    if (m < 1 || m > 32) return -1;
    for (int i = 0; i < m; i++) {
        double z = -cos((2.0 * i + 1.0) * pi / (2.0 * m));
        for (int it = 0; it < 200; it++) {
            double p = jacobi(m, a, 0.0, z), dp = djacobi(m, a, 0.0, z);
            double s = 0.0;
            for (int j = 0; j < i; j++) s += 1.0 / (z - r[j]);
            double dz = p / (dp - p * s);
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        r[i] = z;
    }
    /* polish each root without deflation */
    for (int i = 0; i < m; i++)
        for (int it = 0; it < 3; it++) {
            double dp = djacobi(m, a, 0.0, r[i]);
            if (dp != 0.0) r[i] -= jacobi(m, a, 0.0, r[i]) / dp;
        }
    /* ascending order */
    for (int i = 1; i < m; i++)
        for (int j = i; j > 0 && r[j] < r[j - 1]; j--) {
            double t = r[j]; r[j] = r[j - 1]; r[j - 1] = t;
        }
    for (int i = 0; i < m; i++) {
        double dp = djacobi(m, a, 0.0, r[i]);
        double wi = pow(2.0, a + 1.0) / ((1.0 - r[i] * r[i]) * dp * dp);
        x[i] = 0.5 * (1.0 + r[i]);
        w[i] = wi / pow(2.0, a + 1.0);
    }
    return 0;
}

/* Conical-product rule on the reference tetrahedron {lam1,lam2,lam3 >= 0,
   lam1+lam2+lam3 <= 1} (volume 1/6) with m points per direction:
   lam1 = u, lam2 = (1-u) v, lam3 = (1-u)(1-v) w, lam0 = 1 - lam1 - lam2 - lam3,
   u ~ Gauss-Jacobi (1-u)^2, v ~ Gauss-Jacobi (1-v)^1, w ~ Gauss-Legendre.
   Point q = (iu*m + iv)*m + iw.  Exact for polynomials of degree <= 2m-1. */
int orc_tet_rule(int m, double *lam, double *w)
{
    double xu[32], wu[32], xv[32], wv[32], xw[32], ww[32];
    if (orc_gauss_jacobi(m, 2, xu, wu) || orc_gauss_jacobi(m, 1, xv, wv) ||
        orc_gauss_jacobi(m, 0, xw, ww))
        return -1;
    int q = 0;
    for (int a = 0; a < m; a++)
        for (int b = 0; b < m; b++)
            for (int c = 0; c < m; c++) {
                double l1 = xu[a];
                double l2 = (1.0 - xu[a]) * xv[b];
                double l3 = (1.0 - xu[a]) * (1.0 - xv[b]) * xw[c];
                lam[4 * q + 0] = 1.0 - l1 - l2 - l3;
                lam[4 * q + 1] = l1;
                lam[4 * q + 2] = l2;
                lam[4 * q + 3] = l3;
                w[q] = wu[a] * wv[b] * ww[c];
                q++;
            }
    return 0;
}

/* ------------------------------------------------------- sparse helpers */

void ocsr_free(ocsr *a)
{
    free(a->ptr);
    free(a->col);
    free(a->val);
    memset(a, 0, sizeof(*a));
}

/* sum duplicate (row, col) triplets into sorted CSR */
int ocsr_from_triplets(int n, int m, size_t cnt, const int *ri, const int *ci, const double *v,
                       ocsr *out)
{
    size_t *start = calloc((size_t)n + 1, sizeof(size_t));
    size_t *ord = malloc((cnt ? cnt : 1) * sizeof(size_t));
    int *mark = malloc((size_t)(m > 0 ? m : 1) * sizeof(int));
    double *acc = malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    int *list = malloc((size_t)(m > 0 ? m : 1) * sizeof(int));
    if (!start || !ord || !mark || !acc || !list) return -1;
    for (size_t t = 0; t < cnt; t++) start[ri[t] + 1]++;
    for (int i = 0; i < n; i++) start[i + 1] += start[i];
    size_t *fill = malloc(((size_t)n + 1) * sizeof(size_t));
    memcpy(fill, start, ((size_t)n + 1) * sizeof(size_t));
    for (size_t t = 0; t < cnt; t++) ord[fill[ri[t]]++] = t;
    free(fill);
    for (int j = 0; j < m; j++) mark[j] = -1;

    /* first pass: count unique columns per row */
    out->n = n;
    out->m = m;
    out->ptr = calloc((size_t)n + 1, sizeof(int));
    size_t nnz = 0;
    for (int i = 0; i < n; i++) {
        int c = 0;
        for (size_t s = start[i]; s < start[i + 1]; s++) {
            int j = ci[ord[s]];
            if (mark[j] != i) { mark[j] = i; c++; }
        }
        nnz += c;
        out->ptr[i + 1] = (int)nnz;
    }
    out->col = malloc((nnz ? nnz : 1) * sizeof(int));
    out->val = malloc((nnz ? nnz : 1) * sizeof(double));
    for (int j = 0; j < m; j++) mark[j] = -1;
    for (int i = 0; i < n; i++) {
        int c = 0;
        for (size_t s = start[i]; s < start[i + 1]; s++) {
            size_t t = ord[s];
            int j = ci[t];
            if (mark[j] != i) { mark[j] = i; acc[j] = v[t]; list[c++] = j; }
            else acc[j] += v[t];
        }
        for (int a = 1; a < c; a++)          /* insertion sort of the columns */
            for (int b = a; b > 0 && list[b] < list[b - 1]; b--) {
                int tmp = list[b]; list[b] = list[b - 1]; list[b - 1] = tmp;
            }
        int p = out->ptr[i];
        for (int a = 0; a < c; a++) {
            out->col[p + a] = list[a];
            out->val[p + a] = acc[list[a]];
        }
    }
    free(start); free(ord); free(mark); free(acc); free(list);
    return 0;
}

int ocsr_transpose(const ocsr *a, ocsr *t)
{
    t->n = a->m;
    t->m = a->n;
    int nnz = a->ptr[a->n];
    t->ptr = calloc((size_t)a->m + 1, sizeof(int));
    t->col = malloc((size_t)(nnz ? nnz : 1) * sizeof(int));
    t->val = malloc((size_t)(nnz ? nnz : 1) * sizeof(double));
    for (int e = 0; e < nnz; e++) t->ptr[a->col[e] + 1]++;
    for (int j = 0; j < a->m; j++) t->ptr[j + 1] += t->ptr[j];
    int *fill = malloc(((size_t)a->m + 1) * sizeof(int));
    memcpy(fill, t->ptr, ((size_t)a->m + 1) * sizeof(int));
    for (int i = 0; i < a->n; i++)
        for (int e = a->ptr[i]; e < a->ptr[i + 1]; e++) {
            int p = fill[a->col[e]]++;
            t->col[p] = i;          /* rows visited in increasing order: sorted */
            t->val[p] = a->val[e];
        }
    free(fill);
    return 0;
}

/* C = A B with a dense accumulator per row */
int ocsr_matmul(const ocsr *a, const ocsr *b, ocsr *c)
{
    int n = a->n, m = b->m;
    int *mark = malloc((size_t)(m > 0 ? m : 1) * sizeof(int));
    double *acc = malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    int *list = malloc((size_t)(m > 0 ? m : 1) * sizeof(int));
    for (int j = 0; j < m; j++) mark[j] = -1;
    size_t cap = (size_t)a->ptr[n] + 16, nnz = 0;
    int *col = malloc(cap * sizeof(int));
    double *val = malloc(cap * sizeof(double));
    c->n = n;
    c->m = m;
    c->ptr = calloc((size_t)n + 1, sizeof(int));
    for (int i = 0; i < n; i++) {
        int cnt = 0;
        for (int e = a->ptr[i]; e < a->ptr[i + 1]; e++) {
            int kk = a->col[e];
            double av = a->val[e];
            for (int f = b->ptr[kk]; f < b->ptr[kk + 1]; f++) {
                int j = b->col[f];
                if (mark[j] != i) { mark[j] = i; acc[j] = av * b->val[f]; list[cnt++] = j; }
                else acc[j] += av * b->val[f];
            }
        }
        for (int x = 1; x < cnt; x++)
            for (int y = x; y > 0 && list[y] < list[y - 1]; y--) {
                int tmp = list[y]; list[y] = list[y - 1]; list[y - 1] = tmp;
            }
        if (nnz + cnt > cap) {
            while (nnz + cnt > cap) cap *= 2;
            col = realloc(col, cap * sizeof(int));
            val = realloc(val, cap * sizeof(double));
        }
        for (int x = 0; x < cnt; x++) {
            col[nnz] = list[x];
            val[nnz] = acc[list[x]];
            nnz++;
        }
        c->ptr[i + 1] = (int)nnz;
    }
    c->col = col;
    c->val = val;
    free(mark); free(acc); free(list);
    return 0;
}

/* ----------------------------------------------------------- nodes / dofs */

static int g_k;                 /* key length for the comparators below */
static const int *g_keys;

static int cmp_key_idx(const void *pa, const void *pb)
{
    size_t a = *(const size_t *)pa, b = *(const size_t *)pb;
    const int *ka = g_keys + a * g_k, *kb = g_keys + b * g_k;
    for (int i = 0; i < g_k; i++)
        if (ka[i] != kb[i]) return ka[i] < kb[i] ? -1 : 1;
    return a < b ? -1 : (a > b);
}

static int cmp_tri(const void *pa, const void *pb)
{
    const int *a = pa, *b = pb;
    for (int i = 0; i < 3; i++)
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    return 0;
}

static void sort_small(int *v, int n)
{
    for (int a = 1; a < n; a++)
        for (int b = a; b > 0 && v[b] < v[b - 1]; b--) {
            int t = v[b]; v[b] = v[b - 1]; v[b - 1] = t;
        }
}

static int find_node(const orc *o, const int *key)
{
    int lo = 0, hi = o->nnode - 1, k = o->k;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        const int *km = o->node_key + (size_t)mid * k;
        int c = 0;
        for (int i = 0; i < k && !c; i++)
            if (km[i] != key[i]) c = km[i] < key[i] ? -1 : 1;
        if (!c) return mid;
        if (c < 0) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* Nodes: the local node alpha of tet (v0..v3) is identified by the multiset
   containing v_p alpha_p times (a sorted k-tuple); equal multisets in
   different tets are the same point of the conforming mesh.  Nodes on faces
   that belong to a single tet (the boundary) carry the homogeneous
   Dirichlet condition and are eliminated. */
int orc_build_mesh_dofs(orc *o)
{
    int k = o->k, nloc = o->nloc, nt = o->nt;
    int alpha[35 * 4];
    orc_local_multi_indices(k, alpha);
    size_t N = (size_t)nt * nloc;
    int *keys = malloc(N * k * sizeof(int));
    size_t *idx = malloc(N * sizeof(size_t));
    if (!keys || !idx) return -1;
    for (int t = 0; t < nt; t++)
        for (int a = 0; a < nloc; a++) {
            int *key = keys + ((size_t)t * nloc + a) * k, c = 0;
            for (int p = 0; p < 4; p++)
                for (int r = 0; r < alpha[4 * a + p]; r++) key[c++] = o->tets[4 * t + p];
            sort_small(key, k);
            idx[(size_t)t * nloc + a] = (size_t)t * nloc + a;
        }
    g_k = k;
    g_keys = keys;
    qsort(idx, N, sizeof(size_t), cmp_key_idx);

    o->tet_node = malloc(N * sizeof(int));
    o->node_key = malloc(N * k * sizeof(int));
    int nn = -1;
    for (size_t s = 0; s < N; s++) {
        const int *key = keys + idx[s] * k;
        if (nn < 0 || memcmp(key, o->node_key + (size_t)nn * k, k * sizeof(int)) != 0) {
            nn++;
            memcpy(o->node_key + (size_t)nn * k, key, k * sizeof(int));
        }
        o->tet_node[idx[s]] = nn;
    }
    o->nnode = nn + 1;
    free(keys);
    free(idx);

    /* boundary faces: faces of exactly one tet */
    int *tri = malloc((size_t)nt * 4 * 3 * sizeof(int));
    for (int t = 0; t < nt; t++)
        for (int f = 0; f < 4; f++) {
            int *tr = tri + ((size_t)t * 4 + f) * 3, c = 0;
            for (int p = 0; p < 4; p++)
                if (p != f) tr[c++] = o->tets[4 * t + p];
            sort_small(tr, 3);
        }
    qsort(tri, (size_t)nt * 4, 3 * sizeof(int), cmp_tri);
    char *bnd = calloc((size_t)o->nnode, 1);
    char *vbnd = calloc((size_t)o->nv, 1);
    size_t nf = (size_t)nt * 4;
    for (size_t s = 0; s < nf;) {
        size_t e = s + 1;
        while (e < nf && cmp_tri(tri + 3 * s, tri + 3 * e) == 0) e++;
        if (e - s == 1) {
            const int *tr = tri + 3 * s;
            for (int p = 0; p < 3; p++) vbnd[tr[p]] = 1;
            /* all multisets of size k drawn from the face's three vertices */
            int sel[8];
            for (int i = 0; i < k; i++) sel[i] = 0;
            for (;;) {
                int key[8];
                for (int i = 0; i < k; i++) key[i] = tr[sel[i]];
                int g = find_node(o, key);
                if (g < 0) { free(tri); free(bnd); free(vbnd); return -2; }
                bnd[g] = 1;
                int i = k - 1;
                while (i >= 0 && sel[i] == 2) i--;
                if (i < 0) break;
                sel[i]++;
                for (int j = i + 1; j < k; j++) sel[j] = sel[i];
            }
        }
        s = e;
    }
    free(tri);
    o->node_dof = malloc((size_t)o->nnode * sizeof(int));
    o->ndof = 0;
    for (int g = 0; g < o->nnode; g++) o->node_dof[g] = bnd[g] ? -1 : o->ndof++;
    o->vert_dof = malloc((size_t)o->nv * sizeof(int));
    o->nH = 0;
    for (int v = 0; v < o->nv; v++) o->vert_dof[v] = vbnd[v] ? -1 : o->nH++;
    free(bnd);
    free(vbnd);
    return 0;
}

/* ------------------------------------------------------------- assembly */

/* barycentric gradients of tet t and |det J| */
static double tet_geometry(const orc *o, int t, double grad[4][3])
{
    const double *X[4];
    for (int p = 0; p < 4; p++) X[p] = o->xyz + 3 * (size_t)o->tets[4 * t + p];
    double e[3][3];
    for (int q = 0; q < 3; q++)
        for (int d = 0; d < 3; d++) e[q][d] = X[q + 1][d] - X[0][d];
    double c23[3] = {e[1][1] * e[2][2] - e[1][2] * e[2][1], e[1][2] * e[2][0] - e[1][0] * e[2][2],
                     e[1][0] * e[2][1] - e[1][1] * e[2][0]};
    double c31[3] = {e[2][1] * e[0][2] - e[2][2] * e[0][1], e[2][2] * e[0][0] - e[2][0] * e[0][2],
                     e[2][0] * e[0][1] - e[2][1] * e[0][0]};
    double c12[3] = {e[0][1] * e[1][2] - e[0][2] * e[1][1], e[0][2] * e[1][0] - e[0][0] * e[1][2],
                     e[0][0] * e[1][1] - e[0][1] * e[1][0]};
    double det = e[0][0] * c23[0] + e[0][1] * c23[1] + e[0][2] * c23[2];
    for (int d = 0; d < 3; d++) {
        grad[1][d] = c23[d] / det;   /* rows of J^{-1}, J = [e1 e2 e3] */
        grad[2][d] = c31[d] / det;
        grad[3][d] = c12[d] / det;
        grad[0][d] = -(grad[1][d] + grad[2][d] + grad[3][d]);
    }
    return fabs(det);
}

/* element stiffness kappa_t * int_T grad phi_b . grad phi_a by quadrature */
int orc_element_matrix(const orc *o, int t, double *K)
{
    int k = o->k, nloc = o->nloc, m = k, nq = m * m * m;   /* exact to degree 2k-1 >= 2k-2 */
    int alpha[35 * 4];
    orc_local_multi_indices(k, alpha);
    double lam[4 * 512], w[512], grad[4][3];
    orc_tet_rule(m, lam, w);
    double det = tet_geometry(o, t, grad);
    double G[4][4];
    for (int p = 0; p < 4; p++)
        for (int q = 0; q < 4; q++)
            G[p][q] = grad[p][0] * grad[q][0] + grad[p][1] * grad[q][1] + grad[p][2] * grad[q][2];
    for (int i = 0; i < nloc * nloc; i++) K[i] = 0.0;
    double dl[35][4], gdl[35][4];
    for (int q = 0; q < nq; q++) {
        /* grad phi_a . grad phi_b = sum_{p,r} dphi_a/dlam_p (grad lam_p . grad lam_r) dphi_b/dlam_r */
        for (int a = 0; a < nloc; a++) {
            orc_basis_dlam(k, alpha + 4 * a, lam + 4 * q, dl[a]);
            for (int r = 0; r < 4; r++)
                gdl[a][r] = dl[a][0] * G[0][r] + dl[a][1] * G[1][r] + dl[a][2] * G[2][r] + dl[a][3] * G[3][r];
        }
        for (int a = 0; a < nloc; a++)
            for (int b = 0; b < nloc; b++)
                K[a * nloc + b] += w[q] * (gdl[a][0] * dl[b][0] + gdl[a][1] * dl[b][1] +
                                           gdl[a][2] * dl[b][2] + gdl[a][3] * dl[b][3]);
    }
    double c = o->kappa[t] * det;
    for (int i = 0; i < nloc * nloc; i++) K[i] *= c;
    return 0;
}

/* Stokes with the Hood-Taylor pair P^2-P^1 (Sec. 5, Sec. 6.3): pressure
   psi_q = lambda_q on every vertex q (no boundary condition), velocity the
   interior P^2 dofs of each component, component-major.
     (B)_{q,(c,i)} = - int psi_q dphi_i/dx_c   (B = discrete -div)
     (M_p)_{q,r}   =   int psi_q psi_r
   by quadrature (both integrands have degree 2; the rule with m = 2 points
   per direction is exact to degree 3). */
/* Hood-Taylor P^k - P^{k-1} (Sec. 5), k = 2, 3, 4: pressure in the
   continuous P^{k-1} space on every node of that order (no boundary
   condition), numbered like the velocity nodes by sorted vertex multisets
   (k - 1 vertex ids) in lexicographic order, so P^1 pressures are in vertex
   order.  B_{q,(c,i)} = -int psi_q dphi_i/dx_c and M_p = int psi_q psi_r by
   the conical-product rule with k points per direction, exact for these
   integrands of degree 2k - 2. */
int orc_stokes_assemble(orc *o)
{
    if (o->k < 2 || o->k > 4) return -1;
    const int k = o->k, kp = k - 1, nloc = o->nloc, n = o->ndof, m = k, nq = m * m * m;
    int alpha[35 * 4], beta[20 * 4];
    orc_local_multi_indices(k, alpha);
    const int nlp = orc_local_multi_indices(kp, beta);
    /* pressure nodes */
    const size_t N = (size_t)o->nt * nlp;
    int *keys = malloc(N * kp * sizeof(int));
    size_t *idx = malloc(N * sizeof(size_t));
    o->ptet_node = malloc(N * sizeof(int));
    o->pnode_key = malloc(N * kp * sizeof(int));
    if (!keys || !idx || !o->ptet_node || !o->pnode_key) return -2;
    for (int t = 0; t < o->nt; t++)
        for (int a = 0; a < nlp; a++) {
            int *key = keys + ((size_t)t * nlp + a) * kp, c = 0;
            for (int p = 0; p < 4; p++)
                for (int r = 0; r < beta[4 * a + p]; r++) key[c++] = o->tets[4 * t + p];
            sort_small(key, kp);
            idx[(size_t)t * nlp + a] = (size_t)t * nlp + a;
        }
    g_k = kp;
    g_keys = keys;
    qsort(idx, N, sizeof(size_t), cmp_key_idx);
    int np = -1;
    for (size_t s2 = 0; s2 < N; s2++) {
        const int *key = keys + idx[s2] * kp;
        if (np < 0 || memcmp(key, o->pnode_key + (size_t)np * kp, kp * sizeof(int)) != 0) {
            np++;
            memcpy(o->pnode_key + (size_t)np * kp, key, kp * sizeof(int));
        }
        o->ptet_node[idx[s2]] = np;
    }
    np++;
    free(keys);
    free(idx);
    o->nlp = nlp;

    double *lam = malloc((size_t)nq * 4 * sizeof(double)), *w = malloc((size_t)nq * sizeof(double));
    double grad[4][3];
    orc_tet_rule(m, lam, w);
    size_t capB = (size_t)o->nt * nlp * 3 * nloc, capM = (size_t)o->nt * nlp * nlp, cb = 0, cm = 0;
    int *bri = malloc(capB * sizeof(int)), *bci = malloc(capB * sizeof(int));
    double *bv = malloc(capB * sizeof(double));
    int *mri = malloc(capM * sizeof(int)), *mci = malloc(capM * sizeof(int));
    double *mv = malloc(capM * sizeof(double));
    double (*Bt)[3][35] = malloc(20 * sizeof(*Bt)), (*Mt)[20] = malloc(20 * sizeof(*Mt));
    if (!lam || !w || !bri || !bci || !bv || !mri || !mci || !mv || !Bt || !Mt) return -2;
    double dl[35][4], psi[20];
    for (int t = 0; t < o->nt; t++) {
        double det = tet_geometry(o, t, grad);
        memset(Bt, 0, 20 * sizeof(*Bt));
        memset(Mt, 0, 20 * sizeof(*Mt));
        for (int q = 0; q < nq; q++) {
            const double *lq = lam + 4 * q;
            for (int a = 0; a < nloc; a++) orc_basis_dlam(k, alpha + 4 * a, lq, dl[a]);
            for (int p = 0; p < nlp; p++) psi[p] = orc_basis(kp, beta + 4 * p, lq);
            for (int p = 0; p < nlp; p++) {
                for (int r = 0; r < nlp; r++) Mt[p][r] += w[q] * psi[p] * psi[r];
                for (int c = 0; c < 3; c++)
                    for (int a = 0; a < nloc; a++) {
                        /* dphi_a/dx_c = sum_s dphi_a/dlam_s dlam_s/dx_c */
                        double d = dl[a][0] * grad[0][c] + dl[a][1] * grad[1][c] + dl[a][2] * grad[2][c] +
                                   dl[a][3] * grad[3][c];
                        Bt[p][c][a] += w[q] * psi[p] * d;
                    }
            }
        }
        for (int p = 0; p < nlp; p++) {
            const int row = o->ptet_node[(size_t)t * nlp + p];
            for (int r = 0; r < nlp; r++) {
                mri[cm] = row; mci[cm] = o->ptet_node[(size_t)t * nlp + r]; mv[cm] = det * Mt[p][r]; cm++;
            }
            for (int c = 0; c < 3; c++)
                for (int a = 0; a < nloc; a++) {
                    int i = o->node_dof[o->tet_node[(size_t)t * nloc + a]];
                    if (i < 0) continue;
                    bri[cb] = row; bci[cb] = c * n + i; bv[cb] = -det * Bt[p][c][a]; cb++;
                }
        }
    }
    o->np = np;
    ocsr_from_triplets(np, 3 * n, cb, bri, bci, bv, &o->Bdiv);
    ocsr_from_triplets(np, np, cm, mri, mci, mv, &o->Mp);
    ocsr_transpose(&o->Bdiv, &o->BdivT);
    free(lam); free(w); free(Bt); free(Mt);
    free(bri); free(bci); free(bv); free(mri); free(mci); free(mv);
    return 0;
}

/* ||p - p_h||_{L2} of a pressure field (after orc_stokes_assemble): pq = exact
   p at the points of the m-point rule [nt*m^3], ph [np] */
double orc_pressure_l2_error(const orc *o, int m, const double *pq, const double *ph)
{
    int nq = m * m * m, kp = o->k - 1, nlp = o->nlp;
    int beta[20 * 4];
    orc_local_multi_indices(kp, beta);
    double *lam = malloc((size_t)nq * 4 * sizeof(double)), *w = malloc((size_t)nq * sizeof(double));
    orc_tet_rule(m, lam, w);
    double err = 0.0;
    for (int t = 0; t < o->nt; t++) {
        double grad[4][3];
        double det = tet_geometry(o, t, grad);
        for (int q = 0; q < nq; q++) {
            double v = 0.0;
            for (int a = 0; a < nlp; a++)
                v += ph[o->ptet_node[(size_t)t * nlp + a]] * orc_basis(kp, beta + 4 * a, lam + 4 * q);
            double d = pq[(size_t)t * nq + q] - v;
            err += det * w[q] * d * d;
        }
    }
    free(lam); free(w);
    return sqrt(err);
}

/* A_h, A_H, l1 norms and I_P */
int orc_assemble(orc *o)
{
    int nloc = o->nloc, nt = o->nt, k = o->k;
    size_t cap = (size_t)nt * nloc * nloc, cnt = 0;
    int *ri = malloc(cap * sizeof(int)), *ci = malloc(cap * sizeof(int));
    double *v = malloc(cap * sizeof(double));
    double *K = malloc((size_t)nloc * nloc * sizeof(double));
    if (!ri || !ci || !v || !K) return -1;
    for (int t = 0; t < nt; t++) {
        orc_element_matrix(o, t, K);
        for (int a = 0; a < nloc; a++) {
            int ia = o->node_dof[o->tet_node[(size_t)t * nloc + a]];
            if (ia < 0) continue;
            for (int b = 0; b < nloc; b++) {
                int ib = o->node_dof[o->tet_node[(size_t)t * nloc + b]];
                if (ib < 0) continue;
                ri[cnt] = ia; ci[cnt] = ib; v[cnt] = K[a * nloc + b]; cnt++;
            }
        }
    }
    ocsr_from_triplets(o->ndof, o->ndof, cnt, ri, ci, v, &o->A);
    o->dl1 = malloc((size_t)o->ndof * sizeof(double));
    for (int i = 0; i < o->ndof; i++) {
        double s = 0.0;
        for (int e = o->A.ptr[i]; e < o->A.ptr[i + 1]; e++) s += fabs(o->A.val[e]);
        o->dl1[i] = s;
    }

    /* P^1 stiffness: kappa |T| grad lam_p . grad lam_q on interior vertices */
    cnt = 0;
    for (int t = 0; t < nt; t++) {
        double grad[4][3];
        double det = tet_geometry(o, t, grad);
        double vol = det / 6.0;
        for (int p = 0; p < 4; p++) {
            int ip = o->vert_dof[o->tets[4 * t + p]];
            if (ip < 0) continue;
            for (int q = 0; q < 4; q++) {
                int iq = o->vert_dof[o->tets[4 * t + q]];
                if (iq < 0) continue;
                ri[cnt] = ip; ci[cnt] = iq;
                v[cnt] = o->kappa[t] * vol *
                         (grad[p][0] * grad[q][0] + grad[p][1] * grad[q][1] + grad[p][2] * grad[q][2]);
                cnt++;
            }
        }
    }
    ocsr_from_triplets(o->nH, o->nH, cnt, ri, ci, v, &o->AH);

    /* I_P: c_j^i = psi_j(x_i^h).  Evaluate every hat function of the tet at
       the node's position (barycentric coordinates from the geometry); the
       exact values are multiples of 1/k, to which rounding noise is snapped. */
    int alpha[35 * 4];
    orc_local_multi_indices(k, alpha);
    char *done = calloc((size_t)o->nnode, 1);
    cnt = 0;
    for (int t = 0; t < nt; t++) {
        double grad[4][3];
        tet_geometry(o, t, grad);
        const double *X0 = o->xyz + 3 * (size_t)o->tets[4 * t];
        for (int a = 0; a < nloc; a++) {
            int g = o->tet_node[(size_t)t * nloc + a];
            int i = o->node_dof[g];
            if (i < 0 || done[g]) continue;
            done[g] = 1;
            double x[3] = {0, 0, 0};
            for (int p = 0; p < 4; p++)
                for (int d = 0; d < 3; d++)
                    x[d] += (double)alpha[4 * a + p] / k * o->xyz[3 * (size_t)o->tets[4 * t + p] + d];
            double lam[4];
            lam[0] = 1.0;
            for (int p = 1; p < 4; p++) {
                lam[p] = grad[p][0] * (x[0] - X0[0]) + grad[p][1] * (x[1] - X0[1]) +
                         grad[p][2] * (x[2] - X0[2]);
                lam[0] -= lam[p];
            }
            for (int p = 0; p < 4; p++) {
                double s = round(lam[p] * k);
                if (fabs(lam[p] * k - s) > 1e-6) { free(done); return -3; }
                int j = o->vert_dof[o->tets[4 * t + p]];
                if (j < 0 || s == 0.0) continue;
                ri[cnt] = i; ci[cnt] = j; v[cnt] = s / k; cnt++;
            }
        }
    }
    free(done);
    ocsr_from_triplets(o->ndof, o->nH, cnt, ri, ci, v, &o->IP);
    ocsr_transpose(&o->IP, &o->IR);
    free(ri); free(ci); free(v); free(K);
    return 0;
}

/* ------------------------------------------- load vector and error norms */

int orc_qpoints(const orc *o, int m, double *out)
{
    int nq = m * m * m;
    double *lam = malloc((size_t)nq * 4 * sizeof(double)), *w = malloc((size_t)nq * sizeof(double));
    orc_tet_rule(m, lam, w);
    for (int t = 0; t < o->nt; t++)
        for (int q = 0; q < nq; q++)
            for (int d = 0; d < 3; d++) {
                double s = 0.0;
                for (int p = 0; p < 4; p++) s += lam[4 * q + p] * o->xyz[3 * (size_t)o->tets[4 * t + p] + d];
                out[((size_t)t * nq + q) * 3 + d] = s;
            }
    free(lam); free(w);
    return 0;
}

/* b_i = <f, phi_i> = sum_T int_T f phi_i, f given at the rule's points */
int orc_load(const orc *o, int m, const double *fq, double *b)
{
    int nq = m * m * m, k = o->k, nloc = o->nloc;
    int alpha[35 * 4];
    orc_local_multi_indices(k, alpha);
    double *lam = malloc((size_t)nq * 4 * sizeof(double)), *w = malloc((size_t)nq * sizeof(double));
    orc_tet_rule(m, lam, w);
    for (int i = 0; i < o->ndof; i++) b[i] = 0.0;
    for (int t = 0; t < o->nt; t++) {
        double grad[4][3];
        double det = tet_geometry(o, t, grad);
        for (int a = 0; a < nloc; a++) {
            int i = o->node_dof[o->tet_node[(size_t)t * nloc + a]];
            if (i < 0) continue;
            double s = 0.0;
            for (int q = 0; q < nq; q++)
                s += w[q] * fq[(size_t)t * nq + q] * orc_basis(k, alpha + 4 * a, lam + 4 * q);
            b[i] += det * s;
        }
    }
    free(lam); free(w);
    return 0;
}

/* ||u - u_h||_{L2}: uq = exact u at the rule's points, u = interior dofs */
double orc_l2_error(const orc *o, int m, const double *uq, const double *u)
{
    int nq = m * m * m, k = o->k, nloc = o->nloc;
    int alpha[35 * 4];
    orc_local_multi_indices(k, alpha);
    double *lam = malloc((size_t)nq * 4 * sizeof(double)), *w = malloc((size_t)nq * sizeof(double));
    orc_tet_rule(m, lam, w);
    double err = 0.0;
    for (int t = 0; t < o->nt; t++) {
        double grad[4][3];
        double det = tet_geometry(o, t, grad);
        for (int q = 0; q < nq; q++) {
            double uh = 0.0;
            for (int a = 0; a < nloc; a++) {
                int i = o->node_dof[o->tet_node[(size_t)t * nloc + a]];
                if (i >= 0) uh += u[i] * orc_basis(k, alpha + 4 * a, lam + 4 * q);
            }
            double d = uq[(size_t)t * nq + q] - uh;
            err += det * w[q] * d * d;
        }
    }
    free(lam); free(w);
    return sqrt(err);
}

/* |u - u_h|_{H1}: gq = exact grad u at the rule's points [nt*nq][3] */
double orc_h1_error(const orc *o, int m, const double *gq, const double *u)
{
    int nq = m * m * m, k = o->k, nloc = o->nloc;
    int alpha[35 * 4];
    orc_local_multi_indices(k, alpha);
    double *lam = malloc((size_t)nq * 4 * sizeof(double)), *w = malloc((size_t)nq * sizeof(double));
    orc_tet_rule(m, lam, w);
    double err = 0.0;
    for (int t = 0; t < o->nt; t++) {
        double grad[4][3];
        double det = tet_geometry(o, t, grad);
        for (int q = 0; q < nq; q++) {
            double gh[3] = {0, 0, 0};
            for (int a = 0; a < nloc; a++) {
                int i = o->node_dof[o->tet_node[(size_t)t * nloc + a]];
                if (i < 0) continue;
                double dl[4];
                orc_basis_dlam(k, alpha + 4 * a, lam + 4 * q, dl);
                for (int p = 0; p < 4; p++)
                    for (int d = 0; d < 3; d++) gh[d] += u[i] * dl[p] * grad[p][d];
            }
            for (int d = 0; d < 3; d++) {
                double e = gq[((size_t)t * nq + q) * 3 + d] - gh[d];
                err += det * w[q] * e * e;
            }
        }
    }
    free(lam); free(w);
    return sqrt(err);
}


/* ------------------------------------------------------------------------
 * Intermediate auxiliary space (Remark 6.2).  The P^2 space of the same mesh
 * is a subspace of P^k (k >= 2), so a P^2 function has exact P^k nodal
 * values.  At a P^k node with key multiplicities alpha_p (barycentric
 * coordinates lam_p = alpha_p / k in any tet holding it) the P^2 basis
 * functions that do not vanish belong to the vertices and edges of the key:
 * vertex functions lam_p (2 lam_p - 1) and edge functions 4 lam_p lam_q.
 * Rows: interior P^k dofs; columns: interior P^2 dofs (the Dirichlet nodes'
 * functions vanish on the boundary, so they drop out).  Exact zeros (lam_p =
 * 1/2) are not stored.
 * ------------------------------------------------------------------------ */

/* node of the P^2 problem with key (a, b), a <= b, or -1 */
static int p2_node(const orc *o2, int a, int b)
{
    int lo = 0, hi = o2->nnode;
    while (lo < hi) {
        int mid = lo + (hi - lo) / 2;
        const int *kk = o2->node_key + 2 * (size_t)mid;
        if (kk[0] < a || (kk[0] == a && kk[1] < b)) lo = mid + 1;
        else hi = mid;
    }
    if (lo < o2->nnode && o2->node_key[2 * (size_t)lo] == a && o2->node_key[2 * (size_t)lo + 1] == b) return lo;
    return -1;
}

int orc_nested_transfer(orc *o, const orc *o2)
{
    if (!o2 || o2->k != 2 || o->k < 2 || o2->nv != o->nv || o2->nt != o->nt) return -1;
    if (memcmp(o2->tets, o->tets, (size_t)o->nt * 4 * sizeof(int)) != 0) return -1;
    int k = o->k;
    size_t cap = (size_t)o->ndof * 10 + 1, cnt = 0;
    int *ri = malloc(cap * sizeof(int)), *ci = malloc(cap * sizeof(int));
    double *v = malloc(cap * sizeof(double));
    for (int g = 0; g < o->nnode; g++) {
        int i = o->node_dof[g];
        if (i < 0) continue;
        const int *key = o->node_key + (size_t)g * k;
        int vert[4], mult[4], nd = 0;
        for (int q = 0; q < k; q++) {
            if (nd > 0 && vert[nd - 1] == key[q]) mult[nd - 1]++;
            else { vert[nd] = key[q]; mult[nd] = 1; nd++; }
        }
        double lam[4];
        for (int p = 0; p < nd; p++) lam[p] = (double)mult[p] / k;
        for (int p = 0; p < nd; p++) {
            double w = lam[p] * (2.0 * lam[p] - 1.0);
            int node = p2_node(o2, vert[p], vert[p]);
            int j = node >= 0 ? o2->node_dof[node] : -1;
            if (w != 0.0 && j >= 0) { ri[cnt] = i; ci[cnt] = j; v[cnt] = w; cnt++; }
        }
        for (int p = 0; p < nd; p++)
            for (int q = p + 1; q < nd; q++) {
                double w = 4.0 * lam[p] * lam[q];
                int node = p2_node(o2, vert[p], vert[q]);
                int j = node >= 0 ? o2->node_dof[node] : -1;
                if (j >= 0) { ri[cnt] = i; ci[cnt] = j; v[cnt] = w; cnt++; }
            }
    }
    ocsr_free(&o->I2);
    ocsr_free(&o->I2T);
    int rc = ocsr_from_triplets(o->ndof, o2->ndof, cnt, ri, ci, v, &o->I2);
    if (!rc) rc = ocsr_transpose(&o->I2, &o->I2T);
    free(ri); free(ci); free(v);
    if (!rc) o->aux2 = o2;
    return rc;
}
