// P^k Lagrange discretisation on tetrahedra and the P^1 auxiliary space
// (Sec. 2 of Lee-Leng-Zhang, arXiv:1204.2586).
//
//  * degrees of freedom: the evenly spaced nodes x_i^h of V_h; a node is the
//    multiset of k mesh vertices whose average is its position, so equal
//    multisets in neighbouring tets are the same node; nodes on boundary faces
//    carry u = 0 and are eliminated;
//  * A_h with (A_h)_ij = a(phi_j, phi_i) for a(u,v) = int kappa grad u.grad v
//    (eq. (2.2)-(2.5)); the element matrix is kappa * sum_pq G_pq M^pq, where
//    G_pq = |T| grad(lam_p).grad(lam_q) and M^pq are reference tables obtained
//    by exact integration of barycentric monomials;
//  * A_H the P^1 stiffness, I_P with entries c_j^i = psi_j(x_i^h) = (number of
//    times vertex j occurs in node i's multiset)/k, I_R = I_P^T (eq. "Prol").
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <exception>
#include <thread>

#include "parallel.hpp"
#include "setup.hpp"

namespace auxp {

using u128 = unsigned __int128;

std::vector<int> multi_indices(int k)
{
    std::vector<int> a;
    for (int a0 = 0; a0 <= k; a0++)
        for (int a1 = 0; a1 <= k - a0; a1++)
            for (int a2 = 0; a2 <= k - a0 - a1; a2++) {
                a.push_back(a0);
                a.push_back(a1);
                a.push_back(a2);
                a.push_back(k - a0 - a1 - a2);
            }
    return a;
}

// ------------------------------------------------------------------ tables

namespace {

double fact(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; i++) f *= i;
    return f;
}

// polynomial in one variable t: coefficients c[0..deg]
std::vector<double> lagrange_factor(int k, int a)
{
    // prod_{j<a} (k t - j)/(j+1)
    std::vector<double> c{1.0};
    for (int j = 0; j < a; j++) {
        std::vector<double> n(c.size() + 1, 0.0);
        for (size_t i = 0; i < c.size(); i++) {
            n[i + 1] += c[i] * k / (j + 1);
            n[i] -= c[i] * j / (j + 1);
        }
        c.swap(n);
    }
    return c;
}

std::vector<double> deriv(const std::vector<double> &c)
{
    std::vector<double> d(c.size() > 1 ? c.size() - 1 : 1, 0.0);
    for (size_t i = 1; i < c.size(); i++) d[i - 1] = c[i] * i;
    return d;
}

struct Term {
    int e[4];
    double c;
};

// d phi_alpha / d lam_p as a list of barycentric monomials
std::vector<Term> dphi(int k, const int *alpha, int p)
{
    std::vector<double> f[4];
    for (int q = 0; q < 4; q++) f[q] = lagrange_factor(k, alpha[q]);
    f[p] = deriv(f[p]);
    std::vector<Term> out;
    for (size_t i0 = 0; i0 < f[0].size(); i0++)
        for (size_t i1 = 0; i1 < f[1].size(); i1++)
            for (size_t i2 = 0; i2 < f[2].size(); i2++)
                for (size_t i3 = 0; i3 < f[3].size(); i3++) {
                    double c = f[0][i0] * f[1][i1] * f[2][i2] * f[3][i3];
                    if (c != 0.0) out.push_back({{(int)i0, (int)i1, (int)i2, (int)i3}, c});
                }
    return out;
}

// phi_alpha as a list of barycentric monomials
std::vector<Term> phi(int k, const int *alpha)
{
    std::vector<double> f[4];
    for (int q = 0; q < 4; q++) f[q] = lagrange_factor(k, alpha[q]);
    std::vector<Term> out;
    for (size_t i0 = 0; i0 < f[0].size(); i0++)
        for (size_t i1 = 0; i1 < f[1].size(); i1++)
            for (size_t i2 = 0; i2 < f[2].size(); i2++)
                for (size_t i3 = 0; i3 < f[3].size(); i3++) {
                    double c = f[0][i0] * f[1][i1] * f[2][i2] * f[3][i3];
                    if (c != 0.0) out.push_back({{(int)i0, (int)i1, (int)i2, (int)i3}, c});
                }
    return out;
}

// (1/|T|) int_T lam^e = 3! e0! e1! e2! e3! / (|e|+3)!
double simplex_moment(const int *e)
{
    return 6.0 * fact(e[0]) * fact(e[1]) * fact(e[2]) * fact(e[3]) / fact(e[0] + e[1] + e[2] + e[3] + 3);
}

struct Tables {
    int k = 0, nloc = 0;
    std::vector<double> M;   // [4][4][nloc][nloc]: (1/|T|) int dphi_a/dlam_p dphi_b/dlam_q
};

const Tables &tables(int k)
{
    static std::mutex mu;
    static std::map<int, Tables> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(k);
    if (it != cache.end()) return it->second;
    Tables t;
    t.k = k;
    std::vector<int> al = multi_indices(k);
    t.nloc = (int)al.size() / 4;
    int n = t.nloc;
    std::vector<std::vector<Term>> d((size_t)n * 4);
    for (int a = 0; a < n; a++)
        for (int p = 0; p < 4; p++) d[(size_t)a * 4 + p] = dphi(k, &al[4 * a], p);
    t.M.assign((size_t)16 * n * n, 0.0);
    for (int p = 0; p < 4; p++)
        for (int q = 0; q < 4; q++)
            for (int a = 0; a < n; a++)
                for (int b = 0; b < n; b++) {
                    double s = 0.0;
                    for (const Term &x : d[(size_t)a * 4 + p])
                        for (const Term &y : d[(size_t)b * 4 + q]) {
                            int e[4] = {x.e[0] + y.e[0], x.e[1] + y.e[1], x.e[2] + y.e[2], x.e[3] + y.e[3]};
                            s += x.c * y.c * simplex_moment(e);
                        }
                    t.M[(((size_t)p * 4 + q) * n + a) * n + b] = s;
                }
    return cache.emplace(k, std::move(t)).first->second;
}

}  // namespace

const std::vector<double> &stiffness_tables(int k) { return tables(k).M; }

void stokes_tables(int k, std::vector<double> &C, std::vector<double> &Mp)
{
    const std::vector<int> al = multi_indices(k), be = multi_indices(k - 1);
    const int n = (int)al.size() / 4, np = (int)be.size() / 4;
    std::vector<std::vector<Term>> ps(np);
    for (int p = 0; p < np; p++) ps[p] = phi(k - 1, &be[4 * p]);
    C.assign((size_t)4 * n * np, 0.0);
    for (int q = 0; q < 4; q++)
        for (int a = 0; a < n; a++) {
            const std::vector<Term> d = dphi(k, &al[4 * a], q);
            for (int p = 0; p < np; p++) {
                double s = 0.0;
                for (const Term &x : d)
                    for (const Term &y : ps[p]) {
                        int e[4] = {x.e[0] + y.e[0], x.e[1] + y.e[1], x.e[2] + y.e[2], x.e[3] + y.e[3]};
                        s += x.c * y.c * simplex_moment(e);
                    }
                C[((size_t)q * n + a) * np + p] = s;
            }
        }
    Mp.assign((size_t)np * np, 0.0);
    for (int p = 0; p < np; p++)
        for (int r = 0; r < np; r++) {
            double s = 0.0;
            for (const Term &x : ps[p])
                for (const Term &y : ps[r]) {
                    int e[4] = {x.e[0] + y.e[0], x.e[1] + y.e[1], x.e[2] + y.e[2], x.e[3] + y.e[3]};
                    s += x.c * y.c * simplex_moment(e);
                }
            Mp[(size_t)p * np + r] = s;
        }
}

double tet_gradients(const double *X0, const double *X1, const double *X2, const double *X3, double g[4][3])
{
    double e1[3], e2[3], e3[3];
    for (int d = 0; d < 3; d++) {
        e1[d] = X1[d] - X0[d];
        e2[d] = X2[d] - X0[d];
        e3[d] = X3[d] - X0[d];
    }
    double n1[3] = {e2[1] * e3[2] - e2[2] * e3[1], e2[2] * e3[0] - e2[0] * e3[2], e2[0] * e3[1] - e2[1] * e3[0]};
    double n2[3] = {e3[1] * e1[2] - e3[2] * e1[1], e3[2] * e1[0] - e3[0] * e1[2], e3[0] * e1[1] - e3[1] * e1[0]};
    double n3[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    double det = e1[0] * n1[0] + e1[1] * n1[1] + e1[2] * n1[2];
    for (int d = 0; d < 3; d++) {
        g[1][d] = n1[d] / det;
        g[2][d] = n2[d] / det;
        g[3][d] = n3[d] / det;
        g[0][d] = -g[1][d] - g[2][d] - g[3][d];
    }
    return det;
}

double tet_metric(const double *X0, const double *X1, const double *X2, const double *X3, double G[4][4])
{
    double g[4][3];
    const double det = tet_gradients(X0, X1, X2, X3, g);
    double vol = std::fabs(det) / 6.0;
    for (int p = 0; p < 4; p++)
        for (int q = 0; q < 4; q++) G[p][q] = vol * (g[p][0] * g[q][0] + g[p][1] * g[q][1] + g[p][2] * g[q][2]);
    return std::fabs(det);
}

namespace {

// K_t from the reference tables tb of the discretisation's order
void element_stiffness_from(const Tables &tb, const Discretization &d, int t, double *K)
{
    int n = tb.nloc;
    const int *v = &d.tets[4 * (size_t)t];
    double G[4][4];
    tet_metric(&d.xyz[3 * (size_t)v[0]], &d.xyz[3 * (size_t)v[1]], &d.xyz[3 * (size_t)v[2]],
               &d.xyz[3 * (size_t)v[3]], G);
    double kap = d.kappa[t];
    for (int i = 0; i < n * n; i++) K[i] = 0.0;
    for (int p = 0; p < 4; p++)
        for (int q = 0; q < 4; q++) {
            double g = kap * G[p][q];
            const double *M = &tb.M[((size_t)p * 4 + q) * n * n];
            for (int i = 0; i < n * n; i++) K[i] += g * M[i];
        }
}

}  // namespace

void element_stiffness(const Discretization &d, int t, double *K) { element_stiffness_from(tables(d.k), d, t, K); }

// --------------------------------------------------------------- sparse

Csr transpose(const Csr &a)
{
    Csr t;
    t.n = a.m;
    t.m = a.n;
    t.ptr.assign((size_t)a.m + 1, 0);
    for (int64_t e = 0; e < a.nnz(); e++) t.ptr[a.col[e] + 1]++;
    for (int j = 0; j < a.m; j++) t.ptr[j + 1] += t.ptr[j];
    t.col.resize(a.nnz());
    t.val.resize(a.nnz());
    std::vector<int> fill(t.ptr.begin(), t.ptr.end() - 1);
    for (int i = 0; i < a.n; i++)
        for (int e = a.ptr[i]; e < a.ptr[i + 1]; e++) {
            int p = fill[a.col[e]]++;
            t.col[p] = i;
            t.val[p] = a.val[e];
        }
    return t;
}

namespace {

// std::sort's result, from chunks sorted in parallel and merged pairwise
template <typename T>
void parallel_sort(std::vector<T> &v)
{
    const int nch = setup_threads(v.size());
    std::vector<size_t> b((size_t)nch + 1);
    for (int i = 0; i <= nch; i++) b[i] = v.size() * (size_t)i / (size_t)nch;
    run_tasks(nch, [&](int c) { std::sort(v.begin() + b[c], v.begin() + b[c + 1]); });
    for (int w = 1; w < nch; w *= 2) {
        std::vector<int> first;
        for (int i = 0; i + w < nch; i += 2 * w) first.push_back(i);
        run_tasks((int)first.size(), [&](int t) {
            const int i = first[t], end = std::min(i + 2 * w, nch);
            std::inplace_merge(v.begin() + b[i], v.begin() + b[i + w], v.begin() + b[end]);
        });
    }
}

// Sparsity pattern of the assembled operator whose element dof map is
// emap [nt][nl] (-1 = eliminated): row i couples to every dof of every element
// containing i.  Rows are built in parallel ranges and concatenated in order.
void build_pattern(int ndof, int nt, int nl, const int *emap, Csr &A)
{
    // dof -> elements incidence
    std::vector<int> cnt((size_t)ndof + 1, 0);
    for (size_t s = 0; s < (size_t)nt * nl; s++)
        if (emap[s] >= 0) cnt[emap[s] + 1]++;
    for (int i = 0; i < ndof; i++) cnt[i + 1] += cnt[i];
    std::vector<int> inc(cnt.back());
    std::vector<int> fill(cnt.begin(), cnt.end() - 1);
    for (size_t s = 0; s < (size_t)nt * nl; s++)
        if (emap[s] >= 0) inc[fill[emap[s]]++] = (int)(s / nl);
    A.n = A.m = ndof;
    A.ptr.assign((size_t)ndof + 1, 0);
    A.col.clear();
    const int nth = setup_threads((size_t)nt * nl * nl);
    std::vector<std::vector<int>> cols(nth);
    run_tasks(nth, [&](int w) {
        const int r0 = (int)((long long)ndof * w / nth), r1 = (int)((long long)ndof * (w + 1) / nth);
        std::vector<int> mark(ndof, -1), row;
        for (int i = r0; i < r1; i++) {
            row.clear();
            for (int e = cnt[i]; e < cnt[i + 1]; e++) {
                const int *dm = emap + (size_t)inc[e] * nl;
                for (int b = 0; b < nl; b++) {
                    int j = dm[b];
                    if (j >= 0 && mark[j] != i) {
                        mark[j] = i;
                        row.push_back(j);
                    }
                }
            }
            std::sort(row.begin(), row.end());
            cols[w].insert(cols[w].end(), row.begin(), row.end());
            A.ptr[i + 1] = (int)row.size();
        }
    });
    for (int i = 0; i < ndof; i++) A.ptr[i + 1] += A.ptr[i];
    A.col.reserve(A.ptr[ndof]);
    for (const std::vector<int> &c : cols) A.col.insert(A.col.end(), c.begin(), c.end());
    A.val.assign(A.col.size(), 0.0);
}

inline int find_col(const Csr &A, int i, int j)
{
    const int *b = &A.col[A.ptr[i]], *e = &A.col[0] + A.ptr[i + 1];
    return (int)(std::lower_bound(b, e, j) - &A.col[0]);
}

void check_mesh(int nv, const double *xyz, int nt, const int32_t *tets, const double *kappa)
{
    if (nv < 4 || nt < 1 || !xyz || !tets) throw std::invalid_argument("empty mesh");
    for (int64_t i = 0; i < 3LL * nv; i++)
        if (!std::isfinite(xyz[i])) throw std::invalid_argument("non-finite vertex coordinate");
    for (int t = 0; t < nt; t++) {
        const int32_t *v = tets + 4 * (size_t)t;
        for (int p = 0; p < 4; p++)
            if (v[p] < 0 || v[p] >= nv) throw std::invalid_argument("tet vertex index out of range");
        double G[4][4];
        double det = tet_metric(xyz + 3 * (size_t)v[0], xyz + 3 * (size_t)v[1], xyz + 3 * (size_t)v[2],
                                xyz + 3 * (size_t)v[3], G);
        double s = 0.0;
        for (int p = 1; p < 4; p++)
            for (int d = 0; d < 3; d++) s = std::max(s, std::fabs(xyz[3 * (size_t)v[p] + d] - xyz[3 * (size_t)v[0] + d]));
        if (!(det > 1e-12 * s * s * s)) throw std::invalid_argument("degenerate tetrahedron " + std::to_string(t));
        if (kappa && !(kappa[t] > 0.0 && std::isfinite(kappa[t])))
            throw std::invalid_argument("kappa must be positive and finite (tet " + std::to_string(t) + ")");
    }
}

u128 pack_ids(const int *ids, int n)
{
    u128 x = (u128)(unsigned)n << 120;
    for (int i = 0; i < n; i++) x |= (u128)(uint32_t)ids[i] << (32 * (2 - i));
    return x;
}

}  // namespace

void build_discretization(Discretization &d, int nv, const double *xyz, int nt, const int32_t *tets, int k,
                          const double *kappa)
{
    if (k < 2 || k > 4) throw std::invalid_argument("order must be 2, 3 or 4");
    check_mesh(nv, xyz, nt, tets, kappa);
    d.k = k;
    d.nv = nv;
    d.nt = nt;
    d.xyz.assign(xyz, xyz + 3 * (size_t)nv);
    d.tets.assign(tets, tets + 4 * (size_t)nt);
    d.kappa.assign((size_t)nt, 1.0);
    if (kappa) d.kappa.assign(kappa, kappa + nt);
    std::vector<int> al = multi_indices(k);
    int nl = d.nloc = (int)al.size() / 4;

    // nodes: sorted vertex multisets, numbered in lexicographic order
    std::vector<std::pair<u128, uint32_t>> nk((size_t)nt * nl);
    const int nkth = setup_threads((size_t)nt * nl);
    run_tasks(nkth, [&](int w) {
        for (int t = (int)((long long)nt * w / nkth); t < (int)((long long)nt * (w + 1) / nkth); t++)
            for (int a = 0; a < nl; a++) {
                int m[4], c = 0;
                for (int p = 0; p < 4; p++)
                    for (int r = 0; r < al[4 * a + p]; r++) m[c++] = tets[4 * (size_t)t + p];
                std::sort(m, m + k);
                u128 key = 0;
                for (int i = 0; i < 4; i++) key = (key << 32) | (u128)(uint32_t)(i < k ? m[i] : 0);
                nk[(size_t)t * nl + a] = {key, (uint32_t)((size_t)t * nl + a)};
            }
    });
    parallel_sort(nk);
    std::vector<int> tet_node((size_t)nt * nl);
    std::vector<u128> node_key;
    for (const auto &x : nk) {
        if (node_key.empty() || node_key.back() != x.first) node_key.push_back(x.first);
        tet_node[x.second] = (int)node_key.size() - 1;
    }
    int nnode = (int)node_key.size();

    // boundary sub-simplices: faces of a single tet, their edges and vertices
    std::vector<u128> faces((size_t)nt * 4);
    for (int t = 0; t < nt; t++)
        for (int f = 0; f < 4; f++) {
            int v[3], c = 0;
            for (int p = 0; p < 4; p++)
                if (p != f) v[c++] = tets[4 * (size_t)t + p];
            std::sort(v, v + 3);
            faces[(size_t)t * 4 + f] = pack_ids(v, 3);
        }
    parallel_sort(faces);
    std::vector<u128> bsub;
    for (size_t s = 0; s < faces.size();) {
        size_t e = s;
        while (e < faces.size() && faces[e] == faces[s]) e++;
        if (e - s == 1) {
            int v[3];
            for (int i = 0; i < 3; i++) v[i] = (int)(uint32_t)(faces[s] >> (32 * (2 - i)));
            bsub.push_back(faces[s]);
            for (int i = 0; i < 3; i++) {
                bsub.push_back(pack_ids(&v[i], 1));
                for (int j = i + 1; j < 3; j++) {
                    int ed[2] = {v[i], v[j]};
                    bsub.push_back(pack_ids(ed, 2));
                }
            }
        } else if (e - s > 2) {
            throw std::invalid_argument("non-manifold mesh: a face is shared by more than two tets");
        }
        s = e;
    }
    std::sort(bsub.begin(), bsub.end());
    bsub.erase(std::unique(bsub.begin(), bsub.end()), bsub.end());

    // node -> dof
    std::vector<int> node_dof(nnode);
    d.keys.clear();
    d.ndof = 0;
    for (int g = 0; g < nnode; g++) {
        int m[4], dist[4], nd = 0;
        for (int i = 0; i < k; i++) m[i] = (int)(uint32_t)(node_key[g] >> (32 * (3 - i)));
        for (int i = 0; i < k; i++)
            if (nd == 0 || dist[nd - 1] != m[i]) dist[nd++] = m[i];
        bool bnd = nd <= 3 && std::binary_search(bsub.begin(), bsub.end(), pack_ids(dist, nd));
        node_dof[g] = bnd ? -1 : d.ndof++;
        if (!bnd)
            for (int i = 0; i < k; i++) d.keys.push_back(m[i]);
    }
    d.tet_dof.resize((size_t)nt * nl);
    for (size_t s = 0; s < d.tet_dof.size(); s++) d.tet_dof[s] = node_dof[tet_node[s]];

    d.vert_dof.assign(nv, -1);
    d.nH = 0;
    for (int v = 0; v < nv; v++) {
        int id[1] = {v};
        bool bnd = std::binary_search(bsub.begin(), bsub.end(), pack_ids(id, 1));
        d.vert_dof[v] = bnd ? -1 : d.nH++;
    }

    // A_h
    build_pattern(d.ndof, nt, nl, d.tet_dof.data(), d.A);
    // blocks of tets: the element matrices in parallel, then the scatter in
    // parallel row ranges, each walking the block's tets in order (so every
    // entry is summed in tet order, as a sequential loop would)
    {
        const int nth = setup_threads((size_t)nt * nl * nl);
        const int blk = std::max(256, (1 << 21) / (nl * nl));
        const Tables &tb = tables(k);
        std::vector<double> Kb((size_t)blk * nl * nl);
        for (int t0 = 0; t0 < nt; t0 += blk) {
            const int t1 = std::min(nt, t0 + blk), nb = t1 - t0;
            run_tasks(nth, [&](int w) {
                for (int t = t0 + (int)((long long)nb * w / nth); t < t0 + (int)((long long)nb * (w + 1) / nth); t++)
                    element_stiffness_from(tb, d, t, &Kb[(size_t)(t - t0) * nl * nl]);
            });
            run_tasks(nth, [&](int w) {
                const int r0 = (int)((long long)d.ndof * w / nth), r1 = (int)((long long)d.ndof * (w + 1) / nth);
                std::vector<std::pair<int, int>> js(nl);   // (dof, local index), sorted by dof
                for (int t = t0; t < t1; t++) {
                    const int *dm = &d.tet_dof[(size_t)t * nl];
                    const double *K = &Kb[(size_t)(t - t0) * nl * nl];
                    int nj = -1;                           // sorted lazily, once per tet
                    for (int a = 0; a < nl; a++) {
                        const int i = dm[a];
                        if (i < r0 || i >= r1) continue;
                        if (nj < 0) {
                            nj = 0;
                            for (int b = 0; b < nl; b++)
                                if (dm[b] >= 0) js[nj++] = {dm[b], b};
                            std::sort(js.begin(), js.begin() + nj);
                        }
                        // one merge walk over row i's sorted columns
                        const int *col = d.A.col.data();
                        int e = d.A.ptr[i];
                        for (int q = 0; q < nj; q++) {
                            while (col[e] < js[q].first) e++;
                            d.A.val[e] += K[(size_t)a * nl + js[q].second];
                        }
                    }
                }
            });
        }
    }
    d.l1.assign(d.ndof, 0.0);
    const int l1th = setup_threads(d.A.col.size());
    run_tasks(l1th, [&](int w) {
        for (int i = (int)((long long)d.ndof * w / l1th); i < (int)((long long)d.ndof * (w + 1) / l1th); i++)
            for (int e = d.A.ptr[i]; e < d.A.ptr[i + 1]; e++) d.l1[i] += std::fabs(d.A.val[e]);
    });

    // A_H: kappa |T| grad lam_p . grad lam_q over interior vertices
    std::vector<int> vmap((size_t)nt * 4);
    for (size_t s = 0; s < vmap.size(); s++) vmap[s] = d.vert_dof[tets[s]];
    build_pattern(d.nH, nt, 4, vmap.data(), d.AH);
    for (int t = 0; t < nt; t++) {
        const int *v = tets + 4 * (size_t)t;
        double G[4][4];
        tet_metric(&d.xyz[3 * (size_t)v[0]], &d.xyz[3 * (size_t)v[1]], &d.xyz[3 * (size_t)v[2]],
                   &d.xyz[3 * (size_t)v[3]], G);
        for (int p = 0; p < 4; p++) {
            if (vmap[4 * (size_t)t + p] < 0) continue;
            for (int q = 0; q < 4; q++)
                if (vmap[4 * (size_t)t + q] >= 0)
                    d.AH.val[find_col(d.AH, vmap[4 * (size_t)t + p], vmap[4 * (size_t)t + q])] += d.kappa[t] * G[p][q];
        }
    }

    // I_P: psi_j(x_i) = multiplicity of vertex j in node i's multiset / k
    d.IP.n = d.ndof;
    d.IP.m = d.nH;
    d.IP.ptr.assign((size_t)d.ndof + 1, 0);
    d.IP.col.clear();
    d.IP.val.clear();
    for (int i = 0; i < d.ndof; i++) {
        const int32_t *m = &d.keys[(size_t)i * k];
        for (int s = 0; s < k;) {
            int e = s;
            while (e < k && m[e] == m[s]) e++;
            int j = d.vert_dof[m[s]];
            if (j >= 0) {
                d.IP.col.push_back(j);
                d.IP.val.push_back((double)(e - s) / k);
            }
            s = e;
        }
        d.IP.ptr[i + 1] = (int)d.IP.col.size();
    }
    d.IR = transpose(d.IP);
}

// ------------------------------------------------------------ P^k <- P^2

// P^2 on the same mesh is a subspace of P^k: at a node whose key has
// multiplicities m_p (barycentric coordinates lam_p = m_p / k) the nonzero
// P^2 basis values are those of the key's vertices, lam_p (2 lam_p - 1), and
// of its vertex pairs, 4 lam_p lam_q.  P^2 unknowns are found by their keys
// ((p, p) for a vertex, (p, q) for an edge) among d2's interior dofs;
// boundary ones drop out.  Zero weights (lam_p = 1/2) are not stored.
Csr p2_transfer(const Discretization &d, const Discretization &d2)
{
    if (d2.k != 2 || d.nv != d2.nv || d.nt != d2.nt || d.tets != d2.tets)
        throw std::invalid_argument("p2_transfer: the P^2 discretisation must be on the same mesh");
    const int k = d.k;
    auto find2 = [&](int a, int b) {
        int lo = 0, hi = d2.ndof;
        while (lo < hi) {
            const int mid = lo + (hi - lo) / 2;
            const int32_t *q = &d2.keys[(size_t)mid * 2];
            if (q[0] < a || (q[0] == a && q[1] < b)) lo = mid + 1;
            else hi = mid;
        }
        return lo < d2.ndof && d2.keys[(size_t)lo * 2] == a && d2.keys[(size_t)lo * 2 + 1] == b ? lo : -1;
    };
    Csr T;
    T.n = d.ndof;
    T.m = d2.ndof;
    T.ptr.assign((size_t)d.ndof + 1, 0);
    std::vector<std::pair<int, double>> row;
    for (int i = 0; i < d.ndof; i++) {
        const int32_t *key = &d.keys[(size_t)i * k];
        int vert[4], mult[4], nd = 0;
        for (int q = 0; q < k; q++) {
            if (nd > 0 && vert[nd - 1] == key[q]) {
                mult[nd - 1]++;
            } else {
                vert[nd] = key[q];
                mult[nd] = 1;
                nd++;
            }
        }
        row.clear();
        for (int p = 0; p < nd; p++) {
            const double lam = (double)mult[p] / k;
            const double w = lam * (2.0 * lam - 1.0);
            const int j = find2(vert[p], vert[p]);
            if (w != 0.0 && j >= 0) row.push_back({j, w});
        }
        for (int p = 0; p < nd; p++)
            for (int q = p + 1; q < nd; q++) {
                const double w = 4.0 * ((double)mult[p] / k) * ((double)mult[q] / k);
                const int j = find2(vert[p], vert[q]);
                if (j >= 0) row.push_back({j, w});
            }
        std::sort(row.begin(), row.end());
        for (auto &e : row) {
            T.col.push_back(e.first);
            T.val.push_back(e.second);
        }
        T.ptr[i + 1] = (int)T.col.size();
    }
    return T;
}

// ------------------------------------------------------------ assembly maps

void assembly_map(const Csr &A, int nt, int nl, const int *emap, std::vector<int> &ptr, std::vector<int> &idx)
{
    if ((int64_t)nt * nl * nl > 0x7fffffff) throw std::invalid_argument("assembly map: too many element entries");
    const size_t nnz = A.col.size();
    ptr.assign(nnz + 1, 0);
    // entry of row i, column j (columns of a row are sorted)
    auto entry = [&](int i, int j) { return find_col(A, i, j); };
    for (int t = 0; t < nt; t++) {
        const int *dm = emap + (size_t)t * nl;
        for (int a = 0; a < nl; a++) {
            if (dm[a] < 0) continue;
            for (int b = 0; b < nl; b++)
                if (dm[b] >= 0) ptr[entry(dm[a], dm[b]) + 1]++;
        }
    }
    for (size_t e = 0; e < nnz; e++) ptr[e + 1] += ptr[e];
    idx.assign((size_t)ptr[nnz], 0);
    std::vector<int> fill(ptr.begin(), ptr.end() - 1);
    for (int t = 0; t < nt; t++) {             // increasing t: the host assembly's order
        const int *dm = emap + (size_t)t * nl;
        for (int a = 0; a < nl; a++) {
            if (dm[a] < 0) continue;
            for (int b = 0; b < nl; b++)
                if (dm[b] >= 0) idx[fill[entry(dm[a], dm[b])]++] = (t * nl + a) * nl + b;
        }
    }
}

// ------------------------------------------------------------ load vector

namespace {

// eigen-decomposition of a small symmetric matrix by cyclic Jacobi rotations
void sym_eig(int n, std::vector<double> &a, std::vector<double> &v)
{
    v.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; i++) v[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; sweep++) {
        double off = 0.0;
        for (int p = 0; p < n; p++)
            for (int q = p + 1; q < n; q++) off += a[(size_t)p * n + q] * a[(size_t)p * n + q];
        if (off < 1e-40) break;
        for (int p = 0; p < n; p++)
            for (int q = p + 1; q < n; q++) {
                double apq = a[(size_t)p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                double theta = (a[(size_t)q * n + q] - a[(size_t)p * n + p]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int r = 0; r < n; r++) {
                    double arp = a[(size_t)r * n + p], arq = a[(size_t)r * n + q];
                    a[(size_t)r * n + p] = c * arp - s * arq;
                    a[(size_t)r * n + q] = s * arp + c * arq;
                }
                for (int r = 0; r < n; r++) {
                    double apr = a[(size_t)p * n + r], aqr = a[(size_t)q * n + r];
                    a[(size_t)p * n + r] = c * apr - s * aqr;
                    a[(size_t)q * n + r] = s * apr + c * aqr;
                }
                for (int r = 0; r < n; r++) {
                    double vrp = v[(size_t)r * n + p], vrq = v[(size_t)r * n + q];
                    v[(size_t)r * n + p] = c * vrp - s * vrq;
                    v[(size_t)r * n + q] = s * vrp + c * vrq;
                }
            }
    }
}

// m-point Gauss rule for int_0^1 (1-x)^a g(x) dx by the Golub-Welsch method
// (eigenvalues of the Jacobi matrix of the monic Jacobi polynomials)
void gauss_jacobi01(int m, int a, std::vector<double> &x, std::vector<double> &w)
{
    double A = a, B = 0.0;
    std::vector<double> J((size_t)m * m, 0.0), V;
    for (int n = 0; n < m; n++) {
        double s = 2.0 * n + A + B;
        J[(size_t)n * m + n] = (n == 0) ? (B - A) / (A + B + 2.0) : (B * B - A * A) / (s * (s + 2.0));
        if (n + 1 < m) {
            double k = n + 1, s1 = 2.0 * k + A + B;
            double beta = 4.0 * k * (k + A) * (k + B) * (k + A + B) / (s1 * s1 * (s1 + 1.0) * (s1 - 1.0));
            J[(size_t)n * m + n + 1] = J[(size_t)(n + 1) * m + n] = std::sqrt(beta);
        }
    }
    sym_eig(m, J, V);
    double mu0 = std::pow(2.0, A + 1.0) / (A + 1.0);
    std::vector<std::pair<double, double>> r(m);
    for (int i = 0; i < m; i++) r[i] = {J[(size_t)i * m + i], mu0 * V[i] * V[i]};
    std::sort(r.begin(), r.end());
    x.resize(m);
    w.resize(m);
    for (int i = 0; i < m; i++) {
        x[i] = 0.5 * (1.0 + r[i].first);
        w[i] = r[i].second / std::pow(2.0, A + 1.0);
    }
}

struct LoadRule {
    int m = 0;
    std::vector<double> lam, w, phi;   // phi: [nq][nloc]
};

const LoadRule &load_rule(int k)
{
    static std::mutex mu;
    static std::map<int, LoadRule> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(k);
    if (it != cache.end()) return it->second;
    LoadRule R;
    R.m = k + 2;
    int m = R.m;
    std::vector<double> xu, wu, xv, wv, xw, ww;
    gauss_jacobi01(m, 2, xu, wu);
    gauss_jacobi01(m, 1, xv, wv);
    gauss_jacobi01(m, 0, xw, ww);
    for (int a = 0; a < m; a++)
        for (int b = 0; b < m; b++)
            for (int c = 0; c < m; c++) {
                double l1 = xu[a], l2 = (1.0 - xu[a]) * xv[b], l3 = (1.0 - xu[a]) * (1.0 - xv[b]) * xw[c];
                R.lam.insert(R.lam.end(), {1.0 - l1 - l2 - l3, l1, l2, l3});
                R.w.push_back(wu[a] * wv[b] * ww[c]);
            }
    std::vector<int> al = multi_indices(k);
    int nl = (int)al.size() / 4, nq = m * m * m;
    for (int q = 0; q < nq; q++)
        for (int s = 0; s < nl; s++) {
            double v = 1.0;
            for (int p = 0; p < 4; p++) {
                std::vector<double> c = lagrange_factor(k, al[4 * s + p]);
                double t = R.lam[4 * (size_t)q + p], acc = 0.0, pw = 1.0;
                for (double ci : c) {
                    acc += ci * pw;
                    pw *= t;
                }
                v *= acc;
            }
            R.phi.push_back(v);
        }
    return cache.emplace(k, std::move(R)).first->second;
}

}  // namespace

int load_rule_points(int k) { return (k + 2) * (k + 2) * (k + 2); }

void quadrature_points(const Discretization &d, int t0, int t1, double *out)
{
    const LoadRule &R = load_rule(d.k);
    int nq = (int)R.w.size();
    for (int t = t0; t < t1; t++) {
        const int *v = &d.tets[4 * (size_t)t];
        for (int q = 0; q < nq; q++)
            for (int c = 0; c < 3; c++) {
                double s = 0.0;
                for (int p = 0; p < 4; p++) s += R.lam[4 * (size_t)q + p] * d.xyz[3 * (size_t)v[p] + c];
                out[((size_t)(t - t0) * nq + q) * 3 + c] = s;
            }
    }
}

void accumulate_load(const Discretization &d, int t0, int t1, const double *fq, double *b)
{
    const LoadRule &R = load_rule(d.k);
    int nq = (int)R.w.size(), nl = d.nloc;
    for (int t = t0; t < t1; t++) {
        const int *v = &d.tets[4 * (size_t)t];
        double G[4][4];
        double det = tet_metric(&d.xyz[3 * (size_t)v[0]], &d.xyz[3 * (size_t)v[1]], &d.xyz[3 * (size_t)v[2]],
                                &d.xyz[3 * (size_t)v[3]], G);
        const double *f = fq + (size_t)(t - t0) * nq;
        for (int a = 0; a < nl; a++) {
            int i = d.tet_dof[(size_t)t * nl + a];
            if (i < 0) continue;
            double s = 0.0;
            for (int q = 0; q < nq; q++) s += R.w[q] * f[q] * R.phi[(size_t)q * nl + a];
            b[i] += det * s;
        }
    }
}

}  // namespace auxp
