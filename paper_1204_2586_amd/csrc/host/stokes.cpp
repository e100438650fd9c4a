// Blocks of the Hood-Taylor P^k - P^{k-1} discretisation of the Stokes system
// (Sec. 5: velocity in P^{k,0}, pressure in P^{k-1,0}, the stable pairs of
// the paper's second test problem, k = 2, 3, 4).  With the velocity test
// functions phi_i e_c and the pressure basis psi_p (Lagrange functions on
// every node of order k-1, no boundary condition on p):
//   B_{p, (c, i)} = -int_T psi_p dphi_i/dx_c,  M_p = int psi_p psi_q.
// Per tet, dphi_i/dx_c = sum_q (dphi_i/dlam_q) (grad lam_q)_c, so the element
// block is -|T| sum_q (grad lam_q)_c C[q][i][p] with the exact moment table
// C[q][i][p] = (1/|T|) int psi_p dphi_i/dlam_q, and the mass matrix is |T|
// times its reference table, both integrated exactly.
#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <vector>

#include "setup.hpp"

namespace auxp {

namespace {

// CSR pattern of rows over `nr` row ids from the per-tet row map
// rmap[nt][rl] coupled with the per-tet column map cmap[nt][cl] (-1 =
// eliminated), columns sorted; values zero.
void coupling_pattern(int nr, int ncol, int nt, int rl, const int *rmap, int cl, const int *cmap, Csr &A)
{
    std::vector<int> cnt((size_t)nr + 1, 0);
    for (size_t s = 0; s < (size_t)nt * rl; s++) cnt[rmap[s] + 1]++;
    for (int i = 0; i < nr; i++) cnt[i + 1] += cnt[i];
    std::vector<int> inc(cnt.back()), fill(cnt.begin(), cnt.end() - 1);
    for (size_t s = 0; s < (size_t)nt * rl; s++) inc[fill[rmap[s]]++] = (int)(s / rl);
    A.n = nr;
    A.m = ncol;
    A.ptr.assign((size_t)nr + 1, 0);
    A.col.clear();
    std::vector<int> mark(ncol, -1), row;
    for (int i = 0; i < nr; i++) {
        row.clear();
        for (int e = cnt[i]; e < cnt[i + 1]; e++) {
            const int *cm = cmap + (size_t)inc[e] * cl;
            for (int b = 0; b < cl; b++) {
                const int j = cm[b];
                if (j >= 0 && mark[j] != i) {
                    mark[j] = i;
                    row.push_back(j);
                }
            }
        }
        std::sort(row.begin(), row.end());
        A.col.insert(A.col.end(), row.begin(), row.end());
        A.ptr[i + 1] = (int)A.col.size();
    }
    A.val.assign(A.col.size(), 0.0);
}

// position of column j in row i of A (the pattern holds it)
inline int entry(const Csr &A, int i, int j)
{
    const int *b = A.col.data() + A.ptr[i], *e = A.col.data() + A.ptr[i + 1];
    return (int)(std::lower_bound(b, e, j) - A.col.data());
}

// Pressure nodes: every local node of order kp of every tet, identified by
// its sorted vertex multiset; numbered in lexicographic key order.
int pressure_nodes(const Discretization &d, int kp, std::vector<int> &ptet, std::vector<int32_t> &pkeys)
{
    const std::vector<int> be = multi_indices(kp);
    const int nlp = (int)be.size() / 4, nt = d.nt;
    std::vector<std::vector<int32_t>> keys((size_t)nt * nlp);
    for (int t = 0; t < nt; t++)
        for (int a = 0; a < nlp; a++) {
            std::vector<int32_t> &key = keys[(size_t)t * nlp + a];
            for (int p = 0; p < 4; p++)
                for (int r = 0; r < be[4 * a + p]; r++) key.push_back(d.tets[4 * (size_t)t + p]);
            std::sort(key.begin(), key.end());
        }
    std::vector<std::vector<int32_t>> uniq(keys);
    std::sort(uniq.begin(), uniq.end());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
    ptet.resize(keys.size());
    for (size_t s = 0; s < keys.size(); s++)
        ptet[s] = (int)(std::lower_bound(uniq.begin(), uniq.end(), keys[s]) - uniq.begin());
    pkeys.clear();
    for (const auto &k : uniq) pkeys.insert(pkeys.end(), k.begin(), k.end());
    return (int)uniq.size();
}

}  // namespace

void build_stokes(const Discretization &d, Csr &B, Csr &Mp, std::vector<int32_t> &pkeys)
{
    const int k = d.k;
    if (k < 2 || k > 4) throw std::invalid_argument("the Stokes blocks are built for orders 2, 3 and 4");
    const int nt = d.nt, nl = d.nloc, n = d.ndof, nlp = (int)multi_indices(k - 1).size() / 4;
    std::vector<double> C, Mref;
    stokes_tables(k, C, Mref);
    std::vector<int> ptet;
    const int np = pressure_nodes(d, k - 1, ptet, pkeys);

    // scalar coupling pattern (pressure nodes x dofs), then B with the three
    // component blocks side by side in every row
    Csr S;
    coupling_pattern(np, n, nt, nlp, ptet.data(), nl, d.tet_dof.data(), S);
    B.n = np;
    B.m = 3 * n;
    B.ptr.assign((size_t)np + 1, 0);
    B.col.resize((size_t)3 * S.col.size());
    for (int p = 0; p < np; p++) {
        const int len = S.ptr[p + 1] - S.ptr[p];
        for (int c = 0; c < 3; c++)
            for (int e = 0; e < len; e++) B.col[(size_t)3 * S.ptr[p] + (size_t)c * len + e] = c * n + S.col[S.ptr[p] + e];
        B.ptr[p + 1] = 3 * S.ptr[p + 1];
    }
    B.val.assign(B.col.size(), 0.0);
    coupling_pattern(np, np, nt, nlp, ptet.data(), nlp, ptet.data(), Mp);

    for (int t = 0; t < nt; t++) {
        const int *v = &d.tets[4 * (size_t)t];
        double g[4][3];
        const double vol = std::fabs(tet_gradients(&d.xyz[3 * (size_t)v[0]], &d.xyz[3 * (size_t)v[1]],
                                                   &d.xyz[3 * (size_t)v[2]], &d.xyz[3 * (size_t)v[3]], g)) / 6.0;
        for (int p = 0; p < nlp; p++) {
            const int row = ptet[(size_t)t * nlp + p], len = S.ptr[row + 1] - S.ptr[row];
            for (int a = 0; a < nl; a++) {
                const int i = d.tet_dof[(size_t)t * nl + a];
                if (i < 0) continue;
                const int e = entry(S, row, i) - S.ptr[row];   // offset within each component block
                for (int c = 0; c < 3; c++) {
                    double s = 0.0;
                    for (int q = 0; q < 4; q++) s += g[q][c] * C[((size_t)q * nl + a) * nlp + p];
                    B.val[(size_t)3 * S.ptr[row] + (size_t)c * len + e] -= vol * s;
                }
            }
            for (int r = 0; r < nlp; r++)
                Mp.val[entry(Mp, row, ptet[(size_t)t * nlp + r])] += vol * Mref[(size_t)p * nlp + r];
        }
    }
}

}  // namespace auxp
