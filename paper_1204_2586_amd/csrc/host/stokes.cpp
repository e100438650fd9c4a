// Blocks of the Hood-Taylor P^2-P^1 discretisation of the Stokes system
// (Sec. 5: velocity in P^{2,0}, pressure in P^{1,0}, the stable pair of the
// paper's second test problem).  With the velocity test functions phi_i e_c
// and the pressure basis lam_p (hat functions on every vertex, no boundary
// condition on p):
//   B_{p, (c, i)} = -int_T lam_p dphi_i/dx_c,  M_p = int lam_p lam_q.
// Per tet, dphi_i/dx_c = sum_q (dphi_i/dlam_q) (grad lam_q)_c, so the element
// block is -|T| sum_q (grad lam_q)_c C[q][i][p] with the exact moment table
// C[q][i][p] = (1/|T|) int lam_p dphi_i/dlam_q, and the P^1 mass matrix is
// |T| (1 + delta_pq) / 20, both integrated exactly.
#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <vector>

#include "setup.hpp"

namespace auxp {

namespace {

// CSR pattern of rows over `nr` row ids from the per-tet row map rmap[nt][4]
// coupled with the per-tet column map cmap[nt][nl] (-1 = eliminated),
// columns sorted; values zero.
void coupling_pattern(int nr, int ncol, int nt, const int *rmap, int nl, const int *cmap, Csr &A)
{
    std::vector<int> cnt((size_t)nr + 1, 0);
    for (size_t s = 0; s < (size_t)nt * 4; s++) cnt[rmap[s] + 1]++;
    for (int i = 0; i < nr; i++) cnt[i + 1] += cnt[i];
    std::vector<int> inc(cnt.back()), fill(cnt.begin(), cnt.end() - 1);
    for (size_t s = 0; s < (size_t)nt * 4; s++) inc[fill[rmap[s]]++] = (int)(s / 4);
    A.n = nr;
    A.m = ncol;
    A.ptr.assign((size_t)nr + 1, 0);
    A.col.clear();
    std::vector<int> mark(ncol, -1), row;
    for (int i = 0; i < nr; i++) {
        row.clear();
        for (int e = cnt[i]; e < cnt[i + 1]; e++) {
            const int *cm = cmap + (size_t)inc[e] * nl;
            for (int b = 0; b < nl; b++) {
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

}  // namespace

void build_stokes(const Discretization &d, Csr &B, Csr &Mp)
{
    if (d.k != 2) throw std::invalid_argument("the Stokes blocks are built for order 2 (Hood-Taylor P2-P1) only");
    const int nt = d.nt, nv = d.nv, nl = d.nloc, n = d.ndof;
    const std::vector<double> C = coupling_tables(2);

    // scalar coupling pattern (vertices x dofs), then B with the three
    // component blocks side by side in every row
    Csr S;
    coupling_pattern(nv, n, nt, d.tets.data(), nl, d.tet_dof.data(), S);
    B.n = nv;
    B.m = 3 * n;
    B.ptr.assign((size_t)nv + 1, 0);
    B.col.resize((size_t)3 * S.col.size());
    for (int p = 0; p < nv; p++) {
        const int len = S.ptr[p + 1] - S.ptr[p];
        for (int c = 0; c < 3; c++)
            for (int e = 0; e < len; e++) B.col[(size_t)3 * S.ptr[p] + (size_t)c * len + e] = c * n + S.col[S.ptr[p] + e];
        B.ptr[p + 1] = 3 * S.ptr[p + 1];
    }
    B.val.assign(B.col.size(), 0.0);
    coupling_pattern(nv, nv, nt, d.tets.data(), 4, d.tets.data(), Mp);

    for (int t = 0; t < nt; t++) {
        const int *v = &d.tets[4 * (size_t)t];
        double g[4][3];
        const double vol = std::fabs(tet_gradients(&d.xyz[3 * (size_t)v[0]], &d.xyz[3 * (size_t)v[1]],
                                                   &d.xyz[3 * (size_t)v[2]], &d.xyz[3 * (size_t)v[3]], g)) / 6.0;
        for (int p = 0; p < 4; p++) {
            const int row = v[p], len = S.ptr[row + 1] - S.ptr[row];
            for (int a = 0; a < nl; a++) {
                const int i = d.tet_dof[(size_t)t * nl + a];
                if (i < 0) continue;
                const int e = entry(S, row, i) - S.ptr[row];   // offset within each component block
                for (int c = 0; c < 3; c++) {
                    double s = 0.0;
                    for (int q = 0; q < 4; q++) s += g[q][c] * C[((size_t)q * nl + a) * 4 + p];
                    B.val[(size_t)3 * S.ptr[row] + (size_t)c * len + e] -= vol * s;
                }
            }
            for (int q = 0; q < 4; q++) Mp.val[entry(Mp, row, v[q])] += vol * (p == q ? 0.1 : 0.05);
        }
    }
}

}  // namespace auxp
