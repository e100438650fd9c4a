// AMG setup on the auxiliary P^1 matrix A_H.
//
// The paper solves the P^1 problem (Step 1 of Algorithm 2.1) with BoomerAMG
// using PMIS coarsening and extended+i interpolation (Sec. 1, Sec. 6.1), with
// the strength rule of Sec. 6.2: i depends strongly on j when
// -a_ij > theta * max_{k != i} (-a_ik).  The published methods are:
//  * PMIS (De Sterck, Yang, Heys 2006): measure |S_i^T| + random; points that
//    influence nobody are F; in synchronous rounds, undecided points whose
//    measure beats all undecided strong neighbours become C, and undecided
//    points that depend strongly on a new C point become F;
//  * extended+i interpolation (De Sterck, Falgout, Nolting, Yang 2008) over
//    the distance-two set hat C_i = (S_i cap C) cup (S_k cap C, k in S_i cap F);
//  * Galerkin coarse operators A_{l+1} = P^T A_l P.
// Readings where the paper is silent: strict '>' with ties (equal up to a
// relative 1e-12 of the row maximum) not strong; the random part of the
// measure is the splitmix64 output of (splitmix64(seed) + level*2^32 + i),
// compared as an integer after |S_i^T|, and the lower index wins a full tie;
// no "+cc" restriction and no truncation; coarsening stops at <= coarse_max
// rows, when a level does not shrink, or at max_levels.  The coarsest level is
// inverted exactly (dense Cholesky, explicit inverse).
#include <algorithm>
#include <cmath>
#include <stdexcept>

#include "setup.hpp"

namespace auxp {

namespace {

uint64_t splitmix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

struct Pattern {
    std::vector<int> ptr, col;
};

Pattern strong_dependencies(const Csr &A, double theta)
{
    Pattern S;
    S.ptr.assign((size_t)A.n + 1, 0);
    for (int i = 0; i < A.n; i++) {
        double mx = 0.0;
        bool any = false;
        for (int e = A.ptr[i]; e < A.ptr[i + 1]; e++)
            if (A.col[e] != i && (!any || -A.val[e] > mx)) {
                mx = -A.val[e];
                any = true;
            }
        if (any && mx > 0.0) {
            double cut = mx * (theta + 1e-12);
            for (int e = A.ptr[i]; e < A.ptr[i + 1]; e++)
                if (A.col[e] != i && -A.val[e] > cut) S.col.push_back(A.col[e]);
        }
        S.ptr[i + 1] = (int)S.col.size();
    }
    return S;
}

Pattern transpose_pattern(const Pattern &S, int n)
{
    Pattern T;
    T.ptr.assign((size_t)n + 1, 0);
    for (int j : S.col) T.ptr[j + 1]++;
    for (int i = 0; i < n; i++) T.ptr[i + 1] += T.ptr[i];
    T.col.resize(S.col.size());
    std::vector<int> fill(T.ptr.begin(), T.ptr.end() - 1);
    for (int i = 0; i < n; i++)
        for (int e = S.ptr[i]; e < S.ptr[i + 1]; e++) T.col[fill[S.col[e]]++] = i;
    return T;
}

std::vector<int> pmis_split(const Pattern &S, const Pattern &ST, int n, uint64_t seed, int level)
{
    std::vector<int> infl(n);
    std::vector<uint64_t> rnd(n);
    uint64_t base = splitmix64(seed) + ((uint64_t)level << 32);
    std::vector<int> cf(n, 0), undecided;
    for (int i = 0; i < n; i++) {
        infl[i] = ST.ptr[i + 1] - ST.ptr[i];
        rnd[i] = splitmix64(base + (uint64_t)i);
        if (infl[i] == 0) cf[i] = -1;
        else undecided.push_back(i);
    }
    auto wins = [&](int i, int j) {   // does i's measure exceed j's?
        if (infl[i] != infl[j]) return infl[i] > infl[j];
        if (rnd[i] != rnd[j]) return rnd[i] > rnd[j];
        return i < j;
    };
    std::vector<char> newC(n, 0);
    std::vector<int> sel;
    while (!undecided.empty()) {
        sel.clear();
        for (int i : undecided) {
            bool best = true;
            for (int e = S.ptr[i]; best && e < S.ptr[i + 1]; e++)
                if (cf[S.col[e]] == 0 && !wins(i, S.col[e])) best = false;
            for (int e = ST.ptr[i]; best && e < ST.ptr[i + 1]; e++)
                if (cf[ST.col[e]] == 0 && !wins(i, ST.col[e])) best = false;
            if (best) sel.push_back(i);
        }
        for (int i : sel) newC[i] = 1;
        for (int i : sel) cf[i] = 1;
        std::vector<int> rest;
        for (int i : undecided) {
            if (cf[i] != 0) continue;
            bool dep = false;
            for (int e = S.ptr[i]; !dep && e < S.ptr[i + 1]; e++) dep = newC[S.col[e]];
            if (dep) cf[i] = -1;
            else rest.push_back(i);
        }
        for (int i : sel) newC[i] = 0;
        undecided.swap(rest);
    }
    return cf;
}

Csr extended_i(const Csr &A, const Pattern &S, const std::vector<int> &cf, int &nc)
{
    int n = A.n;
    std::vector<int> cnum(n, -1);
    nc = 0;
    for (int i = 0; i < n; i++)
        if (cf[i] > 0) cnum[i] = nc++;
    std::vector<double> diag(n, 0.0);
    for (int i = 0; i < n; i++)
        for (int e = A.ptr[i]; e < A.ptr[i + 1]; e++)
            if (A.col[e] == i) diag[i] += A.val[e];

    Csr P;
    P.n = n;
    P.m = nc;
    P.ptr.assign((size_t)n + 1, 0);
    std::vector<int> hatc_owner(n, -1), strongF_owner(n, -1);
    std::vector<double> w(n, 0.0);
    std::vector<int> hat;
    for (int i = 0; i < n; i++) {
        if (cf[i] > 0) {
            P.col.push_back(cnum[i]);
            P.val.push_back(1.0);
            P.ptr[i + 1] = (int)P.col.size();
            continue;
        }
        hat.clear();
        for (int e = S.ptr[i]; e < S.ptr[i + 1]; e++) {
            int j = S.col[e];
            if (cf[j] > 0) {
                if (hatc_owner[j] != i) {
                    hatc_owner[j] = i;
                    hat.push_back(j);
                }
            } else {
                strongF_owner[j] = i;
                for (int f = S.ptr[j]; f < S.ptr[j + 1]; f++) {
                    int l = S.col[f];
                    if (cf[l] > 0 && hatc_owner[l] != i) {
                        hatc_owner[l] = i;
                        hat.push_back(l);
                    }
                }
            }
        }
        for (int j : hat) w[j] = 0.0;
        double dii = diag[i];
        for (int e = A.ptr[i]; e < A.ptr[i + 1]; e++) {
            int j = A.col[e];
            if (j == i) continue;
            double aij = A.val[e];
            if (hatc_owner[j] == i) {
                w[j] += aij;
            } else if (strongF_owner[j] == i) {
                // distribute a_ij over hat C_i and i with the entries of row j
                // whose sign is opposite to its diagonal
                double dj = diag[j], den = 0.0;
                for (int f = A.ptr[j]; f < A.ptr[j + 1]; f++) {
                    int l = A.col[f];
                    if ((l == i || hatc_owner[l] == i) && A.val[f] * dj < 0.0) den += A.val[f];
                }
                if (den == 0.0) {
                    dii += aij;
                    continue;
                }
                double scale = aij / den;
                for (int f = A.ptr[j]; f < A.ptr[j + 1]; f++) {
                    int l = A.col[f];
                    if (A.val[f] * dj >= 0.0) continue;
                    if (l == i) dii += scale * A.val[f];
                    else if (hatc_owner[l] == i) w[l] += scale * A.val[f];
                }
            } else {
                dii += aij;   // weak connection lumped onto the diagonal
            }
        }
        std::sort(hat.begin(), hat.end());
        for (int j : hat) {
            P.col.push_back(cnum[j]);
            P.val.push_back(-w[j] / dii);
        }
        P.ptr[i + 1] = (int)P.col.size();
    }
    return P;
}

// C = A B (Gustavson with a dense row accumulator)
Csr spgemm(const Csr &A, const Csr &B)
{
    Csr C;
    C.n = A.n;
    C.m = B.m;
    C.ptr.assign((size_t)A.n + 1, 0);
    std::vector<int> pos(B.m, -1), cols;
    std::vector<double> acc;
    for (int i = 0; i < A.n; i++) {
        cols.clear();
        acc.clear();
        for (int e = A.ptr[i]; e < A.ptr[i + 1]; e++) {
            int k = A.col[e];
            double a = A.val[e];
            for (int f = B.ptr[k]; f < B.ptr[k + 1]; f++) {
                int j = B.col[f];
                if (pos[j] < 0) {
                    pos[j] = (int)cols.size();
                    cols.push_back(j);
                    acc.push_back(a * B.val[f]);
                } else {
                    acc[pos[j]] += a * B.val[f];
                }
            }
        }
        std::vector<int> order(cols.size());
        for (size_t s = 0; s < order.size(); s++) order[s] = (int)s;
        std::sort(order.begin(), order.end(), [&](int x, int y) { return cols[x] < cols[y]; });
        for (int s : order) {
            C.col.push_back(cols[s]);
            C.val.push_back(acc[s]);
        }
        for (int j : cols) pos[j] = -1;
        C.ptr[i + 1] = (int)C.col.size();
    }
    return C;
}

std::vector<double> dense_inverse_spd(const Csr &A)
{
    int n = A.n;
    std::vector<double> L((size_t)n * n, 0.0);
    for (int i = 0; i < n; i++)
        for (int e = A.ptr[i]; e < A.ptr[i + 1]; e++) L[(size_t)i * n + A.col[e]] = A.val[e];
    for (int j = 0; j < n; j++) {
        double d = L[(size_t)j * n + j];
        for (int p = 0; p < j; p++) d -= L[(size_t)j * n + p] * L[(size_t)j * n + p];
        if (!(d > 0.0)) throw std::runtime_error("coarsest AMG operator is not positive definite");
        d = std::sqrt(d);
        L[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; i++) {
            double s = L[(size_t)i * n + j];
            for (int p = 0; p < j; p++) s -= L[(size_t)i * n + p] * L[(size_t)j * n + p];
            L[(size_t)i * n + j] = s / d;
        }
    }
    // columns of A^{-1} by forward and backward substitution
    std::vector<double> inv((size_t)n * n, 0.0), y(n);
    for (int c = 0; c < n; c++) {
        for (int i = 0; i < n; i++) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int p = 0; p < i; p++) s -= L[(size_t)i * n + p] * y[p];
            y[i] = s / L[(size_t)i * n + i];
        }
        for (int i = n - 1; i >= 0; i--) {
            double s = y[i];
            for (int p = i + 1; p < n; p++) s -= L[(size_t)p * n + i] * y[p];
            y[i] = s / L[(size_t)i * n + i];
        }
        for (int i = 0; i < n; i++) inv[(size_t)i * n + c] = y[i];
    }
    // symmetrise the rounding
    for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++) {
            double s = 0.5 * (inv[(size_t)i * n + j] + inv[(size_t)j * n + i]);
            inv[(size_t)i * n + j] = inv[(size_t)j * n + i] = s;
        }
    return inv;
}

std::vector<double> l1_norms(const Csr &A)
{
    std::vector<double> d(A.n, 0.0);
    for (int i = 0; i < A.n; i++)
        for (int e = A.ptr[i]; e < A.ptr[i + 1]; e++) d[i] += std::fabs(A.val[e]);
    return d;
}

}  // namespace

void build_hierarchy(const Csr &AH, const SetupOptions &opt, Hierarchy &h)
{
    h.levels.clear();
    h.levels.emplace_back();
    h.levels[0].A = AH;
    for (int l = 0;; l++) {
        AmgLevel &lv = h.levels[l];
        lv.l1 = l1_norms(lv.A);
        int n = lv.A.n;
        if (n <= opt.coarse_max || l + 1 >= opt.max_levels) break;
        Pattern S = strong_dependencies(lv.A, opt.theta);
        Pattern ST = transpose_pattern(S, n);
        std::vector<int> cf = pmis_split(S, ST, n, opt.seed, l);
        int nc = 0;
        Csr P = extended_i(lv.A, S, cf, nc);
        if (nc == 0 || nc >= n) break;
        lv.cf = std::move(cf);
        lv.P = std::move(P);
        lv.R = transpose(lv.P);
        Csr Ac = spgemm(lv.R, spgemm(lv.A, lv.P));
        h.levels.emplace_back();
        h.levels.back().A = std::move(Ac);
    }
    const Csr &Ac = h.levels.back().A;
    if (Ac.n > 8192) throw std::runtime_error("coarsest AMG level too large for a dense solve");
    h.ncoarse = Ac.n;
    h.coarse_inv = dense_inverse_spd(Ac);
}

}  // namespace auxp
