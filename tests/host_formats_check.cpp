// Checks of two host-side builders of the library, compiled by
// tests/test_host_formats.py against the library's host sources:
//
//  * build_ell (row-split sliced ELL): the placement of every entry, the
//    padding, and the product a wavefront computes from the layout (emulated
//    lane by lane) against the CSR product;
//  * fuse_level + dense_cycle (the bottom of the V-cycle as one dense matrix)
//    against the V(1,1) cycle from a zero guess evaluated step by step
//    (x = D^-1 b, r = b - A x, b' = P^T r, recurse, x += P e,
//    y = x + D^-1 (b - A x); the coarsest level solved exactly), applied to
//    every unit vector.
//
// Prints "ell <lanes> <max relative error>" and "dense <levels> <max relative
// error>" lines; exits non-zero on a layout violation.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <numeric>
#include <random>
#include <vector>

#include "setup.hpp"

using namespace auxp;

namespace {

Csr random_csr(int n, int m, std::mt19937 &rng)
{
    Csr A;
    A.n = n;
    A.m = m;
    A.ptr.assign(n + 1, 0);
    std::uniform_int_distribution<int> len(0, 40), colu(0, m - 1);
    std::uniform_real_distribution<double> v(-1.0, 1.0);
    for (int i = 0; i < n; i++) {
        int L = (i % 7 == 3) ? 0 : len(rng);               // some empty rows
        for (int k = 0; k < L; k++) {
            A.col.push_back(colu(rng));
            A.val.push_back(v(rng));
        }
        A.ptr[i + 1] = (int)A.col.size();
    }
    return A;
}

int check_ell(const Csr &A, int lanes, double &err)
{
    Ell e;
    build_ell(A, lanes, e);
    const int rows = 64 / lanes;
    if (e.nslices != (A.n + rows - 1) / rows) return 1;
    for (int s = 0; s <= e.nslices; s++)
        if (e.slice_off[s] % 64) return 2;
    std::vector<double> x(A.m);
    for (int j = 0; j < A.m; j++) x[j] = std::sin(0.37 * j + 0.1);
    err = 0.0;
    for (int s = 0; s < e.nslices; s++) {
        const int width = (e.slice_off[s + 1] - e.slice_off[s]) / 64;
        std::vector<double> lane_acc(64, 0.0);
        for (int t = 0; t < width; t++)
            for (int l = 0; l < 64; l++) {
                const size_t at = (size_t)e.slice_off[s] + (size_t)t * 64 + l;
                if (e.col[at] < 0 || e.col[at] >= A.m) return 3;
                lane_acc[l] += e.val[at] * x[e.col[at]];
                // placement: entry k = t * lanes + l % lanes of row l / lanes
                const int row = s * rows + l / lanes, k = t * lanes + l % lanes;
                const bool real = row < A.n && k < A.ptr[row + 1] - A.ptr[row];
                if (real) {
                    if (e.col[at] != A.col[A.ptr[row] + k] || e.val[at] != A.val[A.ptr[row] + k]) return 4;
                } else if (e.val[at] != 0.0) {
                    return 5;
                }
            }
        for (int q = 0; q < rows; q++) {
            const int row = s * rows + q;
            if (row >= A.n) break;
            double y = 0.0, ref = 0.0, mag = 0.0;
            for (int l = q * lanes; l < (q + 1) * lanes; l++) y += lane_acc[l];
            for (int p = A.ptr[row]; p < A.ptr[row + 1]; p++) {
                ref += A.val[p] * x[A.col[p]];
                mag += std::fabs(A.val[p] * x[A.col[p]]);
            }
            if (mag > 0) err = std::max(err, std::fabs(y - ref) / mag);
            else if (y != 0.0) return 6;
        }
    }
    return 0;
}

Csr dense_to_csr(const std::vector<double> &M, int n, int m)
{
    Csr C;
    C.n = n;
    C.m = m;
    C.ptr.assign(n + 1, 0);
    for (int i = 0; i < n; i++) {
        for (int j = 0; j < m; j++)
            if (M[(size_t)i * m + j] != 0.0) {
                C.col.push_back(j);
                C.val.push_back(M[(size_t)i * m + j]);
            }
        C.ptr[i + 1] = (int)C.col.size();
    }
    return C;
}

std::vector<double> csr_to_dense(const Csr &C)
{
    std::vector<double> M((size_t)C.n * C.m, 0.0);
    for (int i = 0; i < C.n; i++)
        for (int p = C.ptr[i]; p < C.ptr[i + 1]; p++) M[(size_t)i * C.m + C.col[p]] += C.val[p];
    return M;
}

std::vector<double> matmul(const std::vector<double> &A, const std::vector<double> &B, int n, int k, int m)
{
    std::vector<double> C((size_t)n * m, 0.0);
    for (int i = 0; i < n; i++)
        for (int l = 0; l < k; l++)
            for (int j = 0; j < m; j++) C[(size_t)i * m + j] += A[(size_t)i * k + l] * B[(size_t)l * m + j];
    return C;
}

std::vector<double> transpose(const std::vector<double> &A, int n, int m)
{
    std::vector<double> T((size_t)m * n);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < m; j++) T[(size_t)j * n + i] = A[(size_t)i * m + j];
    return T;
}

std::vector<double> inverse(std::vector<double> A, int n)
{
    std::vector<double> I((size_t)n * n, 0.0);
    for (int i = 0; i < n; i++) I[(size_t)i * n + i] = 1.0;
    for (int c = 0; c < n; c++) {
        int p = c;
        for (int r = c + 1; r < n; r++)
            if (std::fabs(A[(size_t)r * n + c]) > std::fabs(A[(size_t)p * n + c])) p = r;
        for (int j = 0; j < n; j++) {
            std::swap(A[(size_t)c * n + j], A[(size_t)p * n + j]);
            std::swap(I[(size_t)c * n + j], I[(size_t)p * n + j]);
        }
        const double d = A[(size_t)c * n + c];
        for (int j = 0; j < n; j++) {
            A[(size_t)c * n + j] /= d;
            I[(size_t)c * n + j] /= d;
        }
        for (int r = 0; r < n; r++)
            if (r != c) {
                const double f = A[(size_t)r * n + c];
                for (int j = 0; j < n; j++) {
                    A[(size_t)r * n + j] -= f * A[(size_t)c * n + j];
                    I[(size_t)r * n + j] -= f * I[(size_t)c * n + j];
                }
            }
    }
    return I;
}

// linear interpolation from every second point: coarse point c sits at fine
// point 2c + 1 (fine n = 2 nc + 1)
std::vector<double> interpolation(int nc)
{
    const int n = 2 * nc + 1;
    std::vector<double> P((size_t)n * nc, 0.0);
    for (int c = 0; c < nc; c++) {
        P[(size_t)(2 * c + 1) * nc + c] = 1.0;
        P[(size_t)(2 * c) * nc + c] += 0.5;
        P[(size_t)(2 * c + 2) * nc + c] += 0.5;
    }
    return P;
}

// y = cycle(l) b, evaluated step by step
std::vector<double> cycle(const std::vector<std::vector<double>> &A, const std::vector<std::vector<double>> &P,
                          const std::vector<int> &n, const std::vector<double> &cinv, size_t l,
                          const std::vector<double> &b)
{
    const int nl = n[l];
    if (l + 1 == n.size()) {
        std::vector<double> x(nl, 0.0);
        for (int i = 0; i < nl; i++)
            for (int j = 0; j < nl; j++) x[i] += cinv[(size_t)i * nl + j] * b[j];
        return x;
    }
    const int nc = n[l + 1];
    std::vector<double> d(nl, 0.0), x(nl), r(nl), bc(nc, 0.0);
    for (int i = 0; i < nl; i++)
        for (int j = 0; j < nl; j++) d[i] += std::fabs(A[l][(size_t)i * nl + j]);
    for (int i = 0; i < nl; i++) x[i] = b[i] / d[i];
    for (int i = 0; i < nl; i++) {
        double s = b[i];
        for (int j = 0; j < nl; j++) s -= A[l][(size_t)i * nl + j] * x[j];
        r[i] = s;
    }
    for (int c = 0; c < nc; c++)
        for (int i = 0; i < nl; i++) bc[c] += P[l][(size_t)i * nc + c] * r[i];
    const std::vector<double> e = cycle(A, P, n, cinv, l + 1, bc);
    for (int i = 0; i < nl; i++)
        for (int c = 0; c < nc; c++) x[i] += P[l][(size_t)i * nc + c] * e[c];
    std::vector<double> y(nl);
    for (int i = 0; i < nl; i++) {
        double s = b[i];
        for (int j = 0; j < nl; j++) s -= A[l][(size_t)i * nl + j] * x[j];
        y[i] = x[i] + s / d[i];
    }
    return y;
}

double check_dense(int nlev)
{
    // 1D Laplacian with a variable coefficient on the finest level
    std::vector<int> n(nlev);
    n[nlev - 1] = 3;
    for (int l = nlev - 2; l >= 0; l--) n[l] = 2 * n[l + 1] + 1;
    std::vector<std::vector<double>> A(nlev), P(nlev);
    A[0].assign((size_t)n[0] * n[0], 0.0);
    for (int i = 0; i < n[0]; i++) {
        const double a = 1.0 + 0.5 * std::sin(0.7 * i), c = 1.0 + 0.5 * std::sin(0.7 * (i + 1));
        A[0][(size_t)i * n[0] + i] = a + c;
        if (i > 0) A[0][(size_t)i * n[0] + i - 1] = -a;
        if (i + 1 < n[0]) A[0][(size_t)i * n[0] + i + 1] = -c;
    }
    Hierarchy H;
    H.levels.resize(nlev);
    for (int l = 0; l < nlev; l++) {
        AmgLevel &L = H.levels[l];
        L.A = dense_to_csr(A[l], n[l], n[l]);
        L.l1.assign(n[l], 0.0);
        for (int i = 0; i < n[l]; i++)
            for (int j = 0; j < n[l]; j++) L.l1[i] += std::fabs(A[l][(size_t)i * n[l] + j]);
        if (l + 1 < nlev) {
            P[l] = interpolation(n[l + 1]);
            L.P = dense_to_csr(P[l], n[l], n[l + 1]);
            L.R = dense_to_csr(transpose(P[l], n[l], n[l + 1]), n[l + 1], n[l]);
            A[l + 1] = matmul(matmul(transpose(P[l], n[l], n[l + 1]), A[l], n[l + 1], n[l], n[l]), P[l], n[l + 1],
                              n[l], n[l + 1]);
        }
    }
    H.coarse_inv = inverse(A[nlev - 1], n[nlev - 1]);
    H.ncoarse = n[nlev - 1];
    std::vector<FusedLevel> fused(nlev);
    for (int l = 0; l + 1 < nlev; l++) fused[l] = fuse_level(H.levels[l]);
    const std::vector<double> T = dense_cycle(fused, H, 0);
    double err = 0.0, mag = 0.0;
    for (int j = 0; j < n[0]; j++) {
        std::vector<double> b(n[0], 0.0);
        b[j] = 1.0;
        const std::vector<double> y = cycle(A, P, n, H.coarse_inv, 0, b);
        for (int i = 0; i < n[0]; i++) {
            err = std::max(err, std::fabs(T[(size_t)i * n[0] + j] - y[i]));
            mag = std::max(mag, std::fabs(y[i]));
        }
    }
    return err / mag;
}

// Morton order: a permutation whose codes (interleaved bits, computed here
// bit by bit) never decrease; on a 2^k lattice every aligned run of 8^j points
// is a 2^j cube (the Z-order property)
int check_morton(int k)
{
    const int m = 1 << k, n = m * m * m;
    std::vector<double> xyz((size_t)3 * n);
    std::vector<int> ijk((size_t)3 * n);
    for (int p = 0; p < n; p++) {
        const int i = p % m, j = (p / m) % m, l = p / (m * m);
        ijk[3 * p] = i;
        ijk[3 * p + 1] = j;
        ijk[3 * p + 2] = l;
        xyz[3 * p] = i;
        xyz[3 * p + 1] = j;
        xyz[3 * p + 2] = l;
    }
    const std::vector<int> ord = morton_order(xyz, n);
    std::vector<int> seen(n, 0);
    for (int r = 0; r < n; r++) {
        if (ord[r] < 0 || ord[r] >= n || seen[ord[r]]++) return 1;
    }
    // bits of the quantised coordinates: the bounding box is [0, m-1], so
    // coordinate c maps to round(c * (2^21 - 1) / (m - 1))
    auto code = [&](int p) {
        unsigned long long q[3], z = 0;
        for (int c = 0; c < 3; c++)
            q[c] = (unsigned long long)std::floor((double)ijk[3 * p + c] / (m - 1) * 2097151.0 + 0.5);
        for (int b = 0; b < 21; b++)
            for (int c = 0; c < 3; c++) z |= ((q[c] >> b) & 1ULL) << (3 * b + c);
        return z;
    };
    for (int r = 1; r < n; r++)
        if (code(ord[r]) < code(ord[r - 1])) return 2;
    for (int j = 1; j < k && j <= 2; j++) {
        const int run = 1 << (3 * j), side = 1 << j;
        for (int r0 = 0; r0 < n; r0 += run) {
            int lo[3] = {m, m, m}, hi[3] = {-1, -1, -1};
            for (int r = r0; r < r0 + run; r++)
                for (int c = 0; c < 3; c++) {
                    lo[c] = std::min(lo[c], ijk[3 * ord[r] + c]);
                    hi[c] = std::max(hi[c], ijk[3 * ord[r] + c]);
                }
            for (int c = 0; c < 3; c++)
                if (hi[c] - lo[c] != side - 1) return 3;
        }
    }
    return 0;
}

// renumber_cols against a dense reference: a random n x 2h matrix whose
// columns below h and from h on are renumbered by one permutation of h
double check_renumber(int n, int h, std::mt19937 &rng)
{
    const int m = 2 * h;
    Csr B;
    B.n = n;
    B.m = m;
    B.ptr.assign((size_t)n + 1, 0);
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    for (int i = 0; i < n; i++) {
        for (int j = 0; j < m; j++)
            if (rng() % 5 == 0) {
                B.col.push_back(j);
                B.val.push_back(u(rng));
            }
        B.ptr[i + 1] = (int)B.col.size();
    }
    std::vector<int> map(h);
    std::iota(map.begin(), map.end(), 0);
    std::shuffle(map.begin(), map.end(), rng);
    const Csr R = renumber_cols(B, map, h);
    std::vector<double> dense((size_t)n * m, 0.0), got((size_t)n * m, 0.0);
    for (int i = 0; i < n; i++) {
        for (int e = B.ptr[i]; e < B.ptr[i + 1]; e++) {
            const int j = B.col[e];
            dense[(size_t)i * m + (j < h ? map[j] : h + map[j - h])] = B.val[e];
        }
        for (int e = R.ptr[i]; e < R.ptr[i + 1]; e++) {
            if (e > R.ptr[i] && R.col[e] <= R.col[e - 1]) return 1e300;   // sorted, no repeats
            got[(size_t)i * m + R.col[e]] = R.val[e];
        }
    }
    double err = 0.0;
    for (size_t q = 0; q < dense.size(); q++) err = std::max(err, std::fabs(dense[q] - got[q]));
    return err;
}

}  // namespace

int main()
{
    std::mt19937 rng(12345);
    for (int lanes : {1, 2, 4, 8, 16, 32}) {
        for (int n : {1, 63, 130, 517}) {
            const Csr A = random_csr(n, 97, rng);
            double err = 0.0;
            const int bad = check_ell(A, lanes, err);
            if (bad) {
                std::printf("ell layout violation %d (lanes %d, rows %d)\n", bad, lanes, n);
                return 1;
            }
            std::printf("ell %d %.3e\n", lanes, err);
        }
    }
    for (int nlev : {2, 3, 4}) std::printf("dense %d %.3e\n", nlev, check_dense(nlev));
    for (int k : {1, 3, 4}) std::printf("morton %d %d\n", k, check_morton(k));
    for (int n : {2, 64, 130}) std::printf("renum %d %.3e\n", n, check_renumber(n, n / 2 + 1, rng));
    return 0;
}
