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
#include <cmath>
#include <cstdio>
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
    return 0;
}
