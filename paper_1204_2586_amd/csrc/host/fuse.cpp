// Composite operators that let the device evaluate the preconditioner with
// fewer passes (host, once per setup).
//
// The V(1,1) cycle on level l, from a zero guess, is a fixed linear map.
// With D = diag(l1 norms):
//   down:  x = D^-1 b,  r = b - A x,  b' = P^T r     =>  b' = M b,
//          M = P^T (I - A D^-1)
//   up:    x += P e,    y = x + D^-1 (b - A x)       =>  y = N b + Q e,
//          N = 2 D^-1 - D^-1 A D^-1,  Q = P - D^-1 A P
// so each level takes two passes (down, up) instead of four.  At the P^k
// level the residual is only ever restricted:
//   b_0 = I_R (r - A_h z) = I_R r - (I_R A_h) z,
// and I_R A_h has far fewer entries than A_h (a quarter for P2, an eighth
// for P3).  A pass that reads two vectors uses one operator whose columns are
// those of the two blocks side by side ([N Q] on [b; e], [I_R  -I_R A_h] on
// [r; z]).  Products are formed exactly in FP64 (the FP32 copies round the
// composite entries once); only the summation order of the cycle changes.
#include <algorithm>
#include <cstdint>
#include <stdexcept>

#include "parallel.hpp"
#include "setup.hpp"

namespace auxp {

namespace {

// C = A B (Gustavson, dense accumulator per row, columns sorted).  Rows are
// independent: contiguous row ranges go to worker threads, each summing its
// rows in the sequential order, and the ranges are concatenated.
Csr multiply(const Csr &A, const Csr &B)
{
    if (A.m != B.n) throw std::invalid_argument("multiply: shape mismatch");
    Csr C;
    C.n = A.n;
    C.m = B.m;
    C.ptr.assign((size_t)A.n + 1, 0);
    int64_t work = 0;
    for (int i = 0; i < A.n; i++)
        for (int e = A.ptr[i]; e < A.ptr[i + 1]; e++) work += B.ptr[A.col[e] + 1] - B.ptr[A.col[e]];
    const int nth = setup_threads((size_t)work);
    std::vector<std::vector<int>> cols_t(nth);
    std::vector<std::vector<double>> vals_t(nth);
    run_tasks(nth, [&](int w) {
        const int r0 = (int)((long long)A.n * w / nth), r1 = (int)((long long)A.n * (w + 1) / nth);
        std::vector<double> acc((size_t)B.m, 0.0);
        std::vector<int> mark((size_t)B.m, -1), cols;
        std::vector<int> &oc = cols_t[w];
        std::vector<double> &ov = vals_t[w];
        for (int i = r0; i < r1; i++) {
            cols.clear();
            for (int e = A.ptr[i]; e < A.ptr[i + 1]; e++) {
                const int k = A.col[e];
                const double a = A.val[e];
                for (int f = B.ptr[k]; f < B.ptr[k + 1]; f++) {
                    const int j = B.col[f];
                    if (mark[j] != i) {
                        mark[j] = i;
                        acc[j] = 0.0;
                        cols.push_back(j);
                    }
                    acc[j] += a * B.val[f];
                }
            }
            std::sort(cols.begin(), cols.end());
            for (int j : cols) {
                oc.push_back(j);
                ov.push_back(acc[j]);
            }
            C.ptr[i + 1] = (int)cols.size();
        }
    });
    for (int i = 0; i < A.n; i++) C.ptr[i + 1] += C.ptr[i];
    C.col.reserve(C.ptr[A.n]);
    C.val.reserve(C.ptr[A.n]);
    for (int w = 0; w < nth; w++) {
        C.col.insert(C.col.end(), cols_t[w].begin(), cols_t[w].end());
        C.val.insert(C.val.end(), vals_t[w].begin(), vals_t[w].end());
    }
    return C;
}

// a A + b B (same shape), union pattern
Csr combine(double a, const Csr &A, double b, const Csr &B)
{
    if (A.n != B.n || A.m != B.m) throw std::invalid_argument("combine: shape mismatch");
    Csr C;
    C.n = A.n;
    C.m = A.m;
    C.ptr.assign((size_t)A.n + 1, 0);
    for (int i = 0; i < A.n; i++) {
        int e = A.ptr[i], f = B.ptr[i];
        while (e < A.ptr[i + 1] || f < B.ptr[i + 1]) {
            const int ca = e < A.ptr[i + 1] ? A.col[e] : INT32_MAX;
            const int cb = f < B.ptr[i + 1] ? B.col[f] : INT32_MAX;
            const int c = std::min(ca, cb);
            double v = 0.0;
            if (ca == c) v += a * A.val[e++];
            if (cb == c) v += b * B.val[f++];
            C.col.push_back(c);
            C.val.push_back(v);
        }
        C.ptr[i + 1] = (int)C.col.size();
    }
    return C;
}

// diag(left) A diag(right); either may be null
Csr scale(const Csr &A, const std::vector<double> *left, const std::vector<double> *right)
{
    Csr C = A;
    for (int i = 0; i < A.n; i++)
        for (int e = A.ptr[i]; e < A.ptr[i + 1]; e++) {
            if (left) C.val[e] *= (*left)[i];
            if (right) C.val[e] *= (*right)[A.col[e]];
        }
    return C;
}

Csr diagonal(const std::vector<double> &d)
{
    Csr D;
    D.n = D.m = (int)d.size();
    D.ptr.resize(d.size() + 1);
    for (size_t i = 0; i < d.size(); i++) {
        D.ptr[i + 1] = (int)i + 1;
        D.col.push_back((int)i);
        D.val.push_back(d[i]);
    }
    return D;
}

// [A B]: the columns of B follow those of A
Csr side_by_side(const Csr &A, const Csr &B)
{
    if (A.n != B.n) throw std::invalid_argument("side_by_side: row mismatch");
    Csr C;
    C.n = A.n;
    C.m = A.m + B.m;
    C.ptr.assign((size_t)A.n + 1, 0);
    for (int i = 0; i < A.n; i++) {
        for (int e = A.ptr[i]; e < A.ptr[i + 1]; e++) {
            C.col.push_back(A.col[e]);
            C.val.push_back(A.val[e]);
        }
        for (int f = B.ptr[i]; f < B.ptr[i + 1]; f++) {
            C.col.push_back(A.m + B.col[f]);
            C.val.push_back(B.val[f]);
        }
        C.ptr[i + 1] = (int)C.col.size();
    }
    return C;
}

std::vector<double> inverse_of(const std::vector<double> &v)
{
    std::vector<double> r(v.size());
    for (size_t i = 0; i < v.size(); i++) r[i] = 1.0 / v[i];
    return r;
}

}  // namespace

FusedLevel fuse_level(const AmgLevel &L)
{
    const std::vector<double> dinv = inverse_of(L.l1);
    FusedLevel f;
    // M = P^T - P^T A D^-1
    f.down = combine(1.0, L.R, -1.0, scale(multiply(L.R, L.A), nullptr, &dinv));
    // N = 2 D^-1 - D^-1 A D^-1,  Q = P - D^-1 A P
    std::vector<double> two(dinv);
    for (double &v : two) v *= 2.0;
    Csr N = combine(1.0, diagonal(two), -1.0, scale(L.A, &dinv, &dinv));
    Csr Q = combine(1.0, L.P, -1.0, scale(multiply(L.A, L.P), &dinv, nullptr));
    f.up = side_by_side(N, Q);
    return f;
}

Csr fuse_restriction(const Csr &IR, const Csr &A)
{
    Csr C = multiply(IR, A);
    for (double &v : C.val) v = -v;
    return side_by_side(IR, C);
}

std::vector<double> dense_cycle(const std::vector<FusedLevel> &fused, const Hierarchy &H, size_t l0)
{
    const size_t L = H.levels.size();
    if (L == 0 || l0 >= L) throw std::invalid_argument("dense_cycle: level out of range");
    std::vector<double> T = H.coarse_inv;        // nc x nc on the coarsest level
    for (size_t l = L - 1; l-- > l0;) {
        const int n = H.levels[l].A.n, nc = H.levels[l + 1].A.n;
        const Csr &M = fused[l].down, &U = fused[l].up;
        if (M.n != nc || M.m != n || U.n != n || U.m != n + nc)
            throw std::invalid_argument("dense_cycle: operator shapes");
        // Tn = N + (Q T) M, rows of U split at column n into N and Q
        std::vector<double> Tn((size_t)n * n, 0.0), QT((size_t)nc);
        for (int i = 0; i < n; i++) {
            double *row = &Tn[(size_t)i * n];
            std::fill(QT.begin(), QT.end(), 0.0);
            for (int e = U.ptr[i]; e < U.ptr[i + 1]; e++) {
                const int c = U.col[e];
                if (c < n) {
                    row[c] += U.val[e];
                } else {
                    const double q = U.val[e];
                    const double *tr = &T[(size_t)(c - n) * nc];
                    for (int k = 0; k < nc; k++) QT[k] += q * tr[k];
                }
            }
            for (int k = 0; k < nc; k++) {
                const double a = QT[k];
                if (a == 0.0) continue;
                for (int e = M.ptr[k]; e < M.ptr[k + 1]; e++) row[M.col[e]] += a * M.val[e];
            }
        }
        T.swap(Tn);
    }
    return T;
}

}  // namespace auxp
