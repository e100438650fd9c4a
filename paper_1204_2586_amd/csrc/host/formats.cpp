// Device storage formats built on the host (once per setup).
//
// Sliced ELLPACK for the P^k operator.  Rows keep the dof order (which is
// lexicographic in the vertex multisets, so neighbours along one mesh axis
// are adjacent in memory) except that within each window of `window`
// consecutive rows longer rows come first (stable): the rows of a slice then
// have nearly equal lengths.  Consecutive groups of `slice` rows form slices
// whose entries are stored column-major (entry j of the slice's rows is
// contiguous), padded to the slice's longest row with zero values pointing at
// column 0.
#include <algorithm>
#include <numeric>
#include <stdexcept>

#include "setup.hpp"

namespace auxp {

void build_sell(const Csr &A, int slice, int window, Sell &out)
{
    const int n = A.n;
    out.n = n;
    out.slice = slice;
    out.perm.resize(n);
    std::iota(out.perm.begin(), out.perm.end(), 0);
    auto len = [&](int i) { return A.ptr[i + 1] - A.ptr[i]; };
    for (int w0 = 0; w0 < n; w0 += window) {
        int w1 = std::min(n, w0 + window);
        std::stable_sort(out.perm.begin() + w0, out.perm.begin() + w1, [&](int a, int b) { return len(a) > len(b); });
    }
    out.iperm.assign(n, 0);
    for (int i = 0; i < n; i++) out.iperm[out.perm[i]] = i;
    out.nslices = (n + slice - 1) / slice;
    out.slice_off.assign((size_t)out.nslices + 1, 0);
    for (int s = 0; s < out.nslices; s++) {
        int w = 0;
        for (int r = s * slice; r < std::min(n, (s + 1) * slice); r++) w = std::max(w, len(out.perm[r]));
        int64_t next = (int64_t)out.slice_off[s] + (int64_t)w * slice;
        if (next > 0x7fffffff) throw std::invalid_argument("operator too large for 32-bit ELL offsets");
        out.slice_off[s + 1] = (int)next;
    }
    size_t total = (size_t)out.slice_off.back();
    out.col.assign(total, 0);
    out.val.assign(total, 0.0);
    for (int r = 0; r < n; r++) {
        int s = r / slice, lane = r % slice, i = out.perm[r];
        for (int e = A.ptr[i], j = 0; e < A.ptr[i + 1]; e++, j++) {
            size_t pos = (size_t)out.slice_off[s] + (size_t)j * slice + lane;
            out.col[pos] = out.iperm[A.col[e]];
            out.val[pos] = A.val[e];
        }
    }
}

Csr permute_rows(const Csr &A, const std::vector<int> &perm)
{
    Csr B;
    B.n = A.n;
    B.m = A.m;
    B.ptr.assign((size_t)A.n + 1, 0);
    for (int r = 0; r < A.n; r++) {
        int i = perm[r];
        B.col.insert(B.col.end(), A.col.begin() + A.ptr[i], A.col.begin() + A.ptr[i + 1]);
        B.val.insert(B.val.end(), A.val.begin() + A.ptr[i], A.val.begin() + A.ptr[i + 1]);
        B.ptr[r + 1] = (int)B.col.size();
    }
    return B;
}

}  // namespace auxp
