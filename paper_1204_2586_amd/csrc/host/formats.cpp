// Device storage formats built on the host (once per setup).
//
// Sliced ELLPACK for the P^k operator.  Rows keep the dof order (which is
// lexicographic in the vertex multisets, so neighbours along one mesh axis
// are adjacent in memory) except that within each window of `window`
// consecutive rows longer rows come first (stable): the rows of a slice then
// have nearly equal lengths.  Consecutive groups of `slice` rows form slices
// whose entries are stored column-major (entry j of the slice's rows is
// contiguous), padded to the slice's longest row with zero values.  Each
// such group of `slice` entries (a slot) stores its columns as 16-bit
// offsets from a per-slot base when they span less than 2^16, which cuts
// the index stream from 4 to 2 bytes per entry; other slots keep 32-bit
// columns in a side array.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <stdexcept>

#include "setup.hpp"

namespace auxp {

void build_sell(const Csr &A, int slice, int window, bool index16, Sell &out, bool permute_cols)
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
            out.col[pos] = permute_cols ? out.iperm[A.col[e]] : A.col[e];
            out.val[pos] = A.val[e];
        }
    }
    // compressed columns; padding entries (value 0) take the slot's base
    const size_t nslots = total / (size_t)slice;
    out.mode.assign(out.nslices, 0);
    out.base.assign(index16 ? nslots : 0, 0);
    out.off.assign(index16 ? total : 0, 0);
    out.wide.clear();
    out.max_width = 0;
    for (int s = 0; s < out.nslices; s++) {
        const int r0 = s * slice, r1 = std::min(n, r0 + slice);
        const int width = (out.slice_off[s + 1] - out.slice_off[s]) / slice;
        const size_t e0 = (size_t)out.slice_off[s];
        out.max_width = std::max(out.max_width, width);
        bool narrow = index16;
        for (int j = 0; j < width; j++) {
            const size_t t = e0 / slice + j, ej = t * slice;
            int lo = INT32_MAX, hi = INT32_MIN;
            for (int r = r0; r < r1; r++)
                if (len(out.perm[r]) > j) {
                    lo = std::min(lo, out.col[ej + (r - r0)]);
                    hi = std::max(hi, out.col[ej + (r - r0)]);
                }
            if (index16) out.base[t] = lo;
            if ((int64_t)hi - lo >= 65536) narrow = false;
            for (int l = 0; l < slice; l++) {
                const bool valid = r0 + l < r1 && len(out.perm[r0 + l]) > j;
                if (!valid) out.col[ej + l] = lo;     // padding points at a column of the slot
                else if (index16 && (int64_t)hi - lo < 65536) out.off[ej + l] = (uint16_t)(out.col[ej + l] - lo);
            }
        }
        if (!narrow) {
            if (out.wide.size() + (size_t)width * slice > 0x7fffffffu) throw std::invalid_argument("operator too large");
            out.mode[s] = ~(int)out.wide.size();
            out.wide.insert(out.wide.end(), out.col.begin() + e0, out.col.begin() + e0 + (size_t)width * slice);
        }
    }
}

void build_tiles(const Csr &A, const std::vector<int> &iperm, int tile, Tiles &out)
{
    const int n = A.n;
    out = Tiles();
    out.n = n;
    out.tile = tile;
    out.ntiles = (n + tile - 1) / tile;
    out.rows.assign((size_t)out.ntiles * tile, -1);
    out.row_ptr.assign((size_t)out.ntiles * tile + 1, 0);
    out.col_off.assign((size_t)out.ntiles + 1, 0);
    std::vector<int> cols;
    for (int t = 0; t < out.ntiles; t++) {
        const int r0 = t * tile, r1 = std::min(n, r0 + tile);
        cols.clear();
        for (int r = r0; r < r1; r++)
            for (int e = A.ptr[r]; e < A.ptr[r + 1]; e++) cols.push_back(iperm[A.col[e]]);
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        if (cols.size() > 65535) throw std::invalid_argument("build_tiles: tile too wide for 16-bit positions");
        out.ucols.insert(out.ucols.end(), cols.begin(), cols.end());
        out.col_off[t + 1] = (int)out.ucols.size();
        out.max_cols = std::max(out.max_cols, (int)cols.size());
        const size_t first = out.val.size();
        for (int i = 0; i < tile; i++) {
            const int r = r0 + i;
            if (r < r1) {
                out.rows[(size_t)t * tile + i] = iperm[r];
                for (int e = A.ptr[r]; e < A.ptr[r + 1]; e++) {
                    const int c = iperm[A.col[e]];
                    out.lidx.push_back((uint16_t)(std::lower_bound(cols.begin(), cols.end(), c) - cols.begin()));
                    out.val.push_back(A.val[e]);
                }
            }
            if (out.val.size() > 0x7fffffffu) throw std::invalid_argument("build_tiles: operator too large");
            out.row_ptr[(size_t)t * tile + i + 1] = (int)out.val.size();
        }
        out.max_entries = std::max(out.max_entries, (int)(out.val.size() - first));
    }
}

Csr permute_symmetric(const Csr &A, const std::vector<int> &perm, const std::vector<int> &iperm)
{
    Csr B;
    B.n = A.n;
    B.m = A.m;
    B.ptr.assign((size_t)A.n + 1, 0);
    std::vector<std::pair<int, double>> row;
    for (int r = 0; r < A.n; r++) {
        const int i = perm[r];
        row.clear();
        for (int e = A.ptr[i]; e < A.ptr[i + 1]; e++) row.push_back({iperm[A.col[e]], A.val[e]});
        std::sort(row.begin(), row.end());
        for (auto &cv : row) {
            B.col.push_back(cv.first);
            B.val.push_back(cv.second);
        }
        B.ptr[r + 1] = (int)B.col.size();
    }
    return B;
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

std::vector<int> morton_order(const std::vector<double> &xyz, int n)
{
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int i = 0; i < n; i++)
        for (int c = 0; c < 3; c++) {
            lo[c] = std::min(lo[c], xyz[3 * (size_t)i + c]);
            hi[c] = std::max(hi[c], xyz[3 * (size_t)i + c]);
        }
    // spread the 21 low bits of v to every third bit
    auto spread = [](uint64_t v) {
        v &= 0x1fffff;
        v = (v | v << 32) & 0x1f00000000ffffULL;
        v = (v | v << 16) & 0x1f0000ff0000ffULL;
        v = (v | v << 8) & 0x100f00f00f00f00fULL;
        v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
        v = (v | v << 2) & 0x1249249249249249ULL;
        return v;
    };
    std::vector<std::pair<uint64_t, int>> code((size_t)n);
    for (int i = 0; i < n; i++) {
        uint64_t m = 0;
        for (int c = 0; c < 3; c++) {
            const double span = hi[c] - lo[c];
            const double t = span > 0 ? (xyz[3 * (size_t)i + c] - lo[c]) / span : 0.0;
            const uint64_t q = (uint64_t)std::min(2097151.0, std::max(0.0, std::floor(t * 2097151.0 + 0.5)));
            m |= spread(q) << c;
        }
        code[i] = {m, i};
    }
    std::sort(code.begin(), code.end());
    std::vector<int> ord((size_t)n);
    for (int r = 0; r < n; r++) ord[r] = code[r].second;
    return ord;
}

Csr renumber_cols(const Csr &A, const std::vector<int> &map, int split)
{
    Csr B;
    B.n = A.n;
    B.m = A.m;
    B.ptr.assign((size_t)A.n + 1, 0);
    std::vector<std::pair<int, double>> row;
    for (int r = 0; r < A.n; r++) {
        row.clear();
        for (int e = A.ptr[r]; e < A.ptr[r + 1]; e++) {
            const int j = A.col[e];
            row.push_back({j < split ? map[j] : split + map[j - split], A.val[e]});
        }
        std::sort(row.begin(), row.end());
        for (auto &cv : row) {
            B.col.push_back(cv.first);
            B.val.push_back(cv.second);
        }
        B.ptr[r + 1] = (int)B.col.size();
    }
    return B;
}

void build_ell(const Csr &A, int lanes, Ell &out)
{
    if (lanes < 1 || lanes > 64 || (64 % lanes) != 0) throw std::invalid_argument("build_ell: lanes must divide 64");
    const int rows = 64 / lanes;
    out = Ell();
    out.n = A.n;
    out.lanes = lanes;
    out.nslices = (A.n + rows - 1) / rows;
    out.slice_off.assign((size_t)out.nslices + 1, 0);
    for (int s = 0; s < out.nslices; s++) {
        int width = 0;
        for (int q = 0; q < rows && s * rows + q < A.n; q++) {
            const int i = s * rows + q;
            width = std::max(width, (A.ptr[i + 1] - A.ptr[i] + lanes - 1) / lanes);
        }
        out.slice_off[s + 1] = out.slice_off[s] + 64 * width;
    }
    out.col.assign((size_t)out.slice_off[out.nslices], 0);
    out.val.assign((size_t)out.slice_off[out.nslices], 0.0);
    for (int s = 0; s < out.nslices; s++)
        for (int q = 0; q < rows && s * rows + q < A.n; q++) {
            const int i = s * rows + q;
            for (int e = A.ptr[i], k = 0; e < A.ptr[i + 1]; e++, k++) {
                const size_t at = (size_t)out.slice_off[s] + (size_t)(k / lanes) * 64 + q * lanes + k % lanes;
                out.col[at] = A.col[e];
                out.val[at] = A.val[e];
            }
        }
}

}  // namespace auxp
