// AMG setup on the device (gfx950): the hierarchy of the P^1 matrix A_H that
// Step 1 of Algorithm 2.1 is solved with (PMIS coarsening and extended+i
// interpolation as in Sec. 1 and Sec. 6.1, the strength rule of Sec. 6.2,
// Galerkin coarse operators), the composite level operators of the V-cycle
// and its dense bottom part, for a new coefficient without a trip through
// the host.
//
// Every step repeats the host setup's definitions and its arithmetic in its
// order, with contraction into fused multiply-adds off, so that the device
// hierarchy is bitwise the host one (identical C/F splits on every level):
//  * strength, l1 norms and merging of operators: one thread per row, each
//    sum in the host's order; scaling, copies and row sorts: 16 lanes or a
//    wavefront per row;
//  * extended+i: one workgroup per F row, each thread owning one weight and
//    adding its contributions in the host's order (one thread per row for
//    rows beyond the workgroup's LDS);
//  * sparse products: one wavefront per row (one workgroup for long rows),
//    the row's products sorted by (column, order of the factors' entries)
//    and each column summed in that order, as the host's row accumulator
//    adds them;
//  * PMIS: synchronous rounds, a selection pass (an undecided point whose
//    measure beats every undecided strong neighbour, in S or S^T, becomes C)
//    then a marking pass (undecided points that depend strongly on a new C
//    point become F), which is exactly what the host's rounds compute since
//    each reads only the state at the start of its round;
//  * the coarsest level's dense Cholesky factor and inverse, and the dense
//    cycle T_l = N_l + Q_l T_{l+1} M_l: one workgroup or one workgroup per
//    row, each entry's sum in the host's order.
// Variable-length row work (distance-two interpolation sets, product rows
// and their sort keys) lives in workspaces sized by a first pass's upper
// bounds (prefix sums on the device).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <stdexcept>
#include <string>

#include "amgsetup.hpp"
#include "assemble.hpp"

namespace auxp {

namespace {

#define AMG_CHECK(x)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (x);                                                                          \
        if (e_ != hipSuccess) throw std::runtime_error(std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int kB = 256;

inline int rows_grid(long long n) { return (int)std::max<long long>(1, (n + kB - 1) / kB); }

template <typename T>
T *dnew(DevMem &mem, size_t n)
{
    return (T *)mem.alloc(std::max<size_t>(n, 1) * sizeof(T));
}

void dfree(DevMem &mem, void *p)
{
    if (p) mem.release(p);
}

void free_csr(DevMem &mem, DCsr &a)
{
    dfree(mem, a.ptr);
    dfree(mem, a.col);
    dfree(mem, a.val);
    a = DCsr();
}

// ------------------------------------------------------------ prefix sums

constexpr int kScanItems = 4, kScanTile = kB * kScanItems;

template <typename TI>
__global__ __launch_bounds__(kB) void k_scan_tiles(long long n, const TI *__restrict__ in, long long *__restrict__ tsum)
{
    __shared__ long long red[kB];
    const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
    long long s = 0;
    for (int k = 0; k < kScanItems; k++)
        if (base + k < n) s += (long long)in[base + k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kB / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) tsum[blockIdx.x] = red[0];
}

// one workgroup: exclusive prefix sums of the nt tile sums in place, total in tsum[nt]
__global__ __launch_bounds__(kB) void k_scan_tile_sums(int nt, long long *tsum)
{
    __shared__ long long buf[kB];
    long long carry = 0;
    for (int c0 = 0; c0 < nt; c0 += kB) {
        const int i = c0 + (int)threadIdx.x;
        const long long v = i < nt ? tsum[i] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < kB; o <<= 1) {
            const long long t = (int)threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nt) tsum[i] = carry + buf[threadIdx.x] - v;
        carry += buf[kB - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) tsum[nt] = carry;
}

template <typename TI, typename TO>
__global__ __launch_bounds__(kB) void k_scan_apply(long long n, const TI *__restrict__ in,
                                                   const long long *__restrict__ tsum, TO *__restrict__ out)
{
    __shared__ long long buf[kB];
    const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
    long long v[kScanItems], s = 0;
    for (int k = 0; k < kScanItems; k++) {
        v[k] = base + k < n ? (long long)in[base + k] : 0;
        s += v[k];
    }
    buf[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < kB; o <<= 1) {
        const long long t = (int)threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
        __syncthreads();
        buf[threadIdx.x] += t;
        __syncthreads();
    }
    long long run = tsum[blockIdx.x] + buf[threadIdx.x] - s;
    for (int k = 0; k < kScanItems; k++) {
        if (base + k < n) out[base + k] = (TO)run;
        run += v[k];
        if (base + k == n - 1) out[n] = (TO)run;
    }
}

// out[0] = 0, out[i + 1] = out[i] + in[i] (out has n + 1 entries); returns
// the total (synchronises the stream)
template <typename TI, typename TO>
long long scan(hipStream_t s, long long n, const TI *in, TO *out, DevMem &mem)
{
    if (n <= 0) {
        AMG_CHECK(hipMemsetAsync(out, 0, sizeof(TO), s));
        return 0;
    }
    const long long nt = (n + kScanTile - 1) / kScanTile;
    long long *tsum = dnew<long long>(mem, (size_t)nt + 1);
    hipLaunchKernelGGL((k_scan_tiles<TI>), dim3((unsigned)nt), dim3(kB), 0, s, n, in, tsum);
    hipLaunchKernelGGL(k_scan_tile_sums, dim3(1), dim3(kB), 0, s, (int)nt, tsum);
    hipLaunchKernelGGL((k_scan_apply<TI, TO>), dim3((unsigned)nt), dim3(kB), 0, s, n, in, tsum, out);
    AMG_CHECK(hipGetLastError());
    long long total = 0;
    AMG_CHECK(hipMemcpyAsync(&total, tsum + nt, sizeof(long long), hipMemcpyDeviceToHost, s));
    AMG_CHECK(hipStreamSynchronize(s));
    dfree(mem, tsum);
    return total;
}

int checked_int(long long v, const char *what)
{
    if (v < 0 || v > 0x7fffffffLL) throw std::runtime_error(std::string("device AMG setup: ") + what + " exceeds 2^31");
    return (int)v;
}

// ------------------------------------------------------------ strength

// strong[e] = 1 when i depends strongly on col[e]: -a_ij > max_{k != i}(-a_ik)
// (theta + 1e-12), the maximum over a row with an off-diagonal entry and
// positive; cnt[i] = number of strong entries of row i
__global__ __launch_bounds__(kB) void k_strength(int n, const int *__restrict__ ptr, const int *__restrict__ col,
                                                 const double *__restrict__ val, double theta,
                                                 unsigned char *__restrict__ strong, int *__restrict__ cnt)
{
#pragma clang fp contract(off)
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    double mx = 0.0;
    bool any = false;
    for (int e = ptr[i]; e < ptr[i + 1]; e++)
        if (col[e] != i && (!any || -val[e] > mx)) {
            mx = -val[e];
            any = true;
        }
    const bool on = any && mx > 0.0;
    const double cut = mx * (theta + 1e-12);
    int c = 0;
    for (int e = ptr[i]; e < ptr[i + 1]; e++) {
        const bool st = on && col[e] != i && -val[e] > cut;
        strong[e] = st ? 1 : 0;
        c += st ? 1 : 0;
    }
    cnt[i] = c;
}

// the strong columns of each row, in row order
__global__ __launch_bounds__(kB) void k_strong_fill(int n, const int *__restrict__ ptr, const int *__restrict__ col,
                                                    const unsigned char *__restrict__ strong,
                                                    const int *__restrict__ sptr, int *__restrict__ scol)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    int p = sptr[i];
    for (int e = ptr[i]; e < ptr[i + 1]; e++)
        if (strong[e]) scol[p++] = col[e];
}

// ------------------------------------------------------------ transposes

__global__ __launch_bounds__(kB) void k_count_cols(int nnz, const int *__restrict__ col, int *__restrict__ cnt)
{
    const int e = blockIdx.x * kB + threadIdx.x;
    if (e < nnz) atomicAdd(&cnt[col[e]], 1);
}

// entries of row i go to the rows of their columns, in any order (val may be null)
__global__ __launch_bounds__(kB) void k_scatter_transpose(int n, const int *__restrict__ ptr,
                                                          const int *__restrict__ col, const double *__restrict__ val,
                                                          const int *__restrict__ tptr, int *__restrict__ cursor,
                                                          int *__restrict__ tcol, double *__restrict__ tval)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    for (int e = ptr[i]; e < ptr[i + 1]; e++) {
        const int j = col[e];
        const int p = tptr[j] + atomicAdd(&cursor[j], 1);
        tcol[p] = i;
        if (val) tval[p] = val[e];
    }
}

// each row sorted by column (columns distinct within a row; val may be null)
// rows of at most kSortWave entries: k_sort_rows_wave; longer: k_sort_rows
constexpr int kSortWave = 1024;

// Row i sorted by column (columns distinct) by one wavefront: keys (column
// << 32 | position) sorted in LDS (bitonic), values moved with them.
__global__ __launch_bounds__(64) void k_sort_rows_wave(int n, const int *__restrict__ ptr, int *__restrict__ col,
                                                       double *__restrict__ val)
{
    __shared__ unsigned long long keys[kSortWave];
    __shared__ double vs[kSortWave];
    const int i = blockIdx.x, lane = threadIdx.x;
    if (i >= n) return;
    const int b = ptr[i], d = ptr[i + 1] - b;
    if (d < 2 || d > kSortWave) return;
    int np2 = 1;
    while (np2 < d) np2 <<= 1;
    for (int q = lane; q < np2; q += 64) {
        keys[q] = q < d ? ((unsigned long long)(unsigned)col[b + q] << 32) | (unsigned)q : ~0ULL;
        if (val && q < d) vs[q] = val[b + q];
    }
    __syncthreads();
    for (int kk = 2; kk <= np2; kk <<= 1)
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int t = lane; t < np2 / 2; t += 64) {
                const int i1 = 2 * j * (t / j) + (t % j), i2 = i1 + j;
                const bool up = (i1 & kk) == 0;
                const unsigned long long x = keys[i1], y = keys[i2];
                if ((x > y) == up) {
                    keys[i1] = y;
                    keys[i2] = x;
                }
            }
            __syncthreads();
        }
    for (int q = lane; q < d; q += 64) {
        col[b + q] = (int)(keys[q] >> 32);
        if (val) val[b + q] = vs[(unsigned)keys[q]];
    }
}

__global__ __launch_bounds__(kB) void k_sort_rows(int n, const int *__restrict__ ptr, int *__restrict__ col,
                                                  double *__restrict__ val)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    const int b = ptr[i], e = ptr[i + 1];
    if (e - b <= kSortWave) return;                // k_sort_rows_wave's
    for (int p = b + 1; p < e; p++) {
        const int c = col[p];
        const double v = val ? val[p] : 0.0;
        int q = p - 1;
        while (q >= b && col[q] > c) {
            col[q + 1] = col[q];
            if (val) val[q + 1] = val[q];
            q--;
        }
        col[q + 1] = c;
        if (val) val[q + 1] = v;
    }
}

// T = A^T (n x m -> m x n); rows sorted when sorted_rows, as the host's
// counting transpose leaves them
DCsr transpose(hipStream_t s, const DCsr &A, bool values, bool sorted_rows, DevMem &mem)
{
    DCsr T;
    T.n = A.m;
    T.m = A.n;
    T.nnz = A.nnz;
    int *cnt = dnew<int>(mem, (size_t)A.m);
    AMG_CHECK(hipMemsetAsync(cnt, 0, sizeof(int) * std::max(A.m, 1), s));
    if (A.nnz) hipLaunchKernelGGL(k_count_cols, dim3(rows_grid(A.nnz)), dim3(kB), 0, s, A.nnz, A.col, cnt);
    T.ptr = dnew<int>(mem, (size_t)A.m + 1);
    scan(s, A.m, cnt, T.ptr, mem);
    AMG_CHECK(hipMemsetAsync(cnt, 0, sizeof(int) * std::max(A.m, 1), s));
    T.col = dnew<int>(mem, (size_t)A.nnz);
    T.val = values ? dnew<double>(mem, (size_t)A.nnz) : nullptr;
    hipLaunchKernelGGL(k_scatter_transpose, dim3(rows_grid(A.n)), dim3(kB), 0, s, A.n, A.ptr, A.col,
                       values ? A.val : nullptr, T.ptr, cnt, T.col, T.val);
    if (sorted_rows && T.n > 0) {
        hipLaunchKernelGGL(k_sort_rows_wave, dim3(T.n), dim3(64), 0, s, T.n, T.ptr, T.col, T.val);
        hipLaunchKernelGGL(k_sort_rows, dim3(rows_grid(T.n)), dim3(kB), 0, s, T.n, T.ptr, T.col, T.val);
    }
    AMG_CHECK(hipGetLastError());
    dfree(mem, cnt);
    return T;
}

// ------------------------------------------------------------ PMIS

__device__ __forceinline__ uint64_t splitmix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t splitmix64_host(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// measure |S_i^T| (from the transpose's row lengths) + random; points that
// influence nobody are F from the start
__global__ __launch_bounds__(kB) void k_pmis_init(int n, const int *__restrict__ stptr, uint64_t base,
                                                  uint64_t *__restrict__ rnd, int *__restrict__ cf)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    rnd[i] = splitmix64(base + (uint64_t)i);
    cf[i] = stptr[i + 1] - stptr[i] == 0 ? -1 : 0;
}

// does i's measure exceed j's (influence count, then random, then lower index)
__device__ __forceinline__ bool pmis_wins(int i, int j, const int *__restrict__ stptr, const uint64_t *__restrict__ rnd)
{
    const int ii = stptr[i + 1] - stptr[i], ij = stptr[j + 1] - stptr[j];
    if (ii != ij) return ii > ij;
    if (rnd[i] != rnd[j]) return rnd[i] > rnd[j];
    return i < j;
}

__global__ __launch_bounds__(kB) void k_pmis_select(int n, const int *__restrict__ sptr, const int *__restrict__ scol,
                                                    const int *__restrict__ stptr, const int *__restrict__ stcol,
                                                    const uint64_t *__restrict__ rnd, const int *__restrict__ cf,
                                                    unsigned char *__restrict__ newc)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    if (cf[i] != 0) {
        newc[i] = 0;
        return;
    }
    bool best = true;
    for (int e = sptr[i]; best && e < sptr[i + 1]; e++) {
        const int j = scol[e];
        if (cf[j] == 0 && !pmis_wins(i, j, stptr, rnd)) best = false;
    }
    for (int e = stptr[i]; best && e < stptr[i + 1]; e++) {
        const int j = stcol[e];
        if (cf[j] == 0 && !pmis_wins(i, j, stptr, rnd)) best = false;
    }
    newc[i] = best ? 1 : 0;
}

__global__ __launch_bounds__(kB) void k_pmis_mark(int n, const int *__restrict__ sptr, const int *__restrict__ scol,
                                                  const unsigned char *__restrict__ newc, int *__restrict__ cf,
                                                  int *__restrict__ left)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n || cf[i] != 0) return;
    if (newc[i]) {
        cf[i] = 1;
        return;
    }
    bool dep = false;
    for (int e = sptr[i]; !dep && e < sptr[i + 1]; e++) dep = newc[scol[e]] != 0;
    if (dep) cf[i] = -1;
    else atomicAdd(left, 1);
}

// ------------------------------------------------------------ extended+i

__global__ __launch_bounds__(kB) void k_coarse_flag(int n, const int *__restrict__ cf, int *__restrict__ flag)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i < n) flag[i] = cf[i] > 0 ? 1 : 0;
}

// sum of the diagonal entries of each row, from zero
__global__ __launch_bounds__(kB) void k_diag(int n, const int *__restrict__ ptr, const int *__restrict__ col,
                                             const double *__restrict__ val, double *__restrict__ d)
{
#pragma clang fp contract(off)
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int e = ptr[i]; e < ptr[i + 1]; e++)
        if (col[e] == i) s += val[e];
    d[i] = s;
}

// workspace bound of an F row: |S_i| + sum over strong F neighbours j of |S_j|
// Exclusive prefix sum of v over a workgroup of kB threads (every thread
// calls it); total receives the sum over the workgroup.
__device__ __forceinline__ int block_scan(int v, int *wsum, int &total)
{
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int pre = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < kB / 64; q++) {
        const int t = wsum[q];
        if (q < w) pre += t;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return pre + x - v;
}

__global__ __launch_bounds__(kB) void k_exti_bound(int n, const int *__restrict__ sptr, const int *__restrict__ scol,
                                                   const int *__restrict__ cf, long long *__restrict__ ub)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    long long b = 0;
    if (cf[i] <= 0) {
        b = sptr[i + 1] - sptr[i];
        for (int e = sptr[i]; e < sptr[i + 1]; e++) {
            const int j = scol[e];
            if (cf[j] <= 0) b += sptr[j + 1] - sptr[j];
        }
    }
    ub[i] = b;
}

// position of c in the sorted list h[0..len), or -1
__device__ __forceinline__ int find_sorted(const int *h, int len, int c)
{
    int lo = 0, hi = len;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (h[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    return lo < len && h[lo] == c ? lo : -1;
}

// F rows whose candidate set (at most kExtiCand entries counted with
// repeats) and row of A (at most kExtiRow entries) fit the LDS of
// k_exti_rows_wg; the others go to k_exti_rows
constexpr int kExtiCand = 4096, kExtiRow = 512;

__device__ __forceinline__ bool exti_wg_row(long long ub, int na) { return ub <= kExtiCand && na <= kExtiRow; }

// Interpolation row of each F point: the set hat C_i of C points in S_i and
// in S_j for strong F neighbours j (kept sorted), its weights -w_j / d_ii
// with a_ij on hat C_i added to w_j, each strong F neighbour's a_ij spread
// over hat C_i and i in proportion to its row's entries of sign opposite to
// its diagonal (lumped onto the diagonal when there are none), weak entries
// lumped onto the diagonal -- in the host's order of rows and entries.
__global__ __launch_bounds__(kB) void k_exti_rows(int n, const int *__restrict__ ptr, const int *__restrict__ col,
                                                  const double *__restrict__ val,
                                                  const unsigned char *__restrict__ strong,
                                                  const int *__restrict__ sptr, const int *__restrict__ scol,
                                                  const int *__restrict__ cf, const double *__restrict__ diag,
                                                  const long long *__restrict__ woff, int *__restrict__ hcol,
                                                  double *__restrict__ hw, int *__restrict__ cnt)
{
#pragma clang fp contract(off)
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    if (cf[i] > 0) {
        cnt[i] = 1;
        return;
    }
    if (exti_wg_row(woff[i + 1] - woff[i], ptr[i + 1] - ptr[i])) return;   // k_exti_rows_wg's
    int *hat = hcol + woff[i];
    double *w = hw + woff[i];
    int h = 0;
    auto add = [&](int c) {                       // insert into the sorted set
        int q = h;
        while (q > 0 && hat[q - 1] > c) q--;
        if (q > 0 && hat[q - 1] == c) return;
        for (int r = h; r > q; r--) hat[r] = hat[r - 1];
        hat[q] = c;
        h++;
    };
    for (int e = sptr[i]; e < sptr[i + 1]; e++) {
        const int j = scol[e];
        if (cf[j] > 0) {
            add(j);
        } else {
            for (int f = sptr[j]; f < sptr[j + 1]; f++) {
                const int l = scol[f];
                if (cf[l] > 0) add(l);
            }
        }
    }
    for (int q = 0; q < h; q++) w[q] = 0.0;
    double dii = diag[i];
    for (int e = ptr[i]; e < ptr[i + 1]; e++) {
        const int j = col[e];
        if (j == i) continue;
        const double aij = val[e];
        const int pj = find_sorted(hat, h, j);
        if (pj >= 0) {
            w[pj] += aij;
        } else if (strong[e] && cf[j] <= 0) {
            const double dj = diag[j];
            double den = 0.0;
            for (int f = ptr[j]; f < ptr[j + 1]; f++) {
                const int l = col[f];
                if ((l == i || find_sorted(hat, h, l) >= 0) && val[f] * dj < 0.0) den += val[f];
            }
            if (den == 0.0) {
                dii += aij;
                continue;
            }
            const double scale = aij / den;
            for (int f = ptr[j]; f < ptr[j + 1]; f++) {
                if (val[f] * dj >= 0.0) continue;
                const int l = col[f];
                if (l == i) {
                    dii += scale * val[f];
                } else {
                    const int pl = find_sorted(hat, h, l);
                    if (pl >= 0) w[pl] += scale * val[f];
                }
            }
        } else {
            dii += aij;
        }
    }
    for (int q = 0; q < h; q++) w[q] = -w[q] / dii;
    cnt[i] = h;
}

// The rows of k_exti_rows that fit its LDS, one workgroup per F row, with
// every sum in the same order.  The candidates (C points of S_i and of S_j
// for strong F neighbours j) are sorted in LDS and made unique: hat C_i.
// Each entry of A's row is classified (a point of hat C_i, lumped onto the
// diagonal, or a strong F neighbour spread with scale a_ij / den, den
// summed over row j in order by the entry's thread); then each thread owns
// one weight (or d_ii) and walks all entries and their spread rows in the
// host's order, adding only its own contributions, so each weight receives
// exactly the host's sequence of additions.
__global__ __launch_bounds__(kB) void k_exti_rows_wg(int n, const int *__restrict__ ptr, const int *__restrict__ col,
                                                     const double *__restrict__ val,
                                                     const unsigned char *__restrict__ strong,
                                                     const int *__restrict__ sptr, const int *__restrict__ scol,
                                                     const int *__restrict__ cf, const double *__restrict__ diag,
                                                     const long long *__restrict__ woff, int *__restrict__ hcol,
                                                     double *__restrict__ hw, int *__restrict__ cnt)
{
#pragma clang fp contract(off)
    __shared__ int cand[kExtiCand];
    __shared__ int hat[kExtiCand];
    __shared__ int kind[kExtiRow];                 // >= 0 hat position, -1 diagonal, -2 lumped, -3 spread
    __shared__ double escale[kExtiRow];
    __shared__ int wsum[kB / 64];
    __shared__ double dii_sh;
    const int i = blockIdx.x;
    if (i >= n || cf[i] > 0) return;
    const long long ub = woff[i + 1] - woff[i];
    const int a0 = ptr[i], na = ptr[i + 1] - a0;
    if (!exti_wg_row(ub, na)) return;              // a row of k_exti_rows
    const int t = threadIdx.x;
    // candidates, non-C entries of the S_j as INT_MAX
    const int s0 = sptr[i], ns = sptr[i + 1] - s0;
    int m = 0;
    for (int e0 = 0; e0 < ns; e0 += kB) {
        const int e = e0 + t;
        int j = 0, len = 0;
        if (e < ns) {
            j = scol[s0 + e];
            len = cf[j] > 0 ? 1 : sptr[j + 1] - sptr[j];
        }
        int tot;
        const int off = m + block_scan(len, wsum, tot);
        if (e < ns) {
            if (cf[j] > 0) {
                cand[off] = j;
            } else {
                for (int f = 0; f < len; f++) {
                    const int l = scol[sptr[j] + f];
                    cand[off + f] = cf[l] > 0 ? l : INT_MAX;
                }
            }
        }
        m += tot;
    }
    int np2 = 1;
    while (np2 < m) np2 <<= 1;
    for (int q = m + t; q < np2; q += kB) cand[q] = INT_MAX;
    __syncthreads();
    for (int kk = 2; kk <= np2; kk <<= 1)
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int q = t; q < np2 / 2; q += kB) {
                const int i1 = 2 * j * (q / j) + (q % j), i2 = i1 + j;
                const bool up = (i1 & kk) == 0;
                const int x = cand[i1], y = cand[i2];
                if ((x > y) == up) {
                    cand[i1] = y;
                    cand[i2] = x;
                }
            }
            __syncthreads();
        }
    int h = 0;
    for (int q0 = 0; q0 < m; q0 += kB) {
        const int q = q0 + t;
        const int head = q < m && cand[q] != INT_MAX && (q == 0 || cand[q - 1] != cand[q]) ? 1 : 0;
        int tot;
        const int r = h + block_scan(head, wsum, tot);
        if (head) hat[r] = cand[q];
        h += tot;
    }
    __syncthreads();
    // the entries of row i
    for (int e = t; e < na; e += kB) {
        const int j = col[a0 + e];
        int k = -1;
        if (j != i) {
            const int pj = find_sorted(hat, h, j);
            if (pj >= 0) {
                k = pj;
            } else if (strong[a0 + e] && cf[j] <= 0) {
                const double dj = diag[j];
                double den = 0.0;
                for (int f = ptr[j]; f < ptr[j + 1]; f++) {
                    const int l = col[f];
                    if ((l == i || find_sorted(hat, h, l) >= 0) && val[f] * dj < 0.0) den += val[f];
                }
                if (den == 0.0) {
                    k = -2;
                } else {
                    k = -3;
                    escale[e] = val[a0 + e] / den;
                }
            } else {
                k = -2;
            }
        }
        kind[e] = k;
    }
    __syncthreads();
    // thread t of a pass owns weight q0 + t (q == h: d_ii)
    int *hc = hcol + woff[i];
    double *w = hw + woff[i];
    for (int q0 = 0; q0 <= h; q0 += kB) {
        const int q = q0 + t;
        const int mine = q < h ? hat[q] : -1;
        double acc = q == h ? diag[i] : 0.0;
        for (int e = 0; e < na; e++) {
            const int k = kind[e];
            if (k == -1) continue;
            if (k >= 0) {
                if (q == k) acc += val[a0 + e];
            } else if (k == -2) {
                if (q == h) acc += val[a0 + e];
            } else {
                const int j = col[a0 + e];
                const double dj = diag[j], sc = escale[e];
                for (int f = ptr[j]; f < ptr[j + 1]; f++) {
                    const double vf = val[f];
                    if (vf * dj >= 0.0) continue;
                    const int l = col[f];
                    if (l == i) {
                        if (q == h) acc += sc * vf;
                    } else if (l == mine) {
                        acc += sc * vf;
                    }
                }
            }
        }
        if (q < h) {
            hc[q] = mine;
            w[q] = acc;
        } else if (q == h) {
            dii_sh = acc;
        }
    }
    __syncthreads();
    const double dii = dii_sh;
    for (int q = t; q < h; q += kB) w[q] = -w[q] / dii;
    if (t == 0) cnt[i] = h;
}

__global__ __launch_bounds__(kB) void k_exti_write(int n, const int *__restrict__ cf, const int *__restrict__ cnum,
                                                   const long long *__restrict__ woff, const int *__restrict__ hcol,
                                                   const double *__restrict__ hw, const int *__restrict__ pptr,
                                                   int *__restrict__ pcol, double *__restrict__ pval)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    const int p = pptr[i];
    if (cf[i] > 0) {
        pcol[p] = cnum[i];
        pval[p] = 1.0;
        return;
    }
    const int h = pptr[i + 1] - p;
    for (int q = 0; q < h; q++) {
        pcol[p + q] = cnum[hcol[woff[i] + q]];
        pval[p + q] = hw[woff[i] + q];
    }
}

// ------------------------------------------------------------ sparse products

__global__ __launch_bounds__(kB) void k_product_bound(int n, const int *__restrict__ aptr, const int *__restrict__ acol,
                                                      const int *__restrict__ bptr, long long *__restrict__ ub)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    long long b = 0;
    for (int e = aptr[i]; e < aptr[i + 1]; e++) b += bptr[acol[e] + 1] - bptr[acol[e]];
    ub[i] = b;
}

// Rows of a product by size: at most kSmallProducts products from at most
// kSmallEntries entries of A (0), at most kWaveProducts from kWaveEntries
// (1), both k_product_rows_wave with LDS of that size; longer rows (2)
// k_product_rows_long.  The small form's LDS lets many more rows be in
// flight per compute unit.
constexpr int kSmallProducts = 256, kSmallEntries = 64;
constexpr int kWaveProducts = 2048, kWaveEntries = 256;

__device__ __forceinline__ int product_form(long long ub, int na)
{
    if (ub <= kSmallProducts && na <= kSmallEntries) return 0;
    return ub <= kWaveProducts && na <= kWaveEntries ? 1 : 2;
}
__device__ __forceinline__ bool wave_row(long long ub, int na) { return product_form(ub, na) < 2; }

// Row i of C = A B, one wavefront: the row's products a_ik b_kj are laid
// out in LDS in the order of A's row, then of B's rows (their sequence
// number), sorted by (column, sequence number) with a bitonic network, and
// each column's products are summed in sequence order by the lane that
// holds the column's first one (the first product added to zero when
// zero_init, as the composite-operator product does; taken as the sum
// otherwise, as the Galerkin product does).  The same sums in the same order
// as the host's row accumulator.  The sorted row goes to the workspace at
// woff[i].
template <int CAP, int EC>
__global__ __launch_bounds__(64) void k_product_rows_wave(int n, const int *__restrict__ aptr,
                                                          const int *__restrict__ acol, const double *__restrict__ aval,
                                                          const int *__restrict__ bptr, const int *__restrict__ bcol,
                                                          const double *__restrict__ bval,
                                                          const long long *__restrict__ woff, int *__restrict__ ocol,
                                                          double *__restrict__ oacc, int *__restrict__ cnt, int zero_init)
{
#pragma clang fp contract(off)
    __shared__ unsigned long long keys[CAP];
    __shared__ double vals[CAP];
    __shared__ int off[EC + 1];
    const int i = blockIdx.x, lane = threadIdx.x;
    if (i >= n) return;
    const int a0 = aptr[i], na = aptr[i + 1] - a0;
    const long long ub = woff[i + 1] - woff[i];
    if (product_form(ub, na) != (CAP == kSmallProducts ? 0 : 1)) return;   // another form's row
    if (ub == 0) {
        if (lane == 0) cnt[i] = 0;
        return;
    }
    // first product of each entry of A's row: a prefix sum over the wavefront
    int o = 0;
    for (int e0 = 0; e0 < na; e0 += 64) {
        const int e = e0 + lane;
        int len = 0;
        if (e < na) {
            const int k = acol[a0 + e];
            len = bptr[k + 1] - bptr[k];
        }
        int x = len;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(x, d, 64);
            if (lane >= d) x += y;
        }
        if (e < na) off[e] = o + x - len;
        o += __shfl(x, 63, 64);
    }
    if (lane == 0) off[na] = o;
    __syncthreads();
    const int m = (int)ub;
    int np2 = 1;
    while (np2 < m) np2 <<= 1;
    for (int p = lane; p < np2; p += 64) {
        if (p < m) {
            int lo = 0, hi = na;                   // off[lo] <= p < off[lo + 1]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (off[mid] <= p) lo = mid;
                else hi = mid;
            }
            const int f = bptr[acol[a0 + lo]] + (p - off[lo]);
            keys[p] = ((unsigned long long)(unsigned)bcol[f] << 32) | (unsigned)p;
            vals[p] = aval[a0 + lo] * bval[f];
        } else {
            keys[p] = ~0ULL;
        }
    }
    __syncthreads();
    for (int kk = 2; kk <= np2; kk <<= 1)
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int t = lane; t < np2 / 2; t += 64) {
                const int i1 = 2 * j * (t / j) + (t % j), i2 = i1 + j;
                const bool up = (i1 & kk) == 0;
                const unsigned long long x = keys[i1], y = keys[i2];
                if ((x > y) == up) {
                    keys[i1] = y;
                    keys[i2] = x;
                }
            }
            __syncthreads();
        }
    int base = 0;
    for (int q0 = 0; q0 < m; q0 += 64) {
        const int q = q0 + lane;
        bool head = false;
        int col = 0;
        if (q < m) {
            col = (int)(keys[q] >> 32);
            head = q == 0 || (int)(keys[q - 1] >> 32) != col;
        }
        const unsigned long long mask = __ballot(head);
        if (head) {
            const int rank = base + __popcll(mask & ((1ULL << lane) - 1ULL));
            double acc = vals[(unsigned)keys[q]];
            if (zero_init) acc = 0.0 + acc;
            for (int r = q + 1; r < m && (int)(keys[r] >> 32) == col; r++) acc += vals[(unsigned)keys[r]];
            ocol[woff[i] + rank] = col;
            oacc[woff[i] + rank] = acc;
        }
        base += __popcll(mask);
    }
    if (lane == 0) cnt[i] = base;
}

// workspace slots of the rows k_product_rows_long handles (one per product)
__global__ __launch_bounds__(kB) void k_long_rows(int n, const int *__restrict__ aptr,
                                                  const long long *__restrict__ woff, long long *__restrict__ hub)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    const long long ub = woff[i + 1] - woff[i];
    hub[i] = wave_row(ub, aptr[i + 1] - aptr[i]) ? 0 : ub;
}

// keys sorted in LDS at once by k_product_rows_long
constexpr int kLongChunk = 4096;

// Row i of C = A B for the rows k_product_rows_wave leaves, one workgroup
// per row.  The products a_ik b_kj, numbered in the order of A's row, then
// of B's rows, go to the workspace at hoff[i] with their keys (column << 32
// | number); runs of kLongChunk keys are sorted in LDS (bitonic), then runs
// are merged pairwise (each key's place is its index in its run plus the
// number of keys of the other run below it; keys are distinct); each
// column's products are then summed in number order by the thread holding
// its first one, exactly as in k_product_rows_wave, and the columns written
// in order to the workspace at woff[i].
__global__ __launch_bounds__(kB) void k_product_rows_long(
    int n, const int *__restrict__ aptr, const int *__restrict__ acol, const double *__restrict__ aval,
    const int *__restrict__ bptr, const int *__restrict__ bcol, const double *__restrict__ bval,
    const long long *__restrict__ woff, const long long *__restrict__ hoff, unsigned long long *__restrict__ keya,
    unsigned long long *__restrict__ keyb, double *__restrict__ pval, int *__restrict__ ocol,
    double *__restrict__ oacc, int *__restrict__ cnt, int zero_init)
{
#pragma clang fp contract(off)
    __shared__ unsigned long long sk[kLongChunk];
    __shared__ int wsum[kB / 64];
    const int i = blockIdx.x;
    if (i >= n) return;
    const int a0 = aptr[i], na = aptr[i + 1] - a0;
    const long long ub = woff[i + 1] - woff[i];
    if (wave_row(ub, na)) return;                  // a row of k_product_rows_wave
    const int m = (int)ub;
    unsigned long long *src = keya + hoff[i], *dst = keyb + hoff[i];
    double *pv = pval + hoff[i];
    // the products, numbered in order
    int base = 0;
    for (int e0 = 0; e0 < na; e0 += kB) {
        const int e = e0 + (int)threadIdx.x;
        int k = 0, len = 0;
        if (e < na) {
            k = acol[a0 + e];
            len = bptr[k + 1] - bptr[k];
        }
        int tot;
        const int off = base + block_scan(len, wsum, tot);
        if (e < na) {
            const double a = aval[a0 + e];
            const int f0 = bptr[k];
            for (int f = 0; f < len; f++) {
                src[off + f] = ((unsigned long long)(unsigned)bcol[f0 + f] << 32) | (unsigned)(off + f);
                pv[off + f] = a * bval[f0 + f];
            }
        }
        base += tot;
    }
    __syncthreads();
    // sorted runs
    for (int c0 = 0; c0 < m; c0 += kLongChunk) {
        const int len = std::min(kLongChunk, m - c0);
        int np2 = 1;
        while (np2 < len) np2 <<= 1;
        for (int t = threadIdx.x; t < np2; t += kB) sk[t] = t < len ? src[c0 + t] : ~0ULL;
        __syncthreads();
        for (int kk = 2; kk <= np2; kk <<= 1)
            for (int j = kk >> 1; j > 0; j >>= 1) {
                for (int t = threadIdx.x; t < np2 / 2; t += kB) {
                    const int i1 = 2 * j * (t / j) + (t % j), i2 = i1 + j;
                    const bool up = (i1 & kk) == 0;
                    const unsigned long long x = sk[i1], y = sk[i2];
                    if ((x > y) == up) {
                        sk[i1] = y;
                        sk[i2] = x;
                    }
                }
                __syncthreads();
            }
        for (int t = threadIdx.x; t < len; t += kB) src[c0 + t] = sk[t];
        __syncthreads();
    }
    // pairwise merges of runs of w keys
    for (int w = kLongChunk; w < m; w <<= 1) {
        for (int t = threadIdx.x; t < m; t += kB) {
            const int lo = t / (2 * w) * (2 * w);
            const int mid = std::min(lo + w, m), hi = std::min(lo + 2 * w, m);
            const unsigned long long x = src[t];
            const bool first = t < mid;
            int l = first ? mid : lo, r = first ? hi : mid;
            const int ob = l;
            while (l < r) {
                const int md = (l + r) >> 1;
                if (src[md] < x) l = md + 1;
                else r = md;
            }
            dst[lo + (t - (first ? lo : mid)) + (l - ob)] = x;
        }
        __syncthreads();
        unsigned long long *t = src;
        src = dst;
        dst = t;
    }
    // column sums in number order, columns in order
    int ncols = 0;
    for (int q0 = 0; q0 < m; q0 += kB) {
        const int q = q0 + (int)threadIdx.x;
        int head = 0, col = 0;
        if (q < m) {
            col = (int)(src[q] >> 32);
            head = q == 0 || (int)(src[q - 1] >> 32) != col;
        }
        int tot;
        const int rank = ncols + block_scan(head, wsum, tot);
        if (head) {
            double acc = pv[(unsigned)src[q]];
            if (zero_init) acc = 0.0 + acc;
            for (int r = q + 1; r < m && (int)(src[r] >> 32) == col; r++) acc += pv[(unsigned)src[r]];
            ocol[woff[i] + rank] = col;
            oacc[woff[i] + rank] = acc;
        }
        ncols += tot;
    }
    if (threadIdx.x == 0) cnt[i] = ncols;
}

// lanes per row of the row-wise copy and scaling passes
constexpr int kRowLanes = 16;

__global__ __launch_bounds__(kB) void k_compact_rows(int n, const long long *__restrict__ woff,
                                                     const int *__restrict__ ocol, const double *__restrict__ oacc,
                                                     const int *__restrict__ cptr, int *__restrict__ ccol,
                                                     double *__restrict__ cval)
{
    const long long g = (long long)blockIdx.x * kB + threadIdx.x;
    const int i = (int)(g / kRowLanes), sub = (int)(g % kRowLanes);
    if (i >= n) return;
    const int p = cptr[i], d = cptr[i + 1] - p;
    const long long w0 = woff[i];
    for (int q = sub; q < d; q += kRowLanes) {
        ccol[p + q] = ocol[w0 + q];
        cval[p + q] = oacc[w0 + q];
    }
}

// C = A B
DCsr product(hipStream_t s, const DCsr &A, const DCsr &B, bool zero_init, DevMem &mem)
{
    if (A.m != B.n) throw std::runtime_error("device AMG setup: product shape mismatch");
    DCsr C;
    C.n = A.n;
    C.m = B.m;
    long long *ub = dnew<long long>(mem, (size_t)A.n);
    long long *woff = dnew<long long>(mem, (size_t)A.n + 1);
    hipLaunchKernelGGL(k_product_bound, dim3(rows_grid(A.n)), dim3(kB), 0, s, A.n, A.ptr, A.col, B.ptr, ub);
    const long long total = scan(s, A.n, ub, woff, mem);
    checked_int(total, "products of a sparse product");   // numbers in 32-bit keys
    // sort workspaces only for the rows too long for one wavefront's LDS
    hipLaunchKernelGGL(k_long_rows, dim3(rows_grid(A.n)), dim3(kB), 0, s, A.n, A.ptr, woff, ub);
    long long *hoff = dnew<long long>(mem, (size_t)A.n + 1);
    const long long htotal = scan(s, A.n, ub, hoff, mem);
    dfree(mem, ub);
    unsigned long long *keya = dnew<unsigned long long>(mem, (size_t)htotal);
    unsigned long long *keyb = dnew<unsigned long long>(mem, (size_t)htotal);
    double *pval = dnew<double>(mem, (size_t)htotal);
    int *ocol = dnew<int>(mem, (size_t)total);
    double *oacc = dnew<double>(mem, (size_t)total);
    int *cnt = dnew<int>(mem, (size_t)A.n);
    if (A.n > 0) {
        hipLaunchKernelGGL((k_product_rows_wave<kSmallProducts, kSmallEntries>), dim3(A.n), dim3(64), 0, s, A.n, A.ptr,
                           A.col, A.val, B.ptr, B.col, B.val, woff, ocol, oacc, cnt, zero_init ? 1 : 0);
        hipLaunchKernelGGL((k_product_rows_wave<kWaveProducts, kWaveEntries>), dim3(A.n), dim3(64), 0, s, A.n, A.ptr,
                           A.col, A.val, B.ptr, B.col, B.val, woff, ocol, oacc, cnt, zero_init ? 1 : 0);
    }
    if (htotal > 0)
        hipLaunchKernelGGL(k_product_rows_long, dim3(A.n), dim3(kB), 0, s, A.n, A.ptr, A.col, A.val, B.ptr, B.col,
                           B.val, woff, hoff, keya, keyb, pval, ocol, oacc, cnt, zero_init ? 1 : 0);
    for (void *p : {(void *)keya, (void *)keyb, (void *)pval, (void *)hoff}) dfree(mem, p);
    C.ptr = dnew<int>(mem, (size_t)A.n + 1);
    C.nnz = checked_int(scan(s, A.n, cnt, C.ptr, mem), "product entries");
    C.col = dnew<int>(mem, (size_t)C.nnz);
    C.val = dnew<double>(mem, (size_t)C.nnz);
    hipLaunchKernelGGL(k_compact_rows, dim3(rows_grid((long long)A.n * kRowLanes)), dim3(kB), 0, s, A.n, woff, ocol, oacc, C.ptr, C.col,
                       C.val);
    AMG_CHECK(hipGetLastError());
    for (void *p : {(void *)ocol, (void *)oacc, (void *)cnt, (void *)woff}) dfree(mem, p);
    return C;
}

// ------------------------------------------------------------ composite operators

// diag(left) A diag(right) in place (either may be null): v *= left[i], then v *= right[j]
__global__ __launch_bounds__(kB) void k_scale(int n, const int *__restrict__ ptr, const int *__restrict__ col,
                                              double *__restrict__ val, const double *__restrict__ left,
                                              const double *__restrict__ right)
{
#pragma clang fp contract(off)
    const long long g = (long long)blockIdx.x * kB + threadIdx.x;
    const int i = (int)(g / kRowLanes), sub = (int)(g % kRowLanes);
    if (i >= n) return;
    for (int e = ptr[i] + sub; e < ptr[i + 1]; e += kRowLanes) {
        double v = val[e];
        if (left) v *= left[i];
        if (right) v *= right[col[e]];
        val[e] = v;
    }
}

__global__ __launch_bounds__(kB) void k_merge_count(int n, const int *__restrict__ aptr, const int *__restrict__ acol,
                                                    const int *__restrict__ bptr, const int *__restrict__ bcol,
                                                    int *__restrict__ cnt)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    int e = aptr[i], f = bptr[i], c = 0;
    const int ee = aptr[i + 1], fe = bptr[i + 1];
    while (e < ee || f < fe) {
        const int ca = e < ee ? acol[e] : INT_MAX, cb = f < fe ? bcol[f] : INT_MAX;
        const int m = ca < cb ? ca : cb;
        if (ca == m) e++;
        if (cb == m) f++;
        c++;
    }
    cnt[i] = c;
}

// a A + b B on the union pattern: each entry from zero, the A term first
__global__ __launch_bounds__(kB) void k_merge_fill(int n, double a, const int *__restrict__ aptr,
                                                   const int *__restrict__ acol, const double *__restrict__ aval,
                                                   double b, const int *__restrict__ bptr, const int *__restrict__ bcol,
                                                   const double *__restrict__ bval, const int *__restrict__ cptr,
                                                   int *__restrict__ ccol, double *__restrict__ cval)
{
#pragma clang fp contract(off)
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    int e = aptr[i], f = bptr[i], p = cptr[i];
    const int ee = aptr[i + 1], fe = bptr[i + 1];
    while (e < ee || f < fe) {
        const int ca = e < ee ? acol[e] : INT_MAX, cb = f < fe ? bcol[f] : INT_MAX;
        const int m = ca < cb ? ca : cb;
        double v = 0.0;
        if (ca == m) v += a * aval[e++];
        if (cb == m) v += b * bval[f++];
        ccol[p] = m;
        cval[p] = v;
        p++;
    }
}

DCsr combine(hipStream_t s, double a, const DCsr &A, double b, const DCsr &B, DevMem &mem)
{
    if (A.n != B.n || A.m != B.m) throw std::runtime_error("device AMG setup: combine shape mismatch");
    DCsr C;
    C.n = A.n;
    C.m = A.m;
    int *cnt = dnew<int>(mem, (size_t)A.n);
    hipLaunchKernelGGL(k_merge_count, dim3(rows_grid(A.n)), dim3(kB), 0, s, A.n, A.ptr, A.col, B.ptr, B.col, cnt);
    C.ptr = dnew<int>(mem, (size_t)A.n + 1);
    C.nnz = checked_int(scan(s, A.n, cnt, C.ptr, mem), "combined entries");
    dfree(mem, cnt);
    C.col = dnew<int>(mem, (size_t)C.nnz);
    C.val = dnew<double>(mem, (size_t)C.nnz);
    hipLaunchKernelGGL(k_merge_fill, dim3(rows_grid(A.n)), dim3(kB), 0, s, A.n, a, A.ptr, A.col, A.val, b, B.ptr,
                       B.col, B.val, C.ptr, C.col, C.val);
    AMG_CHECK(hipGetLastError());
    return C;
}

__global__ __launch_bounds__(kB) void k_recip(int n, const double *__restrict__ l1, double *__restrict__ dinv,
                                              double *__restrict__ two_dinv, int *__restrict__ dptr,
                                              int *__restrict__ dcol)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i > n) return;
    dptr[i] = i;
    if (i == n) return;
    const double d = 1.0 / l1[i];
    dinv[i] = d;
    two_dinv[i] = d * 2.0;
    dcol[i] = i;
}

__global__ __launch_bounds__(kB) void k_side_by_side(int n, int am, const int *__restrict__ aptr,
                                                     const int *__restrict__ acol, const double *__restrict__ aval,
                                                     const int *__restrict__ bptr, const int *__restrict__ bcol,
                                                     const double *__restrict__ bval, int *__restrict__ cptr,
                                                     int *__restrict__ ccol, double *__restrict__ cval)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i > n) return;
    cptr[i] = aptr[i] + bptr[i];
    if (i == n) return;
    int p = aptr[i] + bptr[i];
    for (int e = aptr[i]; e < aptr[i + 1]; e++, p++) {
        ccol[p] = acol[e];
        cval[p] = aval[e];
    }
    for (int f = bptr[i]; f < bptr[i + 1]; f++, p++) {
        ccol[p] = am + bcol[f];
        cval[p] = bval[f];
    }
}

DCsr copy_csr(hipStream_t s, const DCsr &A, DevMem &mem)
{
    DCsr C = A;
    C.ptr = dnew<int>(mem, (size_t)A.n + 1);
    C.col = dnew<int>(mem, (size_t)A.nnz);
    C.val = dnew<double>(mem, (size_t)A.nnz);
    AMG_CHECK(hipMemcpyAsync(C.ptr, A.ptr, sizeof(int) * ((size_t)A.n + 1), hipMemcpyDeviceToDevice, s));
    if (A.nnz) {
        AMG_CHECK(hipMemcpyAsync(C.col, A.col, sizeof(int) * (size_t)A.nnz, hipMemcpyDeviceToDevice, s));
        AMG_CHECK(hipMemcpyAsync(C.val, A.val, sizeof(double) * (size_t)A.nnz, hipMemcpyDeviceToDevice, s));
    }
    return C;
}

// down = P^T - (P^T A) D^-1,  up = [2 D^-1 - D^-1 A D^-1,  P - (D^-1 A P)],
// formed in the host's order of operations
void fuse_level_dev(hipStream_t s, const DCsr &A, const DCsr &P, const DCsr &R, const double *l1, DCsr &down,
                    DCsr &up, DevMem &mem)
{
    const int n = A.n;
    double *dinv = dnew<double>(mem, (size_t)n), *two = dnew<double>(mem, (size_t)n);
    DCsr D;
    D.n = D.m = D.nnz = n;
    D.ptr = dnew<int>(mem, (size_t)n + 1);
    D.col = dnew<int>(mem, (size_t)n);
    D.val = two;
    hipLaunchKernelGGL(k_recip, dim3(rows_grid(n + 1)), dim3(kB), 0, s, n, l1, dinv, two, D.ptr, D.col);
    DCsr RA = product(s, R, A, true, mem);
    hipLaunchKernelGGL(k_scale, dim3(rows_grid((long long)RA.n * kRowLanes)), dim3(kB), 0, s, RA.n, RA.ptr, RA.col, RA.val, nullptr, dinv);
    down = combine(s, 1.0, R, -1.0, RA, mem);
    free_csr(mem, RA);
    DCsr SA = copy_csr(s, A, mem);
    hipLaunchKernelGGL(k_scale, dim3(rows_grid((long long)n * kRowLanes)), dim3(kB), 0, s, n, SA.ptr, SA.col, SA.val, dinv, dinv);
    DCsr N = combine(s, 1.0, D, -1.0, SA, mem);
    free_csr(mem, SA);
    free_csr(mem, D);                                  // frees two as D.val
    DCsr AP = product(s, A, P, true, mem);
    hipLaunchKernelGGL(k_scale, dim3(rows_grid((long long)n * kRowLanes)), dim3(kB), 0, s, n, AP.ptr, AP.col, AP.val, dinv, nullptr);
    DCsr Q = combine(s, 1.0, P, -1.0, AP, mem);
    free_csr(mem, AP);
    up.n = n;
    up.m = N.m + Q.m;
    up.nnz = checked_int((long long)N.nnz + Q.nnz, "composite entries");
    up.ptr = dnew<int>(mem, (size_t)n + 1);
    up.col = dnew<int>(mem, (size_t)up.nnz);
    up.val = dnew<double>(mem, (size_t)up.nnz);
    hipLaunchKernelGGL(k_side_by_side, dim3(rows_grid(n + 1)), dim3(kB), 0, s, n, N.m, N.ptr, N.col, N.val, Q.ptr,
                       Q.col, Q.val, up.ptr, up.col, up.val);
    AMG_CHECK(hipGetLastError());
    free_csr(mem, N);
    free_csr(mem, Q);
    dfree(mem, dinv);
}

// ------------------------------------------------------------ dense parts

// Cholesky factor L (row-major, lower part) and the explicit inverse of the
// coarsest operator, one workgroup: each pivot and each entry of the factor
// summed in the host's order, each column of the inverse by forward and
// backward substitution in its own workspace row, then the rounding
// symmetrised.  err = 1 when a pivot is not positive.
__global__ __launch_bounds__(kB) void k_dense_inverse(int n, const int *__restrict__ ptr, const int *__restrict__ col,
                                                      const double *__restrict__ val, double *__restrict__ L,
                                                      double *__restrict__ Y, double *__restrict__ inv,
                                                      int *__restrict__ err)
{
#pragma clang fp contract(off)
    __shared__ double piv;
    __shared__ int bad;
    const long long nn = (long long)n * n;
    for (long long q = threadIdx.x; q < nn; q += kB) L[q] = 0.0;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kB)
        for (int e = ptr[i]; e < ptr[i + 1]; e++) L[(size_t)i * n + col[e]] = val[e];
    __syncthreads();
    for (int j = 0; j < n; j++) {
        if (threadIdx.x == 0) {
            double d = L[(size_t)j * n + j];
            for (int p = 0; p < j; p++) d -= L[(size_t)j * n + p] * L[(size_t)j * n + p];
            if (!(d > 0.0)) bad = 1;
            d = sqrt(d);
            L[(size_t)j * n + j] = d;
            piv = d;
        }
        __syncthreads();
        if (bad) break;
        const double d = piv;
        for (int i = j + 1 + threadIdx.x; i < n; i += kB) {
            double s = L[(size_t)i * n + j];
            for (int p = 0; p < j; p++) s -= L[(size_t)i * n + p] * L[(size_t)j * n + p];
            L[(size_t)i * n + j] = s / d;
        }
        __syncthreads();
    }
    if (bad) {
        if (threadIdx.x == 0) *err = 1;
        return;
    }
    for (int c = threadIdx.x; c < n; c += kB) {
        double *y = Y + (size_t)c * n;
        for (int i = 0; i < n; i++) {
            double s = i == c ? 1.0 : 0.0;
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
    __syncthreads();
    for (long long q = threadIdx.x; q < nn; q += kB) {
        const int i = (int)(q / n), j = (int)(q % n);
        if (j <= i) continue;
        const double s = 0.5 * (inv[(size_t)i * n + j] + inv[(size_t)j * n + i]);
        inv[(size_t)i * n + j] = s;
        inv[(size_t)j * n + i] = s;
    }
}

// Row i of T_l = N + Q T_{l+1} M (one workgroup per row): QT[k] over the
// row's Q entries in order, then each T_l[i][j] from zero: its N entry, then
// QT[k] M[k][j] for k ascending (M^T rows), skipping QT[k] = 0.
__global__ __launch_bounds__(kB) void k_dense_level(int n, int nc, const int *__restrict__ uptr,
                                                    const int *__restrict__ ucol, const double *__restrict__ uval,
                                                    const int *__restrict__ mtptr, const int *__restrict__ mtcol,
                                                    const double *__restrict__ mtval, const double *__restrict__ Tc,
                                                    double *__restrict__ QTw, double *__restrict__ Tn)
{
#pragma clang fp contract(off)
    const int i = blockIdx.x;
    double *QT = QTw + (size_t)i * nc;
    double *row = Tn + (size_t)i * n;
    for (int k = threadIdx.x; k < nc; k += kB) {
        double q = 0.0;
        for (int e = uptr[i]; e < uptr[i + 1]; e++) {
            const int c = ucol[e];
            if (c >= n) q += uval[e] * Tc[(size_t)(c - n) * nc + k];
        }
        QT[k] = q;
    }
    for (int j = threadIdx.x; j < n; j += kB) row[j] = 0.0;
    __syncthreads();
    for (int e = uptr[i] + threadIdx.x; e < uptr[i + 1]; e += kB) {
        const int c = ucol[e];
        if (c < n) row[c] += uval[e];
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += kB) {
        double v = row[j];
        for (int f = mtptr[j]; f < mtptr[j + 1]; f++) {
            const double a = QT[mtcol[f]];
            if (a == 0.0) continue;
            v += a * mtval[f];
        }
        row[j] = v;
    }
}

__global__ __launch_bounds__(kB) void k_to_f32(long long n, const double *__restrict__ a, float *__restrict__ b)
{
    const long long i = (long long)blockIdx.x * kB + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

__global__ __launch_bounds__(kB) void k_reciprocal(int n, const double *__restrict__ a, double *__restrict__ b)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i < n) b[i] = 1.0 / a[i];
}

// ------------------------------------------------------------ row-split sliced ELL

// slots[s] = 64 x the widest row of slice s in groups of `lanes` entries
__global__ __launch_bounds__(kB) void k_ell_width(int nsl, int n, int rows, int lanes, const int *__restrict__ ptr,
                                                  int *__restrict__ slots)
{
    const int s = blockIdx.x * kB + threadIdx.x;
    if (s >= nsl) return;
    int w = 0;
    for (int q = 0; q < rows && s * rows + q < n; q++) {
        const int i = s * rows + q;
        w = max(w, (ptr[i + 1] - ptr[i] + lanes - 1) / lanes);
    }
    slots[s] = 64 * w;
}

// entry k of row i (slice s = i / rows, row q = i % rows of it) goes to slot
// k / lanes of its slice, lane q * lanes + k % lanes
__global__ __launch_bounds__(kB) void k_ell_fill(int n, int rows, int lanes, const int *__restrict__ ptr,
                                                 const int *__restrict__ col, const double *__restrict__ val,
                                                 const int *__restrict__ off, int *__restrict__ ecol,
                                                 double *__restrict__ eval)
{
    const long long g = (long long)blockIdx.x * kB + threadIdx.x;
    const int i = (int)(g / kRowLanes), sub = (int)(g % kRowLanes);
    if (i >= n) return;
    const int s = i / rows, q = i % rows;
    for (int e = ptr[i] + sub, k = sub; e < ptr[i + 1]; e += kRowLanes, k += kRowLanes) {
        const size_t at = (size_t)off[s] + (size_t)(k / lanes) * 64 + q * lanes + k % lanes;
        ecol[at] = col[e];
        eval[at] = val[e];
    }
}

}  // namespace

void device_amg(hipStream_t s, const DCsr &AH, const SetupOptions &opt, bool fuse, int dense_rows, DevMem &mem,
                DevAmg &out)
{
    out = DevAmg();
    out.A.push_back(copy_csr(s, AH, mem));
    int *left = dnew<int>(mem, 1);
    for (int l = 0;; l++) {
        const DCsr A = out.A[l];
        const int n = A.n;
        double *l1 = dnew<double>(mem, (size_t)n);
        row_l1(s, n, A.ptr, A.val, l1);
        out.l1.push_back(l1);
        if (n <= opt.coarse_max || l + 1 >= opt.max_levels) break;
        // strong dependencies S (row order) and S^T
        unsigned char *strong = dnew<unsigned char>(mem, (size_t)A.nnz);
        int *scnt = dnew<int>(mem, (size_t)n);
        hipLaunchKernelGGL(k_strength, dim3(rows_grid(n)), dim3(kB), 0, s, n, A.ptr, A.col, A.val, opt.theta, strong,
                           scnt);
        DCsr S;
        S.n = S.m = n;
        S.ptr = dnew<int>(mem, (size_t)n + 1);
        S.nnz = checked_int(scan(s, n, scnt, S.ptr, mem), "strong entries");
        dfree(mem, scnt);
        S.col = dnew<int>(mem, (size_t)S.nnz);
        hipLaunchKernelGGL(k_strong_fill, dim3(rows_grid(n)), dim3(kB), 0, s, n, A.ptr, A.col, strong, S.ptr, S.col);
        DCsr ST = transpose(s, S, false, false, mem);
        // PMIS rounds
        uint64_t *rnd = dnew<uint64_t>(mem, (size_t)n);
        int *cf = dnew<int>(mem, (size_t)n);
        unsigned char *newc = dnew<unsigned char>(mem, (size_t)n);
        const uint64_t base = splitmix64_host(opt.seed) + ((uint64_t)l << 32);
        hipLaunchKernelGGL(k_pmis_init, dim3(rows_grid(n)), dim3(kB), 0, s, n, ST.ptr, base, rnd, cf);
        for (int round = 0;; round++) {
            if (round > n) throw std::runtime_error("device AMG setup: PMIS does not terminate");
            AMG_CHECK(hipMemsetAsync(left, 0, sizeof(int), s));
            hipLaunchKernelGGL(k_pmis_select, dim3(rows_grid(n)), dim3(kB), 0, s, n, S.ptr, S.col, ST.ptr, ST.col,
                               rnd, cf, newc);
            hipLaunchKernelGGL(k_pmis_mark, dim3(rows_grid(n)), dim3(kB), 0, s, n, S.ptr, S.col, newc, cf, left);
            AMG_CHECK(hipGetLastError());
            int h_left = 0;
            AMG_CHECK(hipMemcpyAsync(&h_left, left, sizeof(int), hipMemcpyDeviceToHost, s));
            AMG_CHECK(hipStreamSynchronize(s));
            if (h_left == 0) break;
        }
        for (void *p : {(void *)rnd, (void *)newc}) dfree(mem, p);
        free_csr(mem, ST);
        // coarse numbering and extended+i interpolation
        int *flag = dnew<int>(mem, (size_t)n), *cnum = dnew<int>(mem, (size_t)n + 1);
        hipLaunchKernelGGL(k_coarse_flag, dim3(rows_grid(n)), dim3(kB), 0, s, n, cf, flag);
        const int nc = checked_int(scan(s, n, flag, cnum, mem), "coarse points");
        dfree(mem, flag);
        if (nc == 0 || nc >= n) {
            for (void *p : {(void *)strong, (void *)cf, (void *)cnum}) dfree(mem, p);
            free_csr(mem, S);
            break;
        }
        double *diag = dnew<double>(mem, (size_t)n);
        hipLaunchKernelGGL(k_diag, dim3(rows_grid(n)), dim3(kB), 0, s, n, A.ptr, A.col, A.val, diag);
        long long *ub = dnew<long long>(mem, (size_t)n), *woff = dnew<long long>(mem, (size_t)n + 1);
        hipLaunchKernelGGL(k_exti_bound, dim3(rows_grid(n)), dim3(kB), 0, s, n, S.ptr, S.col, cf, ub);
        const long long wtot = scan(s, n, ub, woff, mem);
        dfree(mem, ub);
        int *hcol = dnew<int>(mem, (size_t)wtot), *pcnt = dnew<int>(mem, (size_t)n);
        double *hw = dnew<double>(mem, (size_t)wtot);
        hipLaunchKernelGGL(k_exti_rows, dim3(rows_grid(n)), dim3(kB), 0, s, n, A.ptr, A.col, A.val, strong, S.ptr,
                           S.col, cf, diag, woff, hcol, hw, pcnt);
        hipLaunchKernelGGL(k_exti_rows_wg, dim3(std::max(n, 1)), dim3(kB), 0, s, n, A.ptr, A.col, A.val, strong, S.ptr,
                           S.col, cf, diag, woff, hcol, hw, pcnt);
        DCsr P;
        P.n = n;
        P.m = nc;
        P.ptr = dnew<int>(mem, (size_t)n + 1);
        P.nnz = checked_int(scan(s, n, pcnt, P.ptr, mem), "interpolation entries");
        P.col = dnew<int>(mem, (size_t)P.nnz);
        P.val = dnew<double>(mem, (size_t)P.nnz);
        hipLaunchKernelGGL(k_exti_write, dim3(rows_grid(n)), dim3(kB), 0, s, n, cf, cnum, woff, hcol, hw, P.ptr, P.col,
                           P.val);
        AMG_CHECK(hipGetLastError());
        for (void *p : {(void *)hcol, (void *)hw, (void *)pcnt, (void *)woff, (void *)diag, (void *)cnum,
                        (void *)strong})
            dfree(mem, p);
        free_csr(mem, S);
        // R = P^T and the Galerkin operator R (A P)
        DCsr R = transpose(s, P, true, true, mem);
        DCsr AP = product(s, A, P, false, mem);
        DCsr Ac = product(s, R, AP, false, mem);
        free_csr(mem, AP);
        out.cf.push_back(cf);
        out.P.push_back(P);
        out.R.push_back(R);
        out.A.push_back(Ac);
    }
    dfree(mem, left);
    const size_t L = out.A.size();
    // the coarsest operator's exact inverse
    const DCsr &Ac = out.A[L - 1];
    if (Ac.n > 8192) throw std::runtime_error("coarsest AMG level too large for a dense solve");
    out.ncoarse = Ac.n;
    {
        const size_t nn = (size_t)Ac.n * Ac.n;
        double *Lf = dnew<double>(mem, nn), *Y = dnew<double>(mem, nn);
        out.coarse_inv = dnew<double>(mem, nn);
        int *err = dnew<int>(mem, 1);
        AMG_CHECK(hipMemsetAsync(err, 0, sizeof(int), s));
        hipLaunchKernelGGL(k_dense_inverse, dim3(1), dim3(kB), 0, s, Ac.n, Ac.ptr, Ac.col, Ac.val, Lf, Y,
                           out.coarse_inv, err);
        AMG_CHECK(hipGetLastError());
        int h_err = 0;
        AMG_CHECK(hipMemcpyAsync(&h_err, err, sizeof(int), hipMemcpyDeviceToHost, s));
        AMG_CHECK(hipStreamSynchronize(s));
        for (void *p : {(void *)Lf, (void *)Y, (void *)err}) dfree(mem, p);
        if (h_err) throw std::runtime_error("coarsest AMG operator is not positive definite");
    }
    if (!fuse) return;
    out.down.resize(L - 1);
    out.up.resize(L - 1);
    for (size_t l = 0; l + 1 < L; l++) fuse_level_dev(s, out.A[l], out.P[l], out.R[l], out.l1[l], out.down[l], out.up[l], mem);
    if (dense_rows <= 0) return;
    size_t l0 = L;
    for (size_t l = 0; l + 1 < L; l++)
        if (out.A[l].n <= dense_rows) {
            l0 = l;
            break;
        }
    if (l0 == L) return;
    // T = coarse_inv on the coarsest level, T_l = N_l + Q_l T_{l+1} M_l above it
    double *T = dnew<double>(mem, (size_t)out.ncoarse * out.ncoarse);
    AMG_CHECK(hipMemcpyAsync(T, out.coarse_inv, sizeof(double) * (size_t)out.ncoarse * out.ncoarse,
                             hipMemcpyDeviceToDevice, s));
    for (size_t l = L - 1; l-- > l0;) {
        const int n = out.A[l].n, nc = out.A[l + 1].n;
        DCsr MT = transpose(s, out.down[l], true, true, mem);
        double *QT = dnew<double>(mem, (size_t)n * nc), *Tn = dnew<double>(mem, (size_t)n * n);
        hipLaunchKernelGGL(k_dense_level, dim3(n), dim3(kB), 0, s, n, nc, out.up[l].ptr, out.up[l].col, out.up[l].val,
                           MT.ptr, MT.col, MT.val, T, QT, Tn);
        AMG_CHECK(hipGetLastError());
        free_csr(mem, MT);
        dfree(mem, QT);
        dfree(mem, T);
        T = Tn;
    }
    out.dense = T;
    out.dense_first = (int)l0;
    out.dense_n = out.A[l0].n;
    AMG_CHECK(hipStreamSynchronize(s));
}

namespace {

Csr download_csr(hipStream_t s, const DCsr &a)
{
    Csr c;
    c.n = a.n;
    c.m = a.m;
    c.ptr.resize((size_t)a.n + 1);
    c.col.resize((size_t)a.nnz);
    c.val.resize((size_t)a.nnz);
    AMG_CHECK(hipMemcpyAsync(c.ptr.data(), a.ptr, sizeof(int) * ((size_t)a.n + 1), hipMemcpyDeviceToHost, s));
    if (a.nnz) {
        AMG_CHECK(hipMemcpyAsync(c.col.data(), a.col, sizeof(int) * (size_t)a.nnz, hipMemcpyDeviceToHost, s));
        AMG_CHECK(hipMemcpyAsync(c.val.data(), a.val, sizeof(double) * (size_t)a.nnz, hipMemcpyDeviceToHost, s));
    }
    return c;
}

}  // namespace

void download_amg(hipStream_t s, const DevAmg &d, Hierarchy &h, std::vector<FusedLevel> *fused)
{
    const size_t L = d.A.size();
    h.levels.assign(L, AmgLevel());
    for (size_t l = 0; l < L; l++) {
        AmgLevel &lv = h.levels[l];
        lv.A = download_csr(s, d.A[l]);
        lv.l1.resize((size_t)d.A[l].n);
        AMG_CHECK(hipMemcpyAsync(lv.l1.data(), d.l1[l], sizeof(double) * lv.l1.size(), hipMemcpyDeviceToHost, s));
        if (l + 1 < L) {
            lv.P = download_csr(s, d.P[l]);
            lv.R = download_csr(s, d.R[l]);
            lv.cf.resize((size_t)d.A[l].n);
            AMG_CHECK(hipMemcpyAsync(lv.cf.data(), d.cf[l], sizeof(int) * lv.cf.size(), hipMemcpyDeviceToHost, s));
        }
    }
    h.ncoarse = d.ncoarse;
    h.coarse_inv.resize((size_t)d.ncoarse * d.ncoarse);
    AMG_CHECK(hipMemcpyAsync(h.coarse_inv.data(), d.coarse_inv, sizeof(double) * h.coarse_inv.size(),
                             hipMemcpyDeviceToHost, s));
    if (fused) {
        fused->assign(L, FusedLevel());
        for (size_t l = 0; l + 1 < L; l++) {
            (*fused)[l].down = download_csr(s, d.down[l]);
            (*fused)[l].up = download_csr(s, d.up[l]);
        }
    }
    AMG_CHECK(hipStreamSynchronize(s));
}

void to_f32_device(hipStream_t s, long long n, const double *a, float *b)
{
    if (n > 0) hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + kB - 1) / kB)), dim3(kB), 0, s, n, a, b);
    AMG_CHECK(hipGetLastError());
}

void reciprocal_device(hipStream_t s, int n, const double *a, double *b)
{
    if (n > 0) hipLaunchKernelGGL(k_reciprocal, dim3(rows_grid(n)), dim3(kB), 0, s, n, a, b);
    AMG_CHECK(hipGetLastError());
}

void ell_from_csr(hipStream_t s, const DCsr &A, int lanes, DevMem &mem, DevEll &out)
{
    if (lanes < 1 || lanes > 64 || (64 % lanes) != 0) throw std::invalid_argument("ell_from_csr: lanes must divide 64");
    out = DevEll();
    const int rows = 64 / lanes, nsl = (A.n + rows - 1) / rows;
    int *slots = dnew<int>(mem, (size_t)nsl);
    if (nsl > 0)
        hipLaunchKernelGGL(k_ell_width, dim3(rows_grid(nsl)), dim3(kB), 0, s, nsl, A.n, rows, lanes, A.ptr, slots);
    out.off = dnew<int>(mem, (size_t)nsl + 1);
    out.stored = checked_int(scan(s, nsl, slots, out.off, mem), "ELL slots");
    dfree(mem, slots);
    out.col = dnew<int>(mem, (size_t)out.stored);
    out.val = dnew<double>(mem, (size_t)out.stored);
    if (out.stored > 0) {
        AMG_CHECK(hipMemsetAsync(out.col, 0, sizeof(int) * (size_t)out.stored, s));
        AMG_CHECK(hipMemsetAsync(out.val, 0, sizeof(double) * (size_t)out.stored, s));
    }
    if (A.n > 0)
        hipLaunchKernelGGL(k_ell_fill, dim3(rows_grid((long long)A.n * kRowLanes)), dim3(kB), 0, s, A.n, rows, lanes, A.ptr, A.col, A.val,
                           out.off, out.col, out.val);
    AMG_CHECK(hipGetLastError());
}

void free_amg(DevMem &mem, DevAmg &d)
{
    for (std::vector<DCsr> *v : {&d.A, &d.P, &d.R, &d.down, &d.up})
        for (DCsr &c : *v) free_csr(mem, c);
    for (double *p : d.l1) dfree(mem, p);
    for (int *p : d.cf) dfree(mem, p);
    dfree(mem, d.coarse_inv);
    dfree(mem, d.dense);
    d = DevAmg();
}

}  // namespace auxp
