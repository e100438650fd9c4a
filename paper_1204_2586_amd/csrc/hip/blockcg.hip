// Kernels of block preconditioned CG (O'Leary 1980) on blocks of NR columns
// stored row-major [n][NR] (gfx950, wave64).
//
// Beside the block products and the block preconditioner shared with the
// lock-step batched solve, block CG needs three passes over the blocks:
//  * the Gram matrix G = U^T V (NR x NR, FP64): each workgroup stages tiles
//    of rows of U and V in LDS and accumulates its share of the NR^2
//    entries over its row range into one partial matrix; a finish kernel
//    sums the partial matrices in a fixed order (no atomics: deterministic);
//  * X += P alpha, R -= Q alpha with the per-column partial sums of r.r and
//    the preconditioner's first sweep from zero (Z0 = D^-1 R, and R in the
//    preconditioner's type), like the lock-step update;
//  * P = Z + P beta.
// alpha and beta (NR x NR) are read from device memory; one row of P and Q
// passes through LDS so every thread of the row reads all of its values.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdexcept>

#include "blockcg.hpp"

namespace auxp {

namespace {

constexpr int kBlk = 256;
// rows per LDS tile of the Gram kernel (32 KiB of LDS for NR = 32 and 64)
template <int NR>
constexpr int gram_tile() { return NR <= 32 ? 64 : 32; }

// G partial of this workgroup: sum over its rows of U[row][a] V[row][b].
// Thread t owns E = NR^2 / 256 entries (NR >= 16) or, for NR = 8, one entry
// over every fourth row of the tile (RG = 4 row groups added at the end in a
// fixed order).
template <int NR, typename TU>
__global__ __launch_bounds__(kBlk) void k_block_gram(int n, const TU *__restrict__ U, const double *__restrict__ V,
                                                     double *__restrict__ partials)
{
    constexpr int RG = NR * NR >= kBlk ? 1 : kBlk / (NR * NR);
    constexpr int E = NR * NR >= kBlk ? NR * NR / kBlk : 1;
    constexpr int kGramTile = gram_tile<NR>();
    __shared__ double su[kGramTile][NR];
    __shared__ double sv[kGramTile][NR];
    __shared__ double sred[RG > 1 ? kBlk : 1];
    const int t = threadIdx.x;
    const int rg = t / (kBlk / RG);                 // row group (NR = 8)
    const int e0 = (t % (kBlk / RG)) * E;           // first owned entry
    const int a = e0 / NR, b0 = e0 % NR;            // entries (a, b0 .. b0 + E - 1)
    const int per = (n + gridDim.x - 1) / gridDim.x;
    const int r0 = blockIdx.x * per, r1 = min(n, r0 + per);
    double acc[E];
#pragma unroll
    for (int e = 0; e < E; e++) acc[e] = 0.0;
    for (int base = r0; base < r1; base += kGramTile) {
        const int rows = min(kGramTile, r1 - base);
        for (int i = t; i < kGramTile * NR; i += kBlk) {
            const int r = i / NR, c = i % NR;
            const bool in = r < rows;
            su[r][c] = in ? (double)U[(size_t)(base + r) * NR + c] : 0.0;
            sv[r][c] = in ? V[(size_t)(base + r) * NR + c] : 0.0;
        }
        __syncthreads();
        for (int r = rg; r < kGramTile; r += RG) {
            const double ua = su[r][a];
#pragma unroll
            for (int e = 0; e < E; e++) acc[e] += ua * sv[r][b0 + e];
        }
        __syncthreads();
    }
    double *out = partials + (size_t)blockIdx.x * NR * NR;
    if (RG == 1) {
#pragma unroll
        for (int e = 0; e < E; e++) out[e0 + e] = acc[e];
    } else {
        sred[t] = acc[0];
        __syncthreads();
        if (rg == 0) {
            double s = 0.0;
            for (int g = 0; g < RG; g++) s += sred[g * (kBlk / RG) + t];
            out[e0] = s;
        }
    }
}

// G = sum over g of partials[g] in increasing g (one thread per entry)
template <int NR>
__global__ __launch_bounds__(kBlk) void k_block_gram_finish(const double *__restrict__ partials, int nparts,
                                                            double *__restrict__ G)
{
    const int e = blockIdx.x * kBlk + threadIdx.x;
    if (e >= NR * NR) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int g = 0;
    for (; g + 3 < nparts; g += 4) {
        s0 += partials[(size_t)g * NR * NR + e];
        s1 += partials[(size_t)(g + 1) * NR * NR + e];
        s2 += partials[(size_t)(g + 2) * NR * NR + e];
        s3 += partials[(size_t)(g + 3) * NR * NR + e];
    }
    for (; g < nparts; g++) s0 += partials[(size_t)g * NR * NR + e];
    G[e] = (s0 + s1) + (s2 + s3);
}

// Rows handled together by one workgroup: kBlk / NR rows, NR threads each.
template <int NR, typename T>
__global__ __launch_bounds__(kBlk) void k_block_update(int n, double *__restrict__ X, double *__restrict__ R,
                                                       const double *__restrict__ P, const double *__restrict__ Q,
                                                       const double *__restrict__ alpha, double *__restrict__ partials,
                                                       const T *__restrict__ dinv, T *__restrict__ Z0,
                                                       T *__restrict__ RT)
{
    constexpr int RB = kBlk / NR;                   // rows per step
    __shared__ double sa[NR][NR];
    __shared__ double sp[RB][NR], sq[RB][NR];
    __shared__ double red[kBlk];
    const int t = threadIdx.x, c = t % NR, q = t / NR;
    for (int i = t; i < NR * NR; i += kBlk) sa[i / NR][i % NR] = alpha[i];
    double acc = 0.0;
    const int steps = (n + RB * gridDim.x - 1) / (RB * gridDim.x);
    for (int it = 0; it < steps; it++) {
        const int row = (it * gridDim.x + blockIdx.x) * RB + q;
        const bool in = row < n;
        const size_t o = (size_t)row * NR + c;
        __syncthreads();
        sp[q][c] = in ? P[o] : 0.0;
        sq[q][c] = in ? Q[o] : 0.0;
        __syncthreads();
        if (in) {
            double dx = 0.0, dr = 0.0;
#pragma unroll 8
            for (int a = 0; a < NR; a++) {
                dx += sp[q][a] * sa[a][c];
                dr += sq[q][a] * sa[a][c];
            }
            X[o] += dx;
            const double r = R[o] - dr;
            R[o] = r;
            acc += r * r;
            const T rt = (T)r;
            Z0[o] = dinv[row] * rt;
            if (RT) RT[o] = rt;
        }
    }
    // per-column partial: the RB rows' sums of column c in a fixed order
    red[t] = acc;
    __syncthreads();
    if (q == 0) {
        double s = 0.0;
        for (int i = 0; i < RB; i++) s += red[i * NR + c];
        partials[(size_t)blockIdx.x * NR + c] = s;
    }
}

// P = Z + P beta, or P = Z when first
template <int NR, typename TZ>
__global__ __launch_bounds__(kBlk) void k_block_direction(int n, const TZ *__restrict__ Z, double *__restrict__ P,
                                                          const double *__restrict__ beta, int first)
{
    constexpr int RB = kBlk / NR;
    __shared__ double sb[NR][NR];
    __shared__ double sp[RB][NR];
    const int t = threadIdx.x, c = t % NR, q = t / NR;
    if (!first)
        for (int i = t; i < NR * NR; i += kBlk) sb[i / NR][i % NR] = beta[i];
    const int steps = (n + RB * gridDim.x - 1) / (RB * gridDim.x);
    for (int it = 0; it < steps; it++) {
        const int row = (it * gridDim.x + blockIdx.x) * RB + q;
        const bool in = row < n;
        const size_t o = (size_t)row * NR + c;
        __syncthreads();
        sp[q][c] = in && !first ? P[o] : 0.0;
        __syncthreads();
        if (in) {
            double v = (double)Z[o];
            if (!first) {
                double d = 0.0;
#pragma unroll 8
                for (int a = 0; a < NR; a++) d += sp[q][a] * sb[a][c];
                v += d;
            }
            P[o] = v;
        }
    }
}

inline int rows_grid(int n, int nr, int cap)
{
    long long need = ((long long)n * nr + kBlk - 1) / kBlk;
    return (int)std::max(1LL, std::min<long long>(need, cap));
}

}  // namespace

#define BNR_SWITCH(nr, CALL)                           \
    switch (nr) {                                      \
    case 8: { constexpr int NR = 8; CALL; } break;     \
    case 16: { constexpr int NR = 16; CALL; } break;   \
    case 32: { constexpr int NR = 32; CALL; } break;   \
    case 64: { constexpr int NR = 64; CALL; } break;   \
    default: throw std::invalid_argument("block width must be 8, 16, 32 or 64"); \
    }

template <typename TU>
void block_gram(hipStream_t s, int nr, int n, const TU *U, const double *V, double *partials, double *G)
{
    const int g = kBlockGramParts;
    BNR_SWITCH(nr, hipLaunchKernelGGL((k_block_gram<NR, TU>), dim3(g), dim3(kBlk), 0, s, n, U, V, partials));
    BNR_SWITCH(nr, hipLaunchKernelGGL((k_block_gram_finish<NR>), dim3((NR * NR + kBlk - 1) / kBlk), dim3(kBlk), 0, s,
                                      partials, g, G));
}

template <typename T>
int block_update(hipStream_t s, int nr, int n, double *X, double *R, const double *P, const double *Q,
                 const double *alpha, double *partials, const T *dinv, T *Z0, T *RT)
{
    const int g = rows_grid(n, nr, kMaxBlocks);
    BNR_SWITCH(nr, hipLaunchKernelGGL((k_block_update<NR, T>), dim3(g), dim3(kBlk), 0, s, n, X, R, P, Q, alpha,
                                      partials, dinv, Z0, RT));
    return g;
}

template <typename TZ>
void block_direction(hipStream_t s, int nr, int n, const TZ *Z, double *P, const double *beta, bool first)
{
    const int g = rows_grid(n, nr, kMaxBlocks);
    BNR_SWITCH(nr, hipLaunchKernelGGL((k_block_direction<NR, TZ>), dim3(g), dim3(kBlk), 0, s, n, Z, P, beta,
                                      first ? 1 : 0));
}

template void block_gram<double>(hipStream_t, int, int, const double *, const double *, double *, double *);
template void block_gram<float>(hipStream_t, int, int, const float *, const double *, double *, double *);
template int block_update<double>(hipStream_t, int, int, double *, double *, const double *, const double *,
                                  const double *, double *, const double *, double *, double *);
template int block_update<float>(hipStream_t, int, int, double *, double *, const double *, const double *,
                                 const double *, double *, const float *, float *, float *);
template void block_direction<double>(hipStream_t, int, int, const double *, double *, const double *, bool);
template void block_direction<float>(hipStream_t, int, int, const float *, double *, const double *, bool);

}  // namespace auxp
