// Matrix-free P^k element operator on the matrix cores (gfx950 MFMA).
//
// A_h x = sum_e P_e^T K_e P_e x with K_e = kappa_e sum_pq G^e_pq M^pq.  Since
// the barycentric gradients sum to zero, G^e has zero row sums and
//     K_e = sum_{p<q} w_e,pq S^pq,   w_e,pq = -kappa_e G^e_pq,
//     S^pq = M^pp + M^qq - M^pq - M^qp,
// six reference matrices shared by every tet.  For a tile of 16 tets the
// products of all six with the gathered element vectors form one dense
// contraction Y[a][t] = sum_{(k,b)} S[a][(k,b)] Z[(k,b)][t] with
// Z[(k,b)][t] = w_t,k x_t,b: an [nloc x 6 nloc] by [6 nloc x 16] product,
// evaluated with v_mfma_*_16x16x4 (A operand = the reference tables, staged
// once per workgroup in LDS in operand lane order and read back per step;
// B operand = Z formed in registers from the lane's gathered values and its
// tet's weights).
//
// Each element result (K_t x_t)_a is written to the slot of (t, a) in an
// array ordered by dof, so the contributions to one dof are contiguous; a
// second pass sums each dof's range in a fixed order -- no atomics, so the
// result is deterministic -- with the smoother or residual update fused in.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"
#include "mfree.hpp"

namespace auxp {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Acc;
// Operand layouts (both 16x16x4 forms): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16].  Result register v of lane l holds D[row][l % 16] with
// row = 4 (l / 16) + v for FP32 and row = (l / 16) + 4 v for FP64.
template <>
struct Acc<float> {
    using V = f32x4;
    static __device__ __forceinline__ V mfma(float a, float b, V c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int grp, int v) { return 4 * grp + v; }
};
template <>
struct Acc<double> {
    using V = f64x4;
    static __device__ __forceinline__ V mfma(double a, double b, V c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int grp, int v) { return grp + 4 * v; }
};

__device__ __forceinline__ bool stop(const int *done) { return done != nullptr && *done != 0; }

constexpr int kTetsPerWave = 16;
constexpr int kDies = 8;
constexpr int kWaves = kBlock / 64;

// Y[slot(t, a)] = (K_t x_t)_a for all tets.
//
// Contraction order: the 6 nloc terms (k, b) are split into steps of four,
// step s covering k = s / NB and b = 4 (s % NB) + g for the four lane groups
// g = lane / 16 (NB = ceil(nloc / 4); b >= nloc is padding).  So lane (g, c)
// of a wave needs only the six weights of its tet c and its NB gathered
// values b = g, g+4, ..., held in registers, from which it forms its B
// operand per step; the A operand (the reference tables) comes from LDS,
// filled once per workgroup before a barrier.  Every register index below is
// a compile-time constant.
template <typename T, int NLOC>
__global__ __launch_bounds__(kBlock) void k_mf_element(MfView<T> op, const T *__restrict__ X, T *__restrict__ Yel,
                                                       const int *done)
{
    if (stop(done)) return;
    constexpr int NB = (NLOC + 3) / 4;           // gathered values per lane
    constexpr int KS = 6 * NB;                   // MFMA steps
    constexpr int MT = (NLOC + 15) / 16;         // 16-row output tiles
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, grp = lane >> 4;

    // Output tiles of 16 rows handled per pass over the tets: all of them for
    // P2/P3; one per pass for P4, whose 35-node tables (41.5 KB in FP32,
    // 83 KB in FP64) would not leave room for enough workgroups per compute
    // unit (the element map, weights and gathers are then read once per pass)
    constexpr int MG = NLOC > 20 ? 1 : MT;
    constexpr int NPASS = MT / MG;

    // A operand: lane (i = lane % 16, g) of step s holds S[16 mt + i][k nloc + b],
    // staged in LDS in that lane order (one conflict-free read per step; in
    // registers the tables would take 60 (FP32) or 120 (FP64) VGPRs at P3 and
    // cap the waves per SIMD at 4 or 2)
    __shared__ T sA[MG * KS * 64];

    // Each die (workgroups are dispatched round-robin over kDies dies, b to
    // b % kDies) takes a contiguous range of tiles, so the slots of a dof,
    // written by neighbouring tets, fill their cache lines in one L2 instead
    // of being written back in pieces from every die.  Any grid visits every
    // tile exactly once; placement affects only speed.
    const int ntiles = (op.nt + kTetsPerWave - 1) / kTetsPerWave;
    int first, end, step;
    {
        const int b = blockIdx.x, g = gridDim.x, w = (int)(threadIdx.x >> 6);
        if (g < kDies) {
            first = b * kWaves + w;
            end = ntiles;
            step = g * kWaves;
        } else {
            const int d = b % kDies, j = b / kDies;
            const int gd = (g - d + kDies - 1) / kDies;          // workgroups on die d
            const int per = (ntiles + kDies - 1) / kDies;
            first = d * per + j * kWaves + w;
            end = min(ntiles, (d + 1) * per);
            step = gd * kWaves;
        }
    }
    for (int pass = 0; pass < NPASS; pass++) {
        if (pass > 0) __syncthreads();          // every wave is done with the previous tables
        for (int i = threadIdx.x; i < MG * KS * 64; i += kBlock) {
            const int l = i % 64, s = (i / 64) % KS, mt = pass * MG + i / (64 * KS);
            const int row = 16 * mt + l % 16, k = s / NB, b = 4 * (s % NB) + l / 16;
            sA[i] = (row < NLOC && b < NLOC) ? op.S[row * 6 * NLOC + k * NLOC + b] : T(0);
        }
        __syncthreads();
        for (int tile = first; tile < end; tile += step) {
            const int t = tile * kTetsPerWave + col;
            const bool tv = t < op.nt;
            const size_t tc = tv ? (size_t)t : 0;   // loads stay unconditional (clamped), so
            T wv[6], xv[NB];                        // all of them are in flight together
            int dv[NB];
#pragma unroll
            for (int k = 0; k < 6; k++) wv[k] = op.w[tc * 6 + k];
#pragma unroll
            for (int j = 0; j < NB; j++) {
                const int b = 4 * j + grp;
                dv[j] = op.emap[tc * NLOC + (b < NLOC ? b : 0)];
                if (!tv || b >= NLOC) dv[j] = -1;
            }
            // slots of this lane's results, loaded with the element map
            int sv[MG][4];
#pragma unroll
            for (int m = 0; m < MG; m++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int a = 16 * (pass * MG + m) + Acc<T>::row(grp, v);
                    sv[m][v] = op.slot[tc * NLOC + (a < NLOC ? a : 0)];
                }
#pragma unroll
            for (int j = 0; j < NB; j++) xv[j] = X[dv[j] >= 0 ? dv[j] : 0];
            // keep the scheduler from interleaving the loads with their uses (it
            // would otherwise reuse one address register and wait on each)
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int m = 0; m < MG; m++)
#pragma unroll
                for (int v = 0; v < 4; v++)
                    if (!tv || 16 * (pass * MG + m) + Acc<T>::row(grp, v) >= NLOC) sv[m][v] = -1;
#pragma unroll
            for (int j = 0; j < NB; j++)
                if (dv[j] < 0) xv[j] = T(0);
#pragma unroll
            for (int k = 0; k < 6; k++)
                if (!tv) wv[k] = T(0);

            // B operand: lane (g, c) holds Z[(k, b)][c] = w_c,k x_c,b, formed step
            // by step (the gathers above are all in flight before the first use)
            typename Acc<T>::V acc[MG];
#pragma unroll
            for (int m = 0; m < MG; m++) acc[m] = typename Acc<T>::V{0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < KS; s++) {
                const T bv = wv[s / NB] * xv[s % NB];
#pragma unroll
                for (int m = 0; m < MG; m++) acc[m] = Acc<T>::mfma(sA[(m * KS + s) * 64 + lane], bv, acc[m]);
            }
            // D: register v of this lane holds row Acc<T>::row(grp, v) of column c
#pragma unroll
            for (int m = 0; m < MG; m++)
#pragma unroll
                for (int v = 0; v < 4; v++)
                    if (sv[m][v] >= 0) Yel[sv[m][v]] = acc[m][v];
        }
    }
}

// gather-sum of the element results per dof, fused with the update:
// MF_RESID: out = rhs - Ax;  MF_SWEEP: out = xin + dinv (rhs - Ax);  MF_PRODUCT:
// out = Ax (each + dot with rdot when DOT)
enum { MF_RESID = 0, MF_SWEEP = 1, MF_PRODUCT = 2 };

template <typename T, typename TR, typename TZ, int MODE, bool DOT>
__global__ __launch_bounds__(kBlock) void k_mf_gather(MfView<T> op, const T *__restrict__ Yel,
                                                      const T *__restrict__ xin, const T *__restrict__ dinv,
                                                      const TR *__restrict__ rhs, TZ *__restrict__ out,
                                                      const double *__restrict__ rdot, double *partials,
                                                      const int *done)
{
    if (stop(done)) return;
    double acc = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < op.n; i += gridDim.x * kBlock) {
        T s = T(0);
        for (int p = op.inc_ptr[i]; p < op.inc_ptr[i + 1]; p++) s += Yel[p];
        T v;
        if (MODE == MF_RESID) v = (T)rhs[i] - s;
        else if (MODE == MF_PRODUCT) v = s;
        else v = xin[i] + dinv[i] * ((T)rhs[i] - s);
        out[i] = (TZ)v;
        if (DOT) acc += rdot[i] * (double)(TZ)v;
    }
    if (DOT) {
        __shared__ double red[kWaves];
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double b = 0.0;
            for (int w = 0; w < kWaves; w++) b += red[w];
            partials[blockIdx.x] = b;
        }
    }
}

inline int cap_grid(long long need)
{
    if (need < 1) need = 1;
    if (need > kMaxBlocks) need = kMaxBlocks;
    return (int)need;
}

}  // namespace

template <typename T>
void mf_apply(hipStream_t s, const MfView<T> &op, const T *x, T *Yel, const int *done)
{
    // (the element kernel's clamped loads read X[0]: nothing to do without unknowns)
    if (op.n == 0 || op.nt == 0) return;
    // persistent waves, a few tiles each (the operand tables are staged once
    // per workgroup): up to 8 workgroups per compute unit at P2, 4 at P3 and
    // P4.  Each wave loads its tile's map, weights, slots and gathers, waits,
    // then runs its matrix-core chain (60 MFMA of 32 cycles at P3), so the
    // waves of a SIMD overlap one another's phases; measured (P3 32^3, P4
    // 24^3, P2 48^3 mixed solves): 1024 workgroups beat 2048 at P3 (8.77 ->
    // 8.33 ms) and P4 (15.04 -> 14.29 ms) and lose at P2 (8.82 -> 8.97 ms);
    // 512, 768 and 1536 were no better.  A software pipeline over each
    // wave's tiles (the next tile's loads and gathers issued before the
    // current contraction) was measured no faster.
    const long long tiles = ((long long)op.nt + kTetsPerWave - 1) / kTetsPerWave;
    const int cap = op.nloc == 10 ? 2048 : 1024;
    int g = (int)std::min<long long>((tiles + kWaves - 1) / kWaves, cap);
    if (g < 1) g = 1;
    if (op.nloc == 10)
        hipLaunchKernelGGL((k_mf_element<T, 10>), dim3(g), dim3(kBlock), 0, s, op, x, Yel, done);
    else if (op.nloc == 20)
        hipLaunchKernelGGL((k_mf_element<T, 20>), dim3(g), dim3(kBlock), 0, s, op, x, Yel, done);
    else
        hipLaunchKernelGGL((k_mf_element<T, 35>), dim3(g), dim3(kBlock), 0, s, op, x, Yel, done);
}

template <typename T>
void mf_resid(hipStream_t s, const MfView<T> &op, const T *Yel, const T *rhs, T *res, const int *done)
{
    int g = cap_grid(((long long)op.n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_mf_gather<T, T, T, MF_RESID, false>), dim3(g), dim3(kBlock), 0, s, op, Yel, (const T *)nullptr,
                       (const T *)nullptr, rhs, res, (const double *)nullptr, (double *)nullptr, done);
}

template <typename T, typename TR, typename TZ>
int mf_sweep(hipStream_t s, const MfView<T> &op, const T *Yel, const T *xin, const T *dinv, const TR *rhs, TZ *out,
             const double *rdot, double *partials, const int *done)
{
    int g = cap_grid(((long long)op.n + kBlock - 1) / kBlock);
    if (partials)
        hipLaunchKernelGGL((k_mf_gather<T, TR, TZ, MF_SWEEP, true>), dim3(g), dim3(kBlock), 0, s, op, Yel, xin, dinv,
                           rhs, out, rdot, partials, done);
    else
        hipLaunchKernelGGL((k_mf_gather<T, TR, TZ, MF_SWEEP, false>), dim3(g), dim3(kBlock), 0, s, op, Yel, xin, dinv,
                           rhs, out, rdot, partials, done);
    return g;
}

template <typename T>
int mf_product(hipStream_t s, const MfView<T> &op, const T *Yel, T *out, const double *rdot, double *partials,
               const int *done)
{
    int g = cap_grid(((long long)op.n + kBlock - 1) / kBlock);
    if (partials)
        hipLaunchKernelGGL((k_mf_gather<T, T, T, MF_PRODUCT, true>), dim3(g), dim3(kBlock), 0, s, op, Yel,
                           (const T *)nullptr, (const T *)nullptr, (const T *)nullptr, out, rdot, partials, done);
    else
        hipLaunchKernelGGL((k_mf_gather<T, T, T, MF_PRODUCT, false>), dim3(g), dim3(kBlock), 0, s, op, Yel,
                           (const T *)nullptr, (const T *)nullptr, (const T *)nullptr, out, rdot, partials, done);
    return g;
}

#define MFINST(T)                                                                                             \
    template void mf_apply<T>(hipStream_t, const MfView<T> &, const T *, T *, const int *);                   \
    template void mf_resid<T>(hipStream_t, const MfView<T> &, const T *, const T *, T *, const int *);        \
    template int mf_product<T>(hipStream_t, const MfView<T> &, const T *, T *, const double *, double *,       \
                               const int *);                                                                  \
    template int mf_sweep<T, T, T>(hipStream_t, const MfView<T> &, const T *, const T *, const T *, const T *, \
                                   T *, const double *, double *, const int *);

MFINST(float)
MFINST(double)
template int mf_sweep<float, double, double>(hipStream_t, const MfView<float> &, const float *, const float *,
                                             const float *, const double *, double *, const double *, double *,
                                             const int *);

}  // namespace auxp
