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
// evaluated with v_mfma_*_16x16x4 (A operand = the reference tables, held in
// registers for the whole kernel; B operand = Z built from LDS).
//
// The element results Y (one row of nloc values per tet) are then summed per
// dof over its (tet, local node) incidences in a fixed order -- no atomics,
// so the result is deterministic -- and the smoother or residual update is
// fused into that gather-sum pass.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "mfree.hpp"

namespace auxp {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Acc;
template <>
struct Acc<float> {
    using V = f32x4;
    static __device__ __forceinline__ V mfma(float a, float b, V c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <>
struct Acc<double> {
    using V = f64x4;
    static __device__ __forceinline__ V mfma(double a, double b, V c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

__device__ __forceinline__ bool stop(const int *done) { return done != nullptr && *done != 0; }

constexpr int kTetsPerWave = 16;
constexpr int kWaves = kBlock / 64;

// Yel[t] = K_t x_t for all tets
template <typename T, int NLOC>
__global__ __launch_bounds__(kBlock) void k_mf_element(MfView<T> op, const T *__restrict__ X, T *__restrict__ Yel,
                                                       const int *done)
{
    if (stop(done)) return;
    constexpr int KK = 6 * NLOC;                 // contraction length
    constexpr int KS = KK / 4;                   // MFMA steps (4 per step)
    constexpr int MT = (NLOC + 15) / 16;         // 16-row output tiles
    __shared__ T xs[kWaves][NLOC][kTetsPerWave];
    __shared__ T ws[kWaves][6][kTetsPerWave];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;

    // A operand: lane (row i = lane % 16, k = lane / 16) of step s holds S[16 mt + i][4 s + k]
    T areg[MT][KS];
#pragma unroll
    for (int mt = 0; mt < MT; mt++)
#pragma unroll
        for (int s = 0; s < KS; s++) {
            const int row = 16 * mt + col;
            areg[mt][s] = row < NLOC ? op.S[row * KK + 4 * s + grp] : T(0);
        }

    const long long ntiles = ((long long)op.nt + kTetsPerWave * kWaves - 1) / (kTetsPerWave * kWaves);
    for (long long bt = blockIdx.x; bt < ntiles; bt += gridDim.x) {
        const int t = (int)(bt * (kTetsPerWave * kWaves)) + wave * kTetsPerWave + col;
        const bool tv = t < op.nt;
        for (int b = grp; b < NLOC; b += 4) {
            T v = T(0);
            if (tv) {
                const int d = op.emap[(size_t)t * NLOC + b];
                if (d >= 0) v = X[d];
            }
            xs[wave][b][col] = v;
        }
        for (int k = grp; k < 6; k += 4) ws[wave][k][col] = tv ? op.w[(size_t)t * 6 + k] : T(0);
        __syncthreads();
        typename Acc<T>::V acc[MT];
#pragma unroll
        for (int mt = 0; mt < MT; mt++) acc[mt] = typename Acc<T>::V{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS; s++) {
            // B operand: lane (k = lane / 16, column = lane % 16) holds Z[4 s + k][column]
            const int kk = 4 * s + grp;
            const T bv = ws[wave][kk / NLOC][col] * xs[wave][kk % NLOC][col];
#pragma unroll
            for (int mt = 0; mt < MT; mt++) acc[mt] = Acc<T>::mfma(areg[mt][s], bv, acc[mt]);
        }
        // D: lane holds rows 4 (lane / 16) + v, v = 0..3, of column lane % 16
        if (tv) {
#pragma unroll
            for (int mt = 0; mt < MT; mt++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int a = 16 * mt + 4 * grp + v;
                    if (a < NLOC) Yel[(size_t)t * NLOC + a] = acc[mt][v];
                }
        }
        __syncthreads();
    }
}

// gather-sum of the element results per dof, fused with the update:
// MODE_RESID: out = rhs - Ax;  MODE_SWEEP: out = xin + dinv (rhs - Ax) (+ dot)
enum { MF_RESID = 0, MF_SWEEP = 1 };

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
        for (int p = op.inc_ptr[i]; p < op.inc_ptr[i + 1]; p++) s += Yel[op.inc[p]];
        T v;
        if (MODE == MF_RESID) v = (T)rhs[i] - s;
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
    int g = cap_grid(((long long)op.nt + kTetsPerWave * kWaves - 1) / (kTetsPerWave * kWaves));
    if (op.nloc == 10)
        hipLaunchKernelGGL((k_mf_element<T, 10>), dim3(g), dim3(kBlock), 0, s, op, x, Yel, done);
    else
        hipLaunchKernelGGL((k_mf_element<T, 20>), dim3(g), dim3(kBlock), 0, s, op, x, Yel, done);
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

#define MFINST(T)                                                                                             \
    template void mf_apply<T>(hipStream_t, const MfView<T> &, const T *, T *, const int *);                   \
    template void mf_resid<T>(hipStream_t, const MfView<T> &, const T *, const T *, T *, const int *);        \
    template int mf_sweep<T, T, T>(hipStream_t, const MfView<T> &, const T *, const T *, const T *, const T *, \
                                   T *, const double *, double *, const int *);

MFINST(float)
MFINST(double)
template int mf_sweep<float, double, double>(hipStream_t, const MfView<float> &, const float *, const float *,
                                             const float *, const double *, double *, const double *, double *,
                                             const int *);

}  // namespace auxp
