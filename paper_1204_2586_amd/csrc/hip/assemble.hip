// Device assembly of the coefficient-dependent operators (gfx950), for a new
// per-tet kappa on an unchanged mesh (Sec. 2, eq. (2.5): (A_h)_ij =
// sum_T kappa_T int_T grad phi_j . grad phi_i).
//
// Everything that depends on the mesh alone is set up once: the tet metrics
// G_T[p][q] = |T| grad lambda_p . grad lambda_q, the reference tables M^pq,
// the sparsity patterns and, for every entry, the list of element-matrix
// entries that sum into it in increasing tet order.  The passes here repeat
// the host assembly's arithmetic in its order (element matrix
// K_T = sum_pq (kappa_T G_T[p][q]) M^pq in (p, q) order, then each entry's sum
// in tet order from zero), with contraction into fused multiply-adds
// switched off, so the device and host operators agree bit for bit.
#include <hip/hip_runtime.h>

#include "assemble.hpp"

namespace auxp {

namespace {

constexpr int kAsmBlock = 256;

inline int asm_grid(long long n)
{
    long long g = (n + kAsmBlock - 1) / kAsmBlock;
    return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

// Ke[(t nl + a) nl + b] = sum_pq (kappa_t G_t[pq]) M[pq][a nl + b]
__global__ __launch_bounds__(kAsmBlock) void k_element_matrices(int nt, int nl, const double *__restrict__ G,
                                                                const double *__restrict__ kappa,
                                                                const double *__restrict__ M, double *__restrict__ Ke)
{
#pragma clang fp contract(off)
    const long long n2 = (long long)nl * nl, total = (long long)nt * n2;
    for (long long u = (long long)blockIdx.x * kAsmBlock + threadIdx.x; u < total;
         u += (long long)gridDim.x * kAsmBlock) {
        const int t = (int)(u / n2), i = (int)(u % n2);
        const double kap = kappa[t];
        double K = 0.0;
        for (int pq = 0; pq < 16; pq++) {
            const double g = kap * G[(size_t)t * 16 + pq];
            K += g * M[(size_t)pq * n2 + i];
        }
        Ke[u] = K;
    }
}

// val[e] = sum of src[idx[c]] over c in [ptr[e], ptr[e+1]), in order; with
// scale, src[idx[c]] is scale[idx[c] / 16] * src[idx[c]] (the P^1 stiffness:
// kappa_t G_t[pq]).  With pos, the value is also written to v64[pos[e]] and,
// rounded, v32[pos[e]].
__global__ __launch_bounds__(kAsmBlock) void k_gather_entries(long long nnz, const int *__restrict__ ptr,
                                                              const int *__restrict__ idx,
                                                              const double *__restrict__ src,
                                                              const double *__restrict__ scale,
                                                              double *__restrict__ val, const int *__restrict__ pos,
                                                              double *__restrict__ v64, float *__restrict__ v32)
{
#pragma clang fp contract(off)
    for (long long e = (long long)blockIdx.x * kAsmBlock + threadIdx.x; e < nnz;
         e += (long long)gridDim.x * kAsmBlock) {
        double v = 0.0;
        for (int c = ptr[e]; c < ptr[e + 1]; c++) {
            const int j = idx[c];
            v += scale ? scale[j / 16] * src[j] : src[j];
        }
        val[e] = v;
        if (pos) {
            v64[pos[e]] = v;
            v32[pos[e]] = (float)v;
        }
    }
}

// l1 row norms sum_e |a_e| of a CSR operator, in entry order
__global__ __launch_bounds__(kAsmBlock) void k_row_l1(int n, const int *__restrict__ ptr,
                                                      const double *__restrict__ val, double *__restrict__ l1)
{
#pragma clang fp contract(off)
    for (int i = blockIdx.x * kAsmBlock + threadIdx.x; i < n; i += gridDim.x * kAsmBlock) {
        double s = 0.0;
        for (int e = ptr[i]; e < ptr[i + 1]; e++) s += fabs(val[e]);
        l1[i] = s;
    }
}

// matrix-free weights w[t][k] = -kappa_t G_t[p_k][q_k] over the six vertex
// pairs (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
__global__ __launch_bounds__(kAsmBlock) void k_mf_weights(int nt, const double *__restrict__ G,
                                                          const double *__restrict__ kappa, double *__restrict__ w64,
                                                          float *__restrict__ w32)
{
    const int pq[6] = {1, 2, 3, 6, 7, 11};
    for (long long u = (long long)blockIdx.x * kAsmBlock + threadIdx.x; u < 6LL * nt;
         u += (long long)gridDim.x * kAsmBlock) {
        const int t = (int)(u / 6), k = (int)(u % 6);
        const double v = -kappa[t] * G[(size_t)t * 16 + pq[k]];
        w64[u] = v;
        w32[u] = (float)v;
    }
}

// Values of the block -I_R A_h of the composite restriction
// RF = [I_R, -I_R A_h] (internal numbering, n columns per block) on its fixed
// pattern: the entry of row I, column n + j, is -sum_k IR[I][k] A[k][j] over
// row I of I_R in storage order, the order of the host's row-by-row product
// (so the values equal the host's bit for bit).  A_h in external CSR
// numbering (columns sorted), perm: internal -> external dof.  One wavefront
// per row, a lane per entry; with ell_lanes > 0 the values also go to the
// row-split ELL copy (entry k of row I at slot k / L of lane (I % (64/L)) L +
// k % L of its slice).
__global__ __launch_bounds__(kAsmBlock) void k_restrict_values(
    int nrows, int n, const int *__restrict__ rf_ptr, const int *__restrict__ rf_col, const int *__restrict__ ir_ptr,
    const int *__restrict__ ir_col, const double *__restrict__ ir_val, const int *__restrict__ a_ptr,
    const int *__restrict__ a_col, const double *__restrict__ a_val, const int *__restrict__ perm,
    double *__restrict__ v64, float *__restrict__ v32, int ell_lanes, const int *__restrict__ ell_off,
    double *__restrict__ e64, float *__restrict__ e32)
{
#pragma clang fp contract(off)
    const int lane = threadIdx.x % 64;
    for (int I = blockIdx.x * (kAsmBlock / 64) + (int)(threadIdx.x / 64); I < nrows;
         I += gridDim.x * (kAsmBlock / 64)) {
        const int r0 = rf_ptr[I], r1 = rf_ptr[I + 1], c0 = ir_ptr[I], c1 = ir_ptr[I + 1];
        for (int e = r0 + lane; e < r1; e += 64) {
            const int col = rf_col[e];
            if (col < n) continue;                          // the I_R block does not change
            const int j = perm[col - n];
            double s = 0.0;
            for (int c = c0; c < c1; c++) {
                const int k = perm[ir_col[c]], end = a_ptr[k + 1];
                int lo = a_ptr[k], hi = end;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (a_col[mid] < j) lo = mid + 1;
                    else hi = mid;
                }
                if (lo < end && a_col[lo] == j) s += ir_val[c] * a_val[lo];
            }
            const double v = -s;
            v64[e] = v;
            v32[e] = (float)v;
            if (ell_lanes > 0) {
                const int rows = 64 / ell_lanes, q = e - r0;
                const long long at = (long long)ell_off[I / rows] + (long long)(q / ell_lanes) * 64 +
                                     (I % rows) * ell_lanes + q % ell_lanes;
                e64[at] = v;
                e32[at] = (float)v;
            }
        }
    }
}

}  // namespace

void element_matrices(hipStream_t s, int nt, int nl, const double *G, const double *kappa, const double *M, double *Ke)
{
    hipLaunchKernelGGL(k_element_matrices, dim3(asm_grid((long long)nt * nl * nl)), dim3(kAsmBlock), 0, s, nt, nl, G,
                       kappa, M, Ke);
}

void gather_entries(hipStream_t s, long long nnz, const int *ptr, const int *idx, const double *src,
                    const double *scale, double *val, const int *pos, double *v64, float *v32)
{
    hipLaunchKernelGGL(k_gather_entries, dim3(asm_grid(nnz)), dim3(kAsmBlock), 0, s, nnz, ptr, idx, src, scale, val,
                       pos, v64, v32);
}

void row_l1(hipStream_t s, int n, const int *ptr, const double *val, double *l1)
{
    hipLaunchKernelGGL(k_row_l1, dim3(asm_grid(n)), dim3(kAsmBlock), 0, s, n, ptr, val, l1);
}

void mf_weights(hipStream_t s, int nt, const double *G, const double *kappa, double *w64, float *w32)
{
    hipLaunchKernelGGL(k_mf_weights, dim3(asm_grid(6LL * nt)), dim3(kAsmBlock), 0, s, nt, G, kappa, w64, w32);
}

void restrict_values(hipStream_t s, int nrows, int n, const int *rf_ptr, const int *rf_col, const int *ir_ptr,
                     const int *ir_col, const double *ir_val, const int *a_ptr, const int *a_col, const double *a_val,
                     const int *perm, double *v64, float *v32, int ell_lanes, const int *ell_off, double *e64,
                     float *e32)
{
    hipLaunchKernelGGL(k_restrict_values, dim3(asm_grid(((long long)nrows + 3) / 4 * kAsmBlock)), dim3(kAsmBlock), 0, s,
                       nrows, n, rf_ptr, rf_col, ir_ptr, ir_col, ir_val, a_ptr, a_col, a_val, perm, v64, v32,
                       ell_lanes, ell_off, e64, e32);
}

}  // namespace auxp
