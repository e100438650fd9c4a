// Device assembly of the coefficient-dependent operators; see assemble.hip.
#pragma once

#include <hip/hip_runtime.h>

namespace auxp {

// Ke [nt][nl][nl] = kappa_t sum_pq G_t[pq] M^pq (G [nt][16], M [16][nl*nl])
void element_matrices(hipStream_t s, int nt, int nl, const double *G, const double *kappa, const double *M, double *Ke);
// val[e] = sum over the entry's list of src[j] (times scale[j / 16] when
// scale is set), in list order; with pos also v64[pos[e]] and v32[pos[e]]
void gather_entries(hipStream_t s, long long nnz, const int *ptr, const int *idx, const double *src,
                    const double *scale, double *val, const int *pos, double *v64, float *v32);
// l1 row norms of a CSR operator
void row_l1(hipStream_t s, int n, const int *ptr, const double *val, double *l1);
// matrix-free weights -kappa_t G_t[p][q] over the six vertex pairs
void mf_weights(hipStream_t s, int nt, const double *G, const double *kappa, double *w64, float *w32);
// values of the block -I_R A_h of RF = [I_R, -I_R A_h] on its pattern (rows
// nrows = n_H, n columns per block, internal numbering) from I_R (internal)
// and A_h (external CSR, perm: internal -> external), in the order of the
// host product; also into RF's row-split ELL copy when ell_lanes > 0
void restrict_values(hipStream_t s, int nrows, int n, const int *rf_ptr, const int *rf_col, const int *ir_ptr,
                     const int *ir_col, const double *ir_val, const int *a_ptr, const int *a_col, const double *a_val,
                     const int *perm, double *v64, float *v32, int ell_lanes, const int *ell_off, double *e64,
                     float *e32);

}  // namespace auxp
