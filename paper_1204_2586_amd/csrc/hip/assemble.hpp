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

}  // namespace auxp
