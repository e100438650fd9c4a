// Matrix-free P^k element operator (see mfree.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace auxp {

template <typename T>
struct MfView {
    int n;               // dofs (internal order)
    int nt;              // tets
    int nloc;            // 10 (P2), 20 (P3) or 35 (P4)
    const int *emap;     // [nt][nloc] internal dof of each local node, -1 on the boundary
    const T *w;          // [nt][6] edge weights -kappa_e G^e_pq, pairs (01,02,03,12,13,23)
    const T *S;          // [nloc][6 nloc] reference tables S[a][k nloc + b] = S^k_ab
    const int *inc_ptr;  // [n+1] incidence range of each dof in the element-result array
    const int *slot;     // [nt][nloc] position of (t, a) in that array, -1 on the boundary
};

// Y[slot[t][a]] = (K_t x_t)_a for every tet (the results of a dof are contiguous)
template <typename T>
void mf_apply(hipStream_t s, const MfView<T> &op, const T *x, T *Yel, const int *done);
// res = rhs - (sum of element results)
template <typename T>
void mf_resid(hipStream_t s, const MfView<T> &op, const T *Yel, const T *rhs, T *res, const int *done);
// out = sum of element results (= A x for the x given to mf_apply); with
// partials also sum rdot*out per block; returns the number of partials
template <typename T>
int mf_product(hipStream_t s, const MfView<T> &op, const T *Yel, T *out, const double *rdot, double *partials,
               const int *done);
// out = xin + dinv (rhs - sum of element results); with partials also sum rdot*out per block
template <typename T, typename TR, typename TZ>
int mf_sweep(hipStream_t s, const MfView<T> &op, const T *Yel, const T *xin, const T *dinv, const TR *rhs, TZ *out,
             const double *rdot, double *partials, const int *done);

}  // namespace auxp
