// Block preconditioned CG kernels (O'Leary 1980); see blockcg.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace auxp {

// workgroups (and partial matrices) of one Gram pass
constexpr int kBlockGramParts = 512;

// G = U^T V (nr x nr, row-major, FP64) for blocks U, V [n][nr]; partials
// holds kBlockGramParts * nr * nr doubles of scratch
template <typename TU>
void block_gram(hipStream_t s, int nr, int n, const TU *U, const double *V, double *partials, double *G);

// X += P alpha, R -= Q alpha (alpha nr x nr row-major), per-column partial
// sums of r.r into partials [grid][nr], Z0 = D^-1 R and (RT non-null) R in
// the preconditioner's type; returns the grid size
template <typename T>
int block_update(hipStream_t s, int nr, int n, double *X, double *R, const double *P, const double *Q,
                 const double *alpha, double *partials, const T *dinv, T *Z0, T *RT);

// P = Z + P beta (beta nr x nr), or P = Z when first
template <typename TZ>
void block_direction(hipStream_t s, int nr, int n, const TZ *Z, double *P, const double *beta, bool first);

}  // namespace auxp
