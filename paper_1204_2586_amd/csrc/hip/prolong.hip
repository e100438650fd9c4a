// The prolongation z += I_P e_H of Step 2 of Algorithm 2.1 (gfx950) in its
// fixed-width form: each P^k node takes the coarse correction of the P^1
// functions at its key's vertices, so a row of I_P has at most four entries;
// they are kept in column-major slots (slot k of row i at k n + i, padding
// value 0 at column 0).  A row's loads depend on nothing but its index, so
// the chain per row is the slots, then the gathered e_H, then z: one
// dependent load fewer than a layout with row offsets.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdexcept>

#include "kernels.hpp"

namespace auxp {

namespace {

template <typename T, int W>
__global__ __launch_bounds__(kBlock) void k_fixed_add(int n, const int *__restrict__ col, const T *__restrict__ val,
                                                      const T *__restrict__ e, T *__restrict__ z, const int *done)
{
    if (done != nullptr && *done != 0) return;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < W; k++) acc += val[(size_t)k * n + i] * e[col[(size_t)k * n + i]];
        z[i] += acc;
    }
}

}  // namespace

template <typename T>
void fixed_matvec_add(hipStream_t s, int n, int w, const int *col, const T *val, const T *e, T *z, const int *done)
{
    const long long need = ((long long)n + kBlock - 1) / kBlock;
    const int g = (int)std::max(1LL, std::min<long long>(need, kMaxBlocks));
    switch (w) {
    case 1: hipLaunchKernelGGL((k_fixed_add<T, 1>), dim3(g), dim3(kBlock), 0, s, n, col, val, e, z, done); break;
    case 2: hipLaunchKernelGGL((k_fixed_add<T, 2>), dim3(g), dim3(kBlock), 0, s, n, col, val, e, z, done); break;
    case 3: hipLaunchKernelGGL((k_fixed_add<T, 3>), dim3(g), dim3(kBlock), 0, s, n, col, val, e, z, done); break;
    case 4: hipLaunchKernelGGL((k_fixed_add<T, 4>), dim3(g), dim3(kBlock), 0, s, n, col, val, e, z, done); break;
    default: throw std::invalid_argument("fixed_matvec_add: 1 to 4 entries per row");
    }
}

template void fixed_matvec_add<double>(hipStream_t, int, int, const int *, const double *, const double *, double *,
                                       const int *);
template void fixed_matvec_add<float>(hipStream_t, int, int, const int *, const float *, const float *, float *,
                                      const int *);

}  // namespace auxp
