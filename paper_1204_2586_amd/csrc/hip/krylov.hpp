// Vector kernels of the flexible GMRES(m) outer iteration (FP64).
#pragma once

#include <hip/hip_runtime.h>

namespace auxp {

constexpr int kKrylovBlocks = 1024;   // workgroups (and partial sums per vector) of one pass
constexpr int kMaxRestart = 128;      // basis vectors of one cycle at most

// out[v] = V_v . w for v < nv (V_v = V + v * ld); partials holds
// kKrylovBlocks * nv doubles.  Sums are in a fixed order (deterministic).
void multi_dot(hipStream_t s, int n, int nv, const double *V, long long ld, const double *w, double *partials,
               double *out);
// w += sign * sum_v c[v] V_v (c on the device); with nrm2 non-null also
// nrm2[0] = w.w of the result
void multi_axpy(hipStream_t s, int n, int nv, const double *V, long long ld, const double *c, double sign, double *w,
                double *partials, double *nrm2);
// out = w / sqrt(nrm2[0]) (out = 0 when nrm2[0] is 0); out may equal w
void scale_unit(hipStream_t s, int n, const double *w, const double *nrm2, double *out);
// y = a - y (a residual from a product written into y)
void sub_from(hipStream_t s, int n, const double *a, double *y);

}  // namespace auxp
