// Device construction of the AMG hierarchy of the P^1 matrix and of the
// composite level operators of the V-cycle; see amgsetup.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <functional>
#include <vector>

#include "../host/setup.hpp"

namespace auxp {

// CSR on the device (rows sorted by column); owns its arrays unless stated
struct DCsr {
    int n = 0, m = 0, nnz = 0;
    int *ptr = nullptr, *col = nullptr;
    double *val = nullptr;
};

// Allocation interface of the caller (device memory, stream-ordered frees)
struct DevMem {
    std::function<void *(size_t)> alloc;
    std::function<void(void *)> release;
};

// The hierarchy and the composite operators as device arrays.  Levels 0 ..
// L-1; P, R, cf, down and up exist for levels 0 .. L-2.  With fuse off
// down and up are empty; dense is the cycle from level dense_first down
// (dense_first < 0: none), row-major n_{dense_first}^2.
struct DevAmg {
    std::vector<DCsr> A, P, R, down, up;
    std::vector<double *> l1;
    std::vector<int *> cf;
    double *coarse_inv = nullptr;
    int ncoarse = 0;
    double *dense = nullptr;
    int dense_first = -1, dense_n = 0;
};

// Builds the hierarchy of AH (device CSR, square, rows sorted, copied: the
// caller keeps AH) with the host setup's rules and arithmetic, so that the
// result is bitwise that of build_hierarchy, fuse_level and dense_cycle.
// fuse: also the composite operators of every level but the coarsest;
// dense_rows > 0 (with fuse): the dense cycle from the first level of at
// most dense_rows rows.  Synchronises the stream.  Throws std::runtime_error
// on a device error, a coarsest level above 8192 rows or a coarsest operator
// that is not positive definite.
void device_amg(hipStream_t s, const DCsr &AH, const SetupOptions &opt, bool fuse, int dense_rows, DevMem &mem,
                DevAmg &out);
// Host copies of the levels (and of the composite operators when present).
void download_amg(hipStream_t s, const DevAmg &d, Hierarchy &h, std::vector<FusedLevel> *fused);
void free_amg(DevMem &mem, DevAmg &d);
// b = (float) a, n entries
void to_f32_device(hipStream_t s, long long n, const double *a, float *b);
// b = 1 / a, n entries
void reciprocal_device(hipStream_t s, int n, const double *a, double *b);

// Row-split sliced ELL of a device CSR matrix, the host build_ell layout:
// slices of 64 / lanes rows, each row's entries dealt in order to its lanes
// (entry k to slot k / lanes, lane q * lanes + k % lanes of row q), a slice
// as wide as its longest row, padding (column 0, value 0).  off has one
// entry per slice plus one (slot offsets); stored = off[last].
struct DevEll {
    int *off = nullptr, *col = nullptr;
    double *val = nullptr;
    int stored = 0;
};
// lanes divides 64 (std::invalid_argument otherwise); synchronises the stream
void ell_from_csr(hipStream_t s, const DCsr &A, int lanes, DevMem &mem, DevEll &out);

}  // namespace auxp
