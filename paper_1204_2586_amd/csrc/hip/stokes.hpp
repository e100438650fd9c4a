// Kernels of the Stokes block-triangular preconditioner Q_t (Sec. 5): the
// pressure block solves M_p y = r_p by diagonally preconditioned CG, run with
// its state in device memory (CgState: the step's alpha and beta are read
// from device memory, and every launch after the stop returns at once), so
// the host enqueues a run of iterations and checks the stop flag once.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace auxp {

// x = 0, r = b, z = D^-1 b (dinv = 1 / diag M); partials[0 .. g) receive
// the workgroups' shares of b.b and partials[kMaxBlocks + 0 .. g) those of
// r.z.  Returns g.
int mass_start(hipStream_t s, int n, const double *b, const double *dinv, double *x, double *r, double *z,
               double *partials);
// q = M p (CSR, a few lanes per row) with the shares of p.q in partials;
// returns the grid size (skipped once the solve stopped).
int mass_product(hipStream_t s, const DevCsrView &M, const double *p, double *q, double *partials,
                 const CgState &st);
// one workgroup: r.r (partials[0 ..)) closes the step (iteration count, stop
// test), then r.z (partials[kMaxBlocks ..)) is recorded for the next step
void mass_finish(hipStream_t s, const double *partials, int nparts, const CgState &st);
// alpha = rz[k] / pq[k]: x += alpha p, r -= alpha q, z = D^-1 r; shares of
// r.r in partials[0 .. g) and of r.z in partials[kMaxBlocks ..).  Returns g.
int mass_update(hipStream_t s, int n, double *x, double *r, const double *p, const double *q, const double *dinv,
                double *z, double *partials, const CgState &st);
// y = -x
void vec_negate(hipStream_t s, int n, const double *x, double *y);

}  // namespace auxp
