/*
 * aux.h -- C ABI of the MI355X auxiliary-space ("GAMG") preconditioned CG
 * solver for P^k (k = 2, 3, 4) Lagrange finite-element Poisson problems on
 * tetrahedral meshes.
 *
 * Method: Lee, Leng and Zhang, "A scalable auxiliary space preconditioner for
 * high-order finite element methods" (arXiv:1204.2586).
 *   - problem: -div(kappa grad u) = f in Omega, u = 0 on the boundary, in the
 *     weak form of Sec. 2, eq. (2.2)-(2.3) (the paper has kappa = 1; here kappa
 *     is one positive value per tetrahedron);
 *   - discrete system A_h u_h = f_h, (A_h)_ij = a(phi_j, phi_i),
 *     f_i = <f, phi_i> (Sec. 2, eq. (2.5));
 *   - preconditioner: Algorithm 2.1 with presmoothing (Remark 2.1): nu l1-Jacobi
 *     sweeps on A_h, restriction with I_R = I_P^T, one AMG V(1,1) cycle on the
 *     P^1 stiffness A_H, prolongation with I_P (eq. "Prol": (I_P)_ij =
 *     psi_j(x_i^h)), nu l1-Jacobi sweeps;
 *   - AMG setup (host, once): strength rule of Sec. 6.2, PMIS coarsening and
 *     extended+i interpolation (the BoomerAMG options named in Sec. 1, 6.1).
 *
 * Degrees of freedom.  A P^k node is identified by the sorted multiset of k
 * mesh vertex ids whose average is its position (vertex v: {v,..,v}; the P2
 * edge midpoint of (a,b): {a,b}; the P3 node of edge (a,b) nearer a:
 * {a,a,b}; the P3 face node: {a,b,c}).  Nodes on boundary faces (faces of a
 * single tet) are eliminated.  The remaining n_h nodes are numbered in
 * lexicographic order of their multisets; every vector of length n_h below
 * uses that order (see aux_dof_keys).  P^1 unknowns are the n_H interior
 * vertices in increasing vertex id.
 *
 * Memory.  "host" arguments are CPU memory borrowed for the call only.
 * "device" arguments are GPU memory owned by the caller, contiguous, FP64,
 * valid on the handle's device, and must not alias each other.  Device work
 * is enqueued on the handle's stream (aux_set_stream); calls return after the
 * work is enqueued unless stated otherwise.
 *
 * Errors.  Every entry point returns AUX_OK (0) or a negative AUX_E* code;
 * aux_last_error() then returns a thread-local message.  On error no output
 * is guaranteed except where stated.
 */
#ifndef AUX_H
#define AUX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AUX_OK 0
#define AUX_EINVAL -1        /* bad argument, mesh or coefficient */
#define AUX_ENOMEM -2        /* host or device allocation failed */
#define AUX_EHIP -3          /* a HIP runtime call failed */
#define AUX_ENOTCONV -4      /* CG reached maxit; the solution holds the last iterate */
#define AUX_EBREAKDOWN -5    /* CG breakdown: p.Ap <= 0 or r.z <= 0 */
#define AUX_ENAN -6          /* a non-finite value appeared in CG */
#define AUX_ESTATE -7        /* call not valid for this handle (e.g. host-only) */

#define AUX_FP64 0           /* preconditioner in FP64 */
#define AUX_MIXED 1          /* preconditioner in FP32 inside FP64 CG */

#define AUX_OP_ASSEMBLED 0   /* P^k smoother products with the assembled (sliced ELL) A_h */
#define AUX_OP_MATFREE 1     /* ... with the matrix-free element operator on the matrix cores */

typedef struct aux_handle aux_handle;

typedef struct aux_mesh {
    int32_t n_vertices;
    const double *xyz;       /* host [n_vertices][3] */
    int32_t n_tets;
    const int32_t *tets;     /* host [n_tets][4] vertex ids, any orientation */
} aux_mesh;

typedef struct aux_options {
    int nu;                  /* l1-Jacobi sweeps before and after the coarse correction (2) */
    double theta;            /* AMG strength threshold, Sec. 6.2 (0.8) */
    int coarse_max;          /* coarsest AMG level size, solved exactly (100) */
    int max_levels;          /* AMG levels at most (25) */
    uint64_t pmis_seed;      /* seed of the PMIS random measure (0) */
    int precision;           /* AUX_FP64 or AUX_MIXED (AUX_FP64) */
    int maxit;               /* CG iteration limit (1000) */
    int host_only;           /* 1: run the host setup only, no device (for tests) */
    int op;                  /* AUX_OP_ASSEMBLED or AUX_OP_MATFREE (AUX_OP_ASSEMBLED) */
    int sell_window;         /* device A_h layout: rows sorted by length within windows of this
                                many dofs; 0 (default) lets the setup time the candidate
                                layouts (and the lanes per row of the large CSR passes) on
                                the device and keep the fastest.  These choices fix the
                                internal dof order and the summation order: two handles
                                agree bitwise only if neither times its choices, i.e. both
                                are given the same window > 0 (then every choice is
                                rule-based) */
    int graph;               /* 1: replay each CG iteration as a captured HIP graph (1) */
    int sell_index16;        /* 1 (default): A_h's column indices may be stored as 16-bit offsets
                                from a base per group of 64 entries, in every 64-row slice whose
                                groups each span less than 2^16 (with sell_window 0 the setup
                                times the layout with and without and keeps the faster);
                                0: 32-bit columns.  Results are identical either way */
    int fuse_cycle;          /* 1 (default): evaluate the V-cycle with composite level operators
                                (two passes per level: b' = P^T (I - A D^-1) b and
                                y = (2 D^-1 - D^-1 A D^-1) b + (P - D^-1 A P) e) and the
                                restricted residual as I_R r - (I_R A_h) z; the same linear
                                operator B as the step-by-step cycle (0), up to rounding */
    int batch_tiles;         /* block products of A_h in the batched solve: 0 one workgroup per
                                64-row slice; 2 tiles of 16/32/64 consecutive rows whose
                                gathered block rows are staged in LDS (the largest that fits);
                                1 (default) the faster of the two, timed per block width and
                                precision (slices when sell_window > 0).  The products are
                                identical; the inner products' partial sums are grouped
                                differently (results agree to rounding) */
    int cycle_lanes;         /* storage of the V-cycle's sparse operators (fused restriction,
                                I_P, fused level operators) in the single-vector solve:
                                0 (default) the fastest of CSR with 2-32 lanes per row and
                                row-split sliced ELL with 1-32 lanes per row, timed per
                                operator (for the level operators only on levels of at least
                                8192 rows; CSR by a rule of the mean row length when
                                sell_window > 0); L in {1,2,4,8,16,32}: row-split ELL with L
                                lanes for all of them; -L: CSR with L lanes for all of them.
                                Results agree to rounding (per-row summation order) */
    int dense_cycle_rows;    /* with fuse_cycle: the V-cycle from the first level of at most
                                this many rows down to the coarsest (a fixed linear map, the
                                cycle starting from zero) is formed at setup as one dense matrix
                                T_l = N_l + Q_l T_{l+1} M_l (FP64, rounded once for FP32) and
                                applied as one dense product, in the single-vector and the
                                batched solve; 0 turns it off; at most 8192; default 2048.
                                Results agree to rounding */
    int batch_order;         /* dof order of the batched and block solves: 0 (default) the order
                                of the single-vector solve with slices round-robin over the dies;
                                1 the dofs along the Morton curve of their node positions with
                                rows sorted by length within windows of 2048 rows, each die of
                                the GPU taking a contiguous range of A_h's slices (gathered
                                block rows stay in one die's cache: fewer bytes fetched past L2,
                                measured no faster).  Results agree to rounding */
    int amg_setup;           /* where the AMG hierarchy of A_H (strength, PMIS, extended+i,
                                Galerkin products), the composite level operators, the dense
                                cycle and the coarsest inverse are built, at setup and on every
                                aux_set_kappa: 1 (default) on the device, 0 on the host.  Both
                                follow the same definitions with the same arithmetic in the same
                                order, so the hierarchies are bitwise equal; host_only handles
                                always build on the host */
    int aux_space;           /* auxiliary space of the two-level method: 1 (default) P^1 with its
                                AMG hierarchy (Algorithm 2.1); 2 (orders 3 and 4) the intermediate
                                space of Remark 6.2: P^2 on the same mesh, its problem solved by
                                one application of its own auxiliary-space preconditioner (P^2
                                l1-Jacobi around the P^1 AMG cycle, with these options), the
                                transfer the embedding of P^2 in P^k.  Batched and block solves
                                need 1 */
    double smoother_weight;  /* omega of the P^k smoother G_h = omega D_l1^-1 (1: plain l1-Jacobi,
                                the default; the AMG levels keep omega = 1).  Finite and nonzero;
                                a negative weight makes B indefinite (CG then reports
                                AUX_EBREAKDOWN), which is how the breakdown path is exercised */
    int true_residual;       /* 1: pcg_solve and pcg_solve_noalloc also compute the true
                                ||f - A_h u||_2 / ||f||_2 of the returned iterate (one more
                                product); 0 (default) leaves aux_solve_info.true_rel_residual -1 */
    int gram_schmidt;        /* passes of classical Gram-Schmidt per FGMRES step (fgmres_solve,
                                stokes_fgmres_solve): 1 (default, as PETSc's GMRES by default) or
                                2 (reorthogonalised; two more passes over the basis) */
} aux_options;

typedef struct aux_device {
    void *stream;            /* hipStream_t to enqueue on (NULL: default stream) */
    /* optional device allocator (e.g. a framework's caching allocator);
       NULL alloc means hipMalloc/hipFree */
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} aux_device;

typedef struct aux_info {
    int64_t n_h, n_H, n_tets, nnz_A, nnz_AH, nnz_IP;
    int32_t order, levels, ncoarse, precision;
    double op_complexity;    /* sum_l nnz(A_l) / nnz(A_h), counting A_h and all P^1 levels */
    double amg_complexity;   /* sum_l nnz(A_l) / nnz(A_H) over the P^1 levels */
    int64_t level_rows[32];
    int64_t level_nnz[32];
    double setup_seconds;
    int64_t device_bytes;    /* device memory held by the handle */
    int64_t stored_A;        /* stored entries of the device P^k operator, slice padding included */
    int64_t sell_window;     /* length-sorting window of the device A_h layout in use */
    int64_t level_nnz_P[32]; /* entries of the interpolation P_l from level l+1 to level l
                                (0 on the coarsest level) */
    int64_t sell_slices;     /* 64-row slices of the device A_h */
    int64_t sell_narrow_slices; /* of which store 16-bit column offsets */
    int64_t sell_index_bytes; /* bytes of the column stream one product reads: 2 per stored
                                entry of a 16-bit slice plus 4 per slot base, 4 per stored
                                entry of a 32-bit slice */
    int64_t nnz_restrict;    /* entries of the fused restriction [I_R, -I_R A_h] (0 if not fused) */
    int64_t level_nnz_down[32]; /* entries of the fused down operator of level l */
    int64_t level_nnz_up[32];   /* entries of the fused up operator of level l */
    int32_t batch_tile_rows[2]; /* block products of the last batch width, FP32 and FP64: rows
                                per LDS tile the batched autotuner chose, 0 = 64-row slices */
    double sell_tune_ms[4];  /* autotuner's time (one FP64 plus one FP32 product, ms) of the
                                candidate layouts: global sort with 16-bit offsets, global
                                sort 32-bit, 4096-row windows 16-bit, windows 32-bit; 0 for a
                                candidate not timed */
    /* Storage of the V-cycle's sparse operators in the single-vector solve:
     * L > 0 row-split sliced ELL with L lanes per row (64 / L rows per
     * wavefront), -L CSR with L lanes per row. */
    int32_t dense_cycle_level; /* first level evaluated by the dense cycle matrix, -1 if none */
    int32_t sell_split;      /* 1: the single-vector A_h passes give each slice two wavefronts
                                (32-bit layout with slices of at least 56 slots on average) */
    int32_t lanes_restrict;  /* fused restriction [I_R, -I_R A_h] (0 if not fused) */
    int32_t lanes_prolong;   /* I_P; 0: fixed-width column-major slots (its rows have 1 to 4
                                entries; the default unless cycle_lanes forces a storage) */
    int32_t lanes_down[32];  /* fused down operator of level l */
    int32_t lanes_up[32];    /* fused up operator of level l */
    double amg_setup_seconds; /* wall time of the last build of the AMG hierarchy and the
                                composite operators (at setup or by aux_set_kappa) */
    int32_t aux_space;       /* 1: P^1 auxiliary space; 2: intermediate P^2 space (the hierarchy
                                fields above are then empty: the P^2 handle holds it) */
} aux_info;

typedef struct aux_solve_info {
    int32_t iterations;      /* CG iterations (updates of u) performed */
    int32_t status;          /* AUX_OK, AUX_ENOTCONV, AUX_EBREAKDOWN or AUX_ENAN */
    double rel_residual;     /* ||r_k||_2 / ||f||_2 of the recursive residual at exit */
    double seconds;          /* wall time of the solve (host clock, includes the final sync) */
    double true_rel_residual; /* ||f - A_h u||_2 / ||f||_2 of the returned iterate when the
                                option true_residual is set (single-vector CG), else -1 */
} aux_solve_info;

/* Fill opt with the defaults listed above. */
void aux_default_options(aux_options *opt);

/* Build the discretisation and transfer on the host, the AMG hierarchy and
 * the composite operators on the device (or on the host: amg_setup, host_only),
 * and copy the solve-phase data to the device.  mesh: host arrays as described; order
 * 2, 3 or 4; kappa: host [n_tets]
 * positive values, or NULL for kappa = 1; opt: NULL for defaults; dev: NULL
 * for hipMalloc on the current device and the default stream.  On success *out owns all buffers; release it with
 * aux_destroy.  Errors: AUX_EINVAL (order, empty or degenerate mesh, vertex id
 * out of range, non-manifold face, kappa <= 0 or non-finite, coordinates not
 * finite), AUX_ENOMEM, AUX_EHIP. */
int aux_setup(const aux_mesh *mesh, int order, const double *kappa, const aux_options *opt,
              const aux_device *dev, aux_handle **out);

/* A new per-tet coefficient on the same mesh (Sec. 2, eq. (2.5) with kappa
 * one positive value per tet): kappa host [n_tets].  The device assembles
 * A_h into its existing sliced-ELL slots (FP64 and FP32), its l1 norms, the
 * P^1 stiffness A_H and the matrix-free weights, repeating the host
 * assembly's arithmetic in its order (the operators equal those of a new
 * aux_setup bit for bit); the AMG hierarchy of the new A_H (strength, PMIS,
 * extended+i, Galerkin products), the composite level operators and the
 * dense cycle are built on the device from the device A_H (amg_setup = 1;
 * on the host from a copy with amg_setup = 0, bitwise the same), and the
 * coefficient-dependent device data are rebuilt.  With amg_setup = 1 the
 * device-built operators are used where they are; their host copies (read by
 * aux_export_csr, aux_export_cf and the batched and block solves) are made
 * on first use.  The dof numbering, patterns, layouts,
 * I_P and tet metrics are kept.  The first call also builds the mesh-only
 * assembly maps (each entry's list of element-matrix contributions, about
 * nnz(A_h) * 3 int32 of device memory).  aux_info.setup_seconds then reports
 * this call's time.  Synchronises the stream.  Errors: AUX_EINVAL (kappa <= 0
 * or not finite, checked before anything changes; or an AMG hierarchy that
 * cannot be built), AUX_ENOMEM, AUX_EHIP.  After a failure past the check
 * the handle's coefficient-dependent data are gone: solves, applications
 * and precision or operator changes return AUX_ESTATE until a later
 * aux_set_kappa succeeds. */
int aux_set_kappa(aux_handle *h, const double *kappa);

/* Residual history of the handle's last single-vector CG solve (pcg_solve or
 * pcg_solve_noalloc): hist host double [max_len] receives ||r_k||_2 / ||f||_2 for
 * k = 0 .. iterations (the recursive residual the stopping test reads), at most
 * max_len values; *len = iterations + 1.  hist may be NULL to query the length.
 * After pcg_solve_noalloc the history lives in the GPU's shared scratch array and
 * is valid until the next such call on that GPU.  Errors: AUX_ESTATE before the
 * first solve. */
int aux_residual_history(aux_handle *h, double *hist, int32_t max_len, int32_t *len);

/* Release everything the handle owns (waits for its stream).  NULL is a no-op. */
int aux_destroy(aux_handle *h);

/* Change the stream later calls enqueue on. */
int aux_set_stream(aux_handle *h, void *stream);

/* Switch the preconditioner precision (AUX_FP64 or AUX_MIXED); the FP32
 * copies are made on first use. */
int aux_set_precision(aux_handle *h, int precision);

/* Choose how the preconditioner's P^k smoothing and residual products are
 * computed: AUX_OP_ASSEMBLED (sliced-ELL A_h) or AUX_OP_MATFREE (element
 * operator K_e = kappa_e sum_pq G^e_pq M^pq, Sec. 2 eq. (2.5), evaluated per
 * tet with MFMA and summed per dof).  With
 * the matrix-free operator the FP64 CG product uses it too.  The element data
 * are built on first use. */
int aux_set_operator(aux_handle *h, int op);

/* Sizes, hierarchy shape and operator complexity (host struct). */
int aux_get_info(const aux_handle *h, aux_info *info);

/* Canonical key of each dof: host int32 [n_h][order], the sorted vertex
 * multiset of the node (lexicographically increasing over the dofs). */
int aux_dof_keys(const aux_handle *h, int32_t *keys);

/* Position of each dof's node (Sec. 2: the nodes of the P^k Lagrange space):
 * host double [n_h][3], the mean of the vertices of its key, i.e.
 * sum_p alpha_p v_p / k for the node with barycentric multi-index alpha. */
int aux_dof_xyz(const aux_handle *h, double *xyz);

/* Load vector f_i = <f, phi_i> (Sec. 2) by a conical-product Gauss-Jacobi
 * rule with (order+2)^3 points per tet.  The caller evaluates f at the points
 * of tets [t0, t1) returned by aux_qpoints (host [(t1-t0)*npts][3], point q of
 * tet t at row (t-t0)*npts+q, npts = aux_qpoints_per_tet) and accumulates
 * with aux_load_accumulate (fq host [(t1-t0)*npts], b host [n_h], added to).
 * Processing all tets in any chunking gives the load vector. */
int aux_qpoints_per_tet(const aux_handle *h);
int aux_qpoints(const aux_handle *h, int32_t t0, int32_t t1, double *xyzq);
int aux_load_accumulate(const aux_handle *h, int32_t t0, int32_t t1, const double *fq, double *b);

/* Export a host copy of a matrix for inspection.  which: 0 = A_h, 1 = A_H,
 * 2 = I_P, 3 = AMG level operator A_level, 4 = AMG interpolation P_level,
 * 5 = Stokes B, 6 = pressure mass matrix M_p (after aux_stokes_setup),
 * 7 = composite down operator P^T (I - A D^-1) of level `level`, 8 = composite
 * up operator [2 D^-1 - D^-1 A D^-1, P - D^-1 A P] of level `level` (fuse_cycle;
 * device handles), 9 = the P^k <- P^2 transfer I_2 (aux_space 2).
 * With ptr == NULL only shape[3] = {rows, cols, nnz} is written; otherwise
 * ptr host int32 [rows+1], col int32 [nnz], val double [nnz] receive the CSR. */
int aux_export_csr(const aux_handle *h, int which, int level, int64_t *shape, int32_t *ptr,
                   int32_t *col, double *val);
/* C/F splitting of an AMG level (host int32 [rows]: +1 coarse, -1 fine). */
int aux_export_cf(const aux_handle *h, int level, int32_t *cf);

/* z = B r, one application of the preconditioner (device r, z [n_h]). */
int aux_apply(aux_handle *h, const double *r, double *z);

/* Preconditioned CG on A_h u = f (Sec. 2, eq. (2.5)).  f: device [n_h] load
 * vector; u: device [n_h], initial guess in, solution out.  Stops when
 * ||f - A_h u_k||_2 (recursive residual) <= tol ||f||_2, or after maxit
 * iterations (tol = 0 runs exactly maxit).  maxit <= 0 uses the handle's
 * option.  Synchronises the stream; info (host, may be NULL) receives the
 * iteration count and final relative residual.  Returns AUX_OK,
 * AUX_ENOTCONV, AUX_EBREAKDOWN or AUX_ENAN (u then holds the last iterate). */
int pcg_solve(aux_handle *h, const double *f, double *u, double tol, int maxit, aux_solve_info *info);

/* pcg_solve without any allocation, for callers that cannot allocate device
 * memory (tight serving loops, code that forbids hipMalloc/hipFree or
 * allocating library calls).  Same arguments, iterations, result and status
 * as pcg_solve (the same kernels in the same order; every launch enqueued
 * directly, no HIP graph).  The solve's scratch memory (reduction partials,
 * CG state and per-iteration histories) is a fixed 128.1 KiB array in the
 * library, one copy per GPU, held until the process ends; concurrent calls
 * on one GPU (any handles) race on it and must be serialised by the caller.
 * maxit (after the <= 0 default) must be at most 4094 (AUX_EINVAL).  The
 * handle's data for the current precision and operator must exist: they are
 * built by aux_setup, aux_set_precision and aux_set_operator (AUX_ESTATE
 * otherwise).  Kernel timing (aux_profile) is not recorded by this call. */
int pcg_solve_noalloc(aux_handle *h, const double *f, double *u, double tol, int maxit, aux_solve_info *info);

/* nrhs independent CG solves in lock-step sharing every sparse-matrix pass.
 * F, U: device row-major [n_h][nrhs] (column j is right-hand side j).  Each
 * column follows exactly the single-right-hand-side algorithm and stops on
 * its own criterion.  infos: host [nrhs] or NULL.  Returns the worst status.
 * The device blocks are n_h x w with w = nrhs rounded up to a power of two
 * (at least 8); the block kernels address them with 32-bit byte offsets, so
 * n_h * w * 8 bytes must not exceed 4 GiB (AUX_EINVAL otherwise: solve fewer
 * right-hand sides per call). */
int pcg_solve_batched(aux_handle *h, const double *F, double *U, int nrhs, double tol, int maxit,
                      aux_solve_info *infos);

/* Block preconditioned CG (O'Leary, "The block conjugate gradient algorithm
 * and related methods", 1980) on A_h X = F for nrhs (1 to 64) right-hand
 * sides with the preconditioner B of every column: every column's iterate
 * lies in the sum of the block Krylov spaces of all columns, so the block
 * converges in at most as many steps as its slowest column does alone.
 * With gamma = Z^T R and delta = P^T A_h P (nrhs x nrhs):
 *   alpha = delta^{-1} gamma, X += P alpha, R -= A_h P alpha, Z = B R,
 *   beta = gamma^{-1} gamma_new, P = Z + P beta.
 * F, U: device row-major [n_h][nrhs]; U is the initial guess in and the
 * block out.  Stops when every column with f_j != 0 has ||r_j||_2 <= tol
 * ||f_j||_2 (recursive residual), after maxit steps (AUX_ENOTCONV), on a
 * non-positive pivot of delta or gamma (AUX_EBREAKDOWN: the columns of the
 * residual block became linearly dependent, e.g. a zero or repeated
 * right-hand side, or a tolerance near rounding) or a non-finite value
 * (AUX_ENAN).  infos (host [nrhs] or NULL): the common step count and each
 * column's relative residual.  Synchronises the stream a few times per step
 * (the nrhs x nrhs solves run on the host).  The 4 GiB block limit of
 * pcg_solve_batched applies. */
int pcg_solve_block(aux_handle *h, const double *F, double *U, int nrhs, double tol, int maxit,
                    aux_solve_info *infos);

/* Flexible GMRES(restart) on A_h x = b with the same preconditioner B, the
 * Krylov method of the paper's experiments (Sec. 6.1; Saad's flexible
 * variant, right preconditioning, so B in FP32 is allowed to vary).  b, x:
 * device [n_h]; x is the initial guess in and the solution out.  Stops when
 * the rotated residual norm of the least-squares problem is
 * <= tol ||b - A_h x_0||_2 (with a zero right-hand side and a random initial
 * guess, the paper's protocol, this is its relative residual), or after maxit
 * Arnoldi steps (maxit <= 0 uses the handle's option).  restart in [1, 128];
 * the basis takes (2 restart + 1) n_h doubles of device memory, kept until
 * the handle is destroyed.  history (host, may be NULL) receives ||r_0||
 * and then the rotated residual norm after every step (iterations + 1
 * values, at most maxit + 1).  info->iterations counts Arnoldi steps and
 * info->rel_residual is the true ||b - A_h x||_2 / ||r_0||_2 at exit.
 * Synchronises the stream once per step.  Returns AUX_OK, AUX_ENOTCONV (x is
 * the last iterate), AUX_ENAN or AUX_EINVAL. */
int fgmres_solve(aux_handle *h, const double *b, double *x, double tol, int restart, int maxit, double *history,
                 aux_solve_info *info);

/* Stokes system of the Hood-Taylor pair P^k - P^{k-1} (Sec. 5, the paper's
 * second test problem; k = the handle's order, 2, 3 or 4) on the handle's
 * mesh:
 *     [A  B^T] [u]   [f]
 *     [B   0 ] [p] = [g],   A = diag(A_h, A_h, A_h),
 * velocity u = (u_0, u_1, u_2) on the handle's dofs (zero on the boundary;
 * A_h with the handle's kappa as viscosity), pressure p in the continuous
 * P^{k-1} space on every node of order k-1 (no boundary condition; constants
 * are the null space of B^T), B_{q,(c,i)} = -int psi_q dphi_i/dx_c (the
 * discrete -div) and M_p the pressure mass matrix (int psi_q psi_r), both
 * integrated exactly.  A Stokes vector is a device double array
 * [3 n_h + n_p]: u_0, u_1, u_2 in the dof order of aux_dof_keys, then p in
 * the order of its node keys (k-1 sorted vertex ids, lexicographic; for
 * P^1 the vertex order, n_p = n_v).
 *
 * aux_stokes_setup builds B and M_p (host assembly, then a device copy of B,
 * B^T and M_p, about 24 nnz(B) bytes) and writes n_p to *n_p (may be NULL);
 * on a host-only handle it builds the host matrices only (aux_export_csr
 * which = 5 is B, 6 is M_p afterwards).  The other calls run it on first
 * use.  Errors: AUX_ENOMEM, AUX_EHIP. */
int aux_stokes_setup(aux_handle *h, int32_t *n_p);
/* Node key of each pressure unknown: host int32 [n_p][k-1] (after
 * aux_stokes_setup; AUX_ESTATE before). */
int aux_stokes_pressure_keys(const aux_handle *h, int32_t *keys);
/* y = [A B^T; B 0] x in FP64 (device x, y [3 n_h + n_p]; the handle's
 * operator form for A_h). */
int stokes_apply_operator(aux_handle *h, const double *x, double *y);
/* z = Q_t r, the block triangular preconditioner of Sec. 5 with the Schur
 * complement replaced by M_p and A^{-1} by the auxiliary-space preconditioner
 * B (one application per velocity component, the handle's precision):
 *     z_p = -M_p^{-1} r_p,   z_c = B (r_c - (B^T z_p)_c),
 * with M_p^{-1} r_p computed by diagonally preconditioned CG from zero until
 * ||r_p - M_p x|| <= 1e-6 ||r_p|| (at most 200 steps).  Device r, z
 * [3 n_h + n_p], not aliased.  mass_steps (host, may be NULL) receives the CG
 * step count.  Synchronises the stream (the mass CG's stop test). */
int stokes_apply_qt(aux_handle *h, const double *r, double *z, int32_t *mass_steps);
/* Flexible GMRES(restart) on the Stokes system with Q_t as the right
 * preconditioner (the paper's Stokes solver: FGMRES with Q_t).  Arguments,
 * stopping rule, history and statuses as fgmres_solve, on vectors
 * [3 n_h + n_p]; the basis takes (2 restart + 1) (3 n_h + n_p) doubles of
 * device memory, kept until the handle is destroyed.  A right-hand side
 * with a pressure part orthogonal to the constants and a compatible
 * velocity part has solutions unique up to a constant pressure. */
int stokes_fgmres_solve(aux_handle *h, const double *b, double *x, double tol, int restart, int maxit,
                        double *history, aux_solve_info *info);

/* y = A_h x (device x, y [n_h]), FP64. */
int aux_matvec(aux_handle *h, const double *x, double *y);

/* Per-tet derivative of a functional L(u(kappa)) with respect to log kappa,
 * g_t = -lam_t^T K_t u_t, where A_h lam = dL/du (the adjoint solution), K_t
 * the element stiffness of tet t and lam_t, u_t its local values (zero on
 * the boundary).  u, lam: device [n_h]; g: device [n_tets]. */
int aux_kappa_grad(aux_handle *h, const double *u, const double *lam, double *g);

/* Kernel timing.  Categories of timed launches: */
#define AUX_PROF_PK_FIRST 0   /* first two fused P^k l1-Jacobi sweeps from zero */
#define AUX_PROF_PK_SWEEP 1   /* P^k l1-Jacobi sweep (preconditioner precision in and out) */
#define AUX_PROF_PK_LAST 2    /* last P^k sweep, writes the FP64 result and reduces r.z */
#define AUX_PROF_PK_RESID 3   /* P^k residual before restriction */
#define AUX_PROF_COARSE 4     /* restriction + AMG V-cycle + prolongation */
#define AUX_PROF_CG_SPMV 5    /* CG product q = A_h p with p.q */
#define AUX_PROF_APPLY 6      /* one whole preconditioner application */
#define AUX_PROF_NCAT 7
/* With enable = 1, later preconditioner and CG calls record a HIP event pair
 * on the handle's stream around each launch of the categories above (launches
 * enqueued after convergence that returned at once are not counted).  With
 * enable = 2 only whole applications (AUX_PROF_APPLY) are recorded, so their
 * times carry no event records between the application's own launches.
 * Resets the sums.  enable = 0 stops recording (AUX_EINVAL for other values). */
int aux_profile(aux_handle *h, int enable);
/* Launch count and summed elapsed milliseconds of a category since the last
 * aux_profile call (synchronises the stream). */
int aux_profile_read(aux_handle *h, int category, int64_t *launches, double *ms);

/* Message of the last error on this thread ("" if none). */
const char *aux_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AUX_H */
