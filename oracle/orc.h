/*
 * Test infrastructure: the CPU oracle of the auxiliary-space ("GAMG")
 * preconditioned CG method of Lee, Leng and Zhang (arXiv:1204.2586).
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * call this code.  It is plain, single-threaded FP64 C with no blocking or
 * fusion, written so that each step can be checked against the paper by eye.
 * It shares no code with the GPU library.
 */
#ifndef ORC_H
#define ORC_H

#include <stddef.h>
#include <stdint.h>

/* compressed sparse rows: n rows, m columns */
typedef struct {
    int n, m;
    int *ptr;     /* [n+1] */
    int *col;     /* [nnz], sorted within each row */
    double *val;  /* [nnz] */
} ocsr;

typedef struct {
    ocsr A;        /* level operator */
    double *dl1;   /* l1 row norms sum_j |a_ij| */
    int *cf;       /* +1 coarse, -1 fine (not set on the coarsest level) */
    int *round;    /* PMIS round in which each point was decided (0: before the first) */
    ocsr P;        /* interpolation n x nc (not set on the coarsest level) */
    ocsr R;        /* P transposed */
    int nc;
} olevel;

#define ORC_MAX_LEVELS 32

typedef struct orc_s {
    /* mesh (copied) */
    int k, nloc, nv, nt;
    double *xyz;     /* [nv][3] */
    int *tets;       /* [nt][4] */
    double *kappa;   /* [nt] */

    /* P^k nodes: global node g has key node_key[g*k .. g*k+k-1], a sorted
       multiset of k vertex ids; nodes are numbered in lexicographic key order */
    int nnode;
    int *node_key;
    int *tet_node;   /* [nt][nloc] global node of each local node */
    int *node_dof;   /* [nnode] interior dof index or -1 (Dirichlet) */
    int ndof;        /* n_h */

    /* P^1 (auxiliary space) */
    int *vert_dof;   /* [nv] interior vertex index or -1 */
    int nH;          /* n_H */

    ocsr A;          /* A_h on interior dofs */
    double *dl1;     /* l1 row norms of A_h */
    ocsr AH;         /* P1 stiffness on interior vertices */
    ocsr IP;         /* n_h x n_H transfer, I_R = IP^T */
    ocsr IR;

    /* AMG hierarchy on AH */
    int nlev;
    olevel lev[ORC_MAX_LEVELS];
    double *chol;    /* dense Cholesky factor of the coarsest operator (lower, row-major) */
    int ncoarse;

    /* Stokes (Sec. 5), Hood-Taylor P^k-P^{k-1}: pressure on every node of
       order k-1, node keys of k-1 sorted vertex ids in lexicographic order */
    int np;          /* pressure unknowns; 0 until orc_stokes_setup */
    int nlp;         /* local pressure nodes per tet */
    int *pnode_key;  /* [np][k-1] */
    int *ptet_node;  /* [nt][nlp] pressure node of each local pressure node */
    ocsr Bdiv;       /* np x 3 ndof discrete divergence, columns component-major */
    ocsr BdivT;
    ocsr Mp;         /* np x np pressure mass matrix */

    /* intermediate auxiliary space (Remark 6.2), after orc_nested_transfer:
       the P^2 problem on the same mesh (not owned, its AMG set up) in place
       of P^1, and the transfer I_2 (n_h x n_2, the embedding of P^2 in P^k)
       with its transpose */
    const struct orc_s *aux2;
    ocsr I2, I2T;

    /* options */
    double omega;    /* weight of the P^k smoother G_h = omega D_l1^{-1} (1 unless set) */
    double theta;
    int nu, coarse_max, max_levels;
    uint64_t seed;
} orc;

/* fem */
int orc_local_multi_indices(int k, int *alpha /* [nloc][4] */);
double orc_basis(int k, const int *alpha, const double *lam);
void orc_basis_dlam(int k, const int *alpha, const double *lam, double *d /* [4] */);
int orc_gauss_jacobi(int m, int a, double *x, double *w);   /* on [0,1], weight (1-x)^a */
int orc_tet_rule(int m, double *lam /* [m^3][4] */, double *w /* [m^3] */);
int orc_build_mesh_dofs(orc *o);
int orc_assemble(orc *o);

/* sparse helpers */
void ocsr_free(ocsr *a);
int ocsr_transpose(const ocsr *a, ocsr *t);
int ocsr_matmul(const ocsr *a, const ocsr *b, ocsr *c);
int ocsr_from_triplets(int n, int m, size_t cnt, const int *ri, const int *ci, const double *v, ocsr *out);

/* amg */
int orc_amg_setup(orc *o);

/* Stokes: divergence and pressure mass matrix (orc_fem.c) */
int orc_stokes_assemble(orc *o);

/* intermediate auxiliary space: I_2 from the P^2 problem o2 on the same mesh (orc_fem.c) */
int orc_nested_transfer(orc *o, const orc *o2);
double orc_pressure_l2_error(const orc *o, int m, const double *pq, const double *ph);

/* flexible GMRES(m) on vectors of length n with an operator and a
   preconditioner given as callbacks (orc_solve.c) */
typedef void (*orc_vecop)(const orc *o, void *ctx, const double *in, double *out);
int orc_fgmres_core(const orc *o, int n, orc_vecop op, orc_vecop prec, void *ctx, const double *b, double *x,
                    double tol, int m, int maxit, int *iters, double *relres, double *hist);

#endif
