// Host-side setup of the auxiliary-space preconditioner: P^k degrees of
// freedom, finite-element assembly, the P^k <- P^1 transfer and the AMG
// hierarchy on the P^1 matrix.  Runs once per (mesh, order, kappa); the
// solve phase on the GPU only consumes the arrays produced here.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace auxp {

struct Csr {
    int n = 0, m = 0;
    std::vector<int> ptr{0};
    std::vector<int> col;
    std::vector<double> val;
    int64_t nnz() const { return ptr.empty() ? 0 : ptr.back(); }
};

struct AmgLevel {
    Csr A;                    // level operator
    std::vector<double> l1;   // sum_j |a_ij|
    std::vector<int> cf;      // +1 coarse / -1 fine (empty on the coarsest level)
    Csr P;                    // interpolation n x nc
    Csr R;                    // P^T
};

struct SetupOptions {
    double theta = 0.8;
    int coarse_max = 100;
    int max_levels = 25;
    uint64_t seed = 0;
};

struct Discretization {
    int k = 0, nloc = 0, nv = 0, nt = 0;
    std::vector<double> xyz;     // [nv][3]
    std::vector<int> tets;       // [nt][4]
    std::vector<double> kappa;   // [nt]

    int ndof = 0;                // interior P^k nodes (n_h)
    int nH = 0;                  // interior vertices (n_H)
    std::vector<int32_t> keys;   // [ndof][k] sorted vertex multiset of each dof
    std::vector<int> tet_dof;    // [nt][nloc] dof of each local node, -1 on the boundary
    std::vector<int> vert_dof;   // [nv] P^1 index or -1

    Csr A;                       // A_h
    std::vector<double> l1;      // l1 row norms of A_h
    Csr AH;                      // P^1 stiffness
    Csr IP;                      // n_h x n_H
    Csr IR;                      // I_P^T
};

struct Hierarchy {
    std::vector<AmgLevel> levels;
    std::vector<double> coarse_inv;   // dense inverse of the coarsest operator, row-major
    int ncoarse = 0;
};

// local multi-indices of the P^k tet (|alpha| = k), lexicographic
std::vector<int> multi_indices(int k);

// For each entry e of the operator A assembled from the element map emap
// [nt][nl] (-1 = eliminated): the element-matrix entries (t * nl + a) * nl + b
// that sum into it, in increasing t, the order of the host assembly
// (entry e takes idx[ptr[e] .. ptr[e+1])).  Depends on the mesh only.
void assembly_map(const Csr &A, int nt, int nl, const int *emap, std::vector<int> &ptr, std::vector<int> &idx);

// Throws std::invalid_argument on bad input.
void build_discretization(Discretization &d, int nv, const double *xyz, int nt, const int32_t *tets,
                          int k, const double *kappa);
void build_hierarchy(const Csr &AH, const SetupOptions &opt, Hierarchy &h);

// reference tables M^pq_ab = (1/|T|) int dphi_a/dlam_p dphi_b/dlam_q, [4][4][nloc][nloc]
const std::vector<double> &stiffness_tables(int k);
// element stiffness of tet t (kappa included) = kappa * sum_pq G_pq M^pq
void element_stiffness(const Discretization &d, int t, double *K);
// gradient inner products |T| grad(lam_p).grad(lam_q) (4x4) of tet t, returns |det J|
double tet_metric(const double *X0, const double *X1, const double *X2, const double *X3,
                  double G[4][4]);
// barycentric gradients g[p] = grad lam_p of a tet, returns the signed det J
double tet_gradients(const double *X0, const double *X1, const double *X2, const double *X3, double g[4][3]);
// Reference tables of the Hood-Taylor pair P^k - P^{k-1} (psi_p the P^{k-1}
// basis, phi_a the P^k basis, exact integration of barycentric monomials):
//   C[q][a][p] = (1/|T|) int_T psi_p dphi_a/dlam_q   ([4][nloc][nlp])
//   Mp[p][r]   = (1/|T|) int_T psi_p psi_r           ([nlp][nlp])
void stokes_tables(int k, std::vector<double> &C, std::vector<double> &Mp);

// Hood-Taylor P^k - P^{k-1} Stokes blocks (stokes.cpp), k = 2, 3, 4: the
// pressure on every node of order k-1 (no boundary condition), numbered by
// its key (k-1 sorted vertex ids) in lexicographic order (vertex order for
// P^1), keys returned in pkeys [np][k-1]; velocity on the interior P^k dofs,
// component blocks c = 0, 1, 2 of n_h columns each:
//   B   (n_p x 3 n_h):  B_{p, c n_h + i} = -int psi_p dphi_i/dx_c  (-div)
//   M_p (n_p x n_p):    (M_p)_pq = int psi_p psi_q
// Entries are summed in tet order.  Throws std::invalid_argument for other k.
void build_stokes(const Discretization &d, Csr &B, Csr &Mp, std::vector<int32_t> &pkeys);

// load vector by the conical-product rule with k+2 points per direction
int load_rule_points(int k);                               // points per tet
void quadrature_points(const Discretization &d, int t0, int t1, double *out);
void accumulate_load(const Discretization &d, int t0, int t1, const double *fq, double *b);

Csr transpose(const Csr &a);

// The embedding of P^2 in P^k on one mesh (the intermediate auxiliary space
// of Remark 6.2): n_h(k) x n_h(2), rows and columns in the two
// discretisations' dof orders.  Throws std::invalid_argument if d2 is not
// the order-2 discretisation of the same mesh.
Csr p2_transfer(const Discretization &d, const Discretization &d2);

// Composite operators of the preconditioner (fuse.cpp).  For an AMG level
// with D = diag(l1):  down = P^T (I - A D^-1)  (n_{l+1} x n_l);
// up = [2 D^-1 - D^-1 A D^-1,  P - D^-1 A P]  (n_l x (n_l + n_{l+1})), so
// that one V(1,1) cycle from zero is  b' = down b,  y = up [b; e].
struct FusedLevel {
    Csr down, up;
};
FusedLevel fuse_level(const AmgLevel &L);
// [I_R, -I_R A] (n_H x 2 n_h): the restricted residual I_R (r - A z) of [r; z]
Csr fuse_restriction(const Csr &IR, const Csr &A);
// The cycle below and including level l0, from a zero guess, as one dense
// matrix: y_l0 = T b_l0 with T = coarse_inv on the coarsest level and
// T_l = N_l + Q_l T_{l+1} M_l above it (M_l = fused[l].down, [N_l Q_l] =
// fused[l].up).  Row-major n_l0 x n_l0, formed in FP64.
std::vector<double> dense_cycle(const std::vector<FusedLevel> &fused, const Hierarchy &H, size_t l0);

}  // namespace auxp

namespace auxp {

// Sliced ELLPACK in an internal row order (see formats.cpp).
struct Sell {
    int n = 0, slice = 64, nslices = 0;
    std::vector<int> perm;        // internal row -> original row
    std::vector<int> iperm;       // original row -> internal row
    std::vector<int> slice_off;   // [nslices+1]
    std::vector<int> col;         // internal column numbers
    std::vector<double> val;
    // Column indices as stored on the device.  A slice is narrow when, for
    // every slot t of it (the t-th group of `slice` consecutive entries), the
    // columns of the slot span less than 2^16: then entry e has column
    // base[t] + off[e] and mode[s] = 0.  Otherwise mode[s] = ~w and the
    // slice's entries have 32-bit columns wide[w + (e - slice_off[s])].
    std::vector<int> mode;        // [nslices]
    std::vector<int> base;        // [slice_off[nslices] / slice]
    std::vector<uint16_t> off;    // [slice_off[nslices]]
    std::vector<int> wide;        // columns of the wide slices
    int max_width = 0;            // longest slice, in slots
};

// Row-split sliced ELL for the V-cycle's sparse operators: slices of
// 64 / lanes consecutive rows, one wavefront each; entry k of the slice's
// row q sits in slot k / lanes at lane q * lanes + k % lanes, so every slot
// is 64 consecutive entries (coalesced loads) and a row's lanes add their
// partial sums at the end.  Each slice is padded to its longest row with
// column 0 and value 0.  Rows keep their order.
struct Ell {
    int n = 0, lanes = 1, nslices = 0;
    std::vector<int> slice_off;   // [nslices+1], multiples of 64
    std::vector<int> col;
    std::vector<double> val;
};
void build_ell(const Csr &A, int lanes, Ell &out);

// Row tiles for products with a block of vectors (batched solve).  Tile t
// holds `tile` consecutive rows of A in the original order (neighbouring
// dofs, which share most of their columns); ucols lists the distinct columns
// of the tile (in the internal numbering), and each entry stores the 16-bit
// position of its column in that list, so a workgroup can stage the gathered
// block rows once per tile.  Rows and columns are renumbered with iperm.
struct Tiles {
    int n = 0, tile = 0, ntiles = 0;
    std::vector<int> rows;        // [ntiles*tile] internal row of each tile row, -1 past the end
    std::vector<int> row_ptr;     // [ntiles*tile + 1] entry offsets, tile rows in order
    std::vector<uint16_t> lidx;   // per entry: position of its column in the tile's list
    std::vector<double> val;
    std::vector<int> col_off;     // [ntiles+1] offsets into ucols
    std::vector<int> ucols;       // distinct internal columns of each tile, sorted
    int max_cols = 0, max_entries = 0;
};
void build_tiles(const Csr &A, const std::vector<int> &iperm, int tile, Tiles &out);

// Rows sorted by decreasing length (stably) within windows of `window` rows;
// index16 = false stores every slice with plain 32-bit columns.  With
// permute_cols the columns are renumbered like the rows (a square operator
// acting on vectors in the internal order); otherwise only the rows move
// (results go to row perm[r]).
void build_sell(const Csr &A, int slice, int window, bool index16, Sell &out, bool permute_cols = true);
// rows of A in the order perm (row r of the result is row perm[r] of A)
Csr permute_rows(const Csr &A, const std::vector<int> &perm);
// Points ordered along the Morton (Z-order) curve of their positions
// (xyz [n][3], 21 bits per coordinate over the bounding box; equal codes keep
// their index order): result[r] = the point at position r of the curve.
std::vector<int> morton_order(const std::vector<double> &xyz, int n);
// columns renumbered: column j < split becomes map[j], column j >= split
// becomes split + map[j - split]; each row's columns sorted again
Csr renumber_cols(const Csr &A, const std::vector<int> &map, int split);
// rows and columns renumbered: entry (r, iperm[j]) of the result is a_{perm[r], j}
Csr permute_symmetric(const Csr &A, const std::vector<int> &perm, const std::vector<int> &iperm);

}  // namespace auxp
