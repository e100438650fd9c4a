// Device side of the solver: upload of the setup data, the preconditioner
// B (Algorithm 2.1 with presmoothing, Remark 2.1) and preconditioned CG,
// behind the C ABI declared in include/aux.h.
//
// The P^k level runs in an internal dof order (rows sorted by length within
// windows, see formats.cpp); vectors are permuted once on entry to and exit
// from aux_apply / pcg_solve / aux_matvec.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <functional>
#include <mutex>
#include <numeric>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "../host/setup.hpp"
#include "aux.h"
#include "amgsetup.hpp"
#include "assemble.hpp"
#include "batched.hpp"
#include "blockcg.hpp"
#include "kernels.hpp"
#include "krylov.hpp"
#include "mfree.hpp"
#include "stokes.hpp"

using namespace auxp;

namespace {

thread_local std::string g_error;

struct AuxError : std::runtime_error {
    int code;
    AuxError(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define HIPCHECK(x)                                                                                  \
    do {                                                                                             \
        hipError_t e_ = (x);                                                                         \
        if (e_ != hipSuccess)                                                                        \
            throw AuxError(AUX_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));                \
    } while (0)

struct DevOp {   // CSR with values in both precisions
    int n = 0, m = 0;
    int64_t nnz = 0;
    int *ptr = nullptr, *col = nullptr;
    double *v64 = nullptr;
    float *v32 = nullptr;
    int lpr = 1;
    // row-split sliced ELL copy (ell_lanes > 0: the products use it)
    int ell_lanes = 0;
    int64_t ell_stored = 0;
    int *ell_off = nullptr, *ell_col = nullptr;
    double *ell_v64 = nullptr;
    float *ell_v32 = nullptr;
    template <typename T>
    DevCsrView view() const
    {
        const bool f = std::is_same<T, float>::value;
        return {n, ptr, col, f ? (const void *)v32 : (const void *)v64, lpr,
                ell_lanes, ell_off, ell_col, f ? (const void *)ell_v32 : (const void *)ell_v64};
    }
    // lanes of the form in use: > 0 row-split ELL, < 0 CSR (minus its lanes per row)
    int lanes_code() const { return ell_lanes > 0 ? ell_lanes : -lpr; }
};

struct DevSell {
    int n = 0, nslices = 0, max_width = 0;
    int64_t stored = 0, narrow_slices = 0, index_bytes = 0;
    int *slice_off = nullptr, *mode = nullptr, *base = nullptr, *wide = nullptr;
    unsigned short *off = nullptr;
    double *v64 = nullptr;
    float *v32 = nullptr;
    // 32-bit layouts whose slices average at least this many slots give each
    // slice two wavefronts in the single-vector kernels: P4 (72 slots) gains
    // 10-14 %, P3 (47) loses up to 5 % in FP64, P2 (28) keeps one
    static constexpr int kSplitSlots = 56;
    bool split() const { return narrow_slices == 0 && nslices > 0 && stored >= (int64_t)kSplitSlots * 64 * nslices; }
    template <typename T>
    DevSellView view() const
    {
        return {n, nslices, max_width, narrow_slices > 0 ? 1 : 0, slice_off, mode, base, off, wide,
                std::is_same<T, float>::value ? (const void *)v32 : (const void *)v64, split() ? 1 : 0};
    }
};

struct DevTiles {
    int n = 0, tile = 0, ntiles = 0, max_cols = 0, max_entries = 0;
    int *rows = nullptr, *row_ptr = nullptr, *col_off = nullptr, *ucols = nullptr;
    unsigned short *lidx = nullptr;
    double *v64 = nullptr;
    float *v32 = nullptr;
    template <typename T>
    DevTilesView view() const
    {
        return {n, tile, ntiles, max_cols, max_entries, rows, row_ptr, col_off, ucols, lidx,
                std::is_same<T, float>::value ? (const void *)v32 : (const void *)v64};
    }
};

template <typename T>
struct Work {
    bool ready = false;
    T *za = nullptr, *zb = nullptr, *res = nullptr, *rT = nullptr;
    T *nb = nullptr, *ne = nullptr;   // intermediate-space right-hand side and correction
    std::vector<T *> b, x, r, y;
};

double seconds_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

constexpr int kSellWindow = 4096;

}  // namespace

// Device memory of the allocation-free CG entry point (pcg_solve_noalloc):
// the reduction partials, the CG state and the per-iteration r.z, p.Ap and
// r.r histories of one solve.  Each GPU the library runs on holds its own
// copy until the process ends; calls on one GPU share it (the last call's
// contents stay), so such calls must not overlap on one device.  Host code
// never uses the name of this array as an address: it takes each device's
// address once with hipGetSymbolAddress (scratch_address below).
constexpr int kNoAllocHist = 4096;                 // histories: maxit + 2 <= this
constexpr size_t kScratchPartials = 0;
constexpr size_t kScratchScal = kScratchPartials + kMaxBlocks;
constexpr size_t kScratchState = kScratchScal + 8;  // 4 ints in 2 doubles
constexpr size_t kScratchHist = kScratchState + 8;
constexpr size_t kScratchDoubles = kScratchHist + 3 * (size_t)kNoAllocHist;   // 16,400 doubles, 128.1 KiB
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Address of the scratch array on `device` (the current device), looked up
// once per device.
double *scratch_address(int device)
{
    if (device < 0 || device >= kMaxDevices) throw AuxError(AUX_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        HIPCHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) throw AuxError(AUX_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[device] = (double *)ptr;
    }
    return g_scratch_ptr[device];
}

}  // namespace

struct aux_handle {
    Discretization disc;
    Hierarchy hier;
    Sell sell;                       // host copy of the P^k operator format (internal order)
    aux_options opt{};
    aux_device dev{};
    bool host_only = false;
    int device = 0;
    hipStream_t stream = nullptr;
    double setup_seconds = 0.0;
    int64_t device_bytes = 0;
    std::vector<void *> allocs;
    std::vector<size_t> alloc_size;
    int sell_window_used = 0;        // layout window the setup chose
    double tune_ms[4] = {0, 0, 0, 0};

    DevSell A;                       // A_h, internal order
    int *perm = nullptr;             // internal -> external dof
    DevOp IP, IR;                    // I_P rows and I_R columns in internal order
    double *dinv64 = nullptr;
    float *dinv32 = nullptr;
    struct Lev {
        DevOp A, P, R;
        DevOp down, up;              // composite operators (fuse_cycle)
        double *dinv64 = nullptr;
        float *dinv32 = nullptr;
        // levels taken over from the device build: its l1 norms and C/F
        // split, kept for the host copies made on demand
        double *l1 = nullptr;
        int *cf = nullptr;
    };
    DevOp RF;                        // composite restriction [I_R, -I_R A_h] (fuse_cycle)
    // I_P in fixed-width column-major slots (at most 4 entries per row: one
    // per vertex of the node's key; w = 0 when not used)
    struct FixedOp {
        int n = 0, w = 0;
        int *col = nullptr;
        double *v64 = nullptr;
        float *v32 = nullptr;
    } IPf;
    // the cycle from level dense_first down, as one dense matrix (fuse_cycle)
    size_t dense_first = SIZE_MAX;
    double *dcyc64 = nullptr;
    float *dcyc32 = nullptr;
    std::vector<FusedLevel> fused_host;
    // built on the device (amg_setup): fused_host already holds the
    // composite operators, and the dense cycle from level dense_pre_first
    // waits in dense_pre for upload_coefficient_part
    bool fused_pre = false;
    double *dense_pre = nullptr;
    // a device build whose operators upload_coefficient_part takes over as
    // they are (no host round trip); hier and fused_host then stay empty
    // until a host consumer asks (host_hier_stale)
    DevAmg dev_built;
    bool dev_built_ready = false;
    // the coefficient-dependent device data exist (false from their release
    // in set_kappa until the update completes)
    bool coef_ready = true;
    bool host_hier_stale = false;
    int dense_pre_first = -1;
    double amg_seconds = 0.0;
    // intermediate auxiliary space (aux_space = 2, Remark 6.2): the P^2
    // handle on the same mesh and stream, the transfer I_2 (external orders
    // for export; internal orders on the device) and the composite
    // restriction [I_2^T, -I_2^T A_h]
    aux_handle *child = nullptr;
    Csr I2host, I2i, I2Ti, RF2_host;
    DevOp I2d, I2Td, RF2;
    Csr RF_host;
    std::vector<Lev> lev;
    double *cinv64 = nullptr;
    float *cinv32 = nullptr;
    bool fp32_ready = false;

    Work<double> w64;
    Work<float> w32;

    // CG buffers (internal order)
    double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *xi = nullptr, *fi = nullptr;
    double *partials = nullptr;
    double *scal = nullptr;          // [0] f.f, [1] r0.r0, [2] tol^2 f.f
    int *istate = nullptr;           // [0] iter, [1] done
    double *hist = nullptr;          // rz, pq, rr each [hist_cap]
    int hist_cap = 0;
    int *host_state = nullptr;       // pinned: iter, done
    double *host_scal = nullptr;     // pinned: r.r window of the chunk prediction, target, final r.r and f.f,
                                     // true residual r.r
    // the last single-vector CG solve: its r_k.r_k history (device), count and f.f
    const double *last_rr = nullptr;
    int last_iters = -1;
    double last_ff = 0.0;
    std::vector<void *> host_bufs;   // other pinned buffers

    // adjoint data (external dof numbering)
    double *G = nullptr, *kappa_d = nullptr, *Mtab = nullptr;
    int *tet_dof_d = nullptr;

    // matrix-free element operator (internal dof numbering)
    bool mf_ready = false;
    int *mf_emap = nullptr, *mf_inc_ptr = nullptr, *mf_inc = nullptr;   // mf_inc: slot of each (tet, node)
    double *mf_w64 = nullptr, *mf_S64 = nullptr, *mf_Y64 = nullptr;
    float *mf_w32 = nullptr, *mf_S32 = nullptr, *mf_Y32 = nullptr;

    void ensure_mf()
    {
        if (mf_ready) return;
        const int nt = disc.nt, nl = disc.nloc, n = disc.ndof;
        static const int pairs[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
        const std::vector<double> &M = stiffness_tables(disc.k);
        auto Mat = [&](int p, int q, int a, int b) { return M[(((size_t)p * 4 + q) * nl + a) * nl + b]; };
        std::vector<double> S((size_t)nl * 6 * nl);
        for (int k = 0; k < 6; k++) {
            int p = pairs[k][0], q = pairs[k][1];
            for (int a = 0; a < nl; a++)
                for (int b = 0; b < nl; b++)
                    S[(size_t)a * 6 * nl + k * nl + b] = Mat(p, p, a, b) + Mat(q, q, a, b) - Mat(p, q, a, b) - Mat(q, p, a, b);
        }
        std::vector<double> w((size_t)nt * 6);
        std::vector<int> emap((size_t)nt * nl), cnt((size_t)n + 1, 0);
        for (int t = 0; t < nt; t++) {
            const int *v = &disc.tets[4 * (size_t)t];
            double Gt[4][4];
            tet_metric(&disc.xyz[3 * (size_t)v[0]], &disc.xyz[3 * (size_t)v[1]], &disc.xyz[3 * (size_t)v[2]],
                       &disc.xyz[3 * (size_t)v[3]], Gt);
            for (int k = 0; k < 6; k++) w[(size_t)t * 6 + k] = -disc.kappa[t] * Gt[pairs[k][0]][pairs[k][1]];
            for (int a = 0; a < nl; a++) {
                int d = disc.tet_dof[(size_t)t * nl + a];
                emap[(size_t)t * nl + a] = d >= 0 ? sell.iperm[d] : -1;
                if (d >= 0) cnt[sell.iperm[d] + 1]++;
            }
        }
        for (int i = 0; i < n; i++) cnt[i + 1] += cnt[i];
        // slot of each (tet, local node) in the dof-ordered result array
        std::vector<int> slot(emap.size(), -1), fill(cnt.begin(), cnt.end() - 1);
        for (size_t s = 0; s < emap.size(); s++)
            if (emap[s] >= 0) slot[s] = fill[emap[s]]++;
        mf_emap = upload(emap);
        mf_inc_ptr = upload(cnt);
        mf_inc = upload(slot);
        mf_w64 = upload(w);
        mf_S64 = upload(S);
        mf_w32 = upload(to_f32(w));
        mf_S32 = upload(to_f32(S));
        mf_Y64 = dnew<double>((size_t)nt * nl);
        mf_Y32 = dnew<float>((size_t)nt * nl);
        mf_ready = true;
    }
    template <typename T>
    MfView<T> mf_view() const
    {
        MfView<T> v{disc.ndof, disc.nt, disc.nloc, mf_emap, nullptr, nullptr, mf_inc_ptr, mf_inc};
        if constexpr (std::is_same<T, float>::value) {
            v.w = mf_w32;
            v.S = mf_S32;
        } else {
            v.w = mf_w64;
            v.S = mf_S64;
        }
        return v;
    }
    template <typename T>
    T *mf_Y() const
    {
        if constexpr (std::is_same<T, float>::value) return mf_Y32;
        else return mf_Y64;
    }
    bool use_mf() const { return opt.op == AUX_OP_MATFREE; }

    // P^k smoothing sweep zout = zin + D^{-1}(rhs - A zin) with the configured operator
    template <typename T, typename TR, typename TZ>
    int pk_sweep(const T *d, const TR *rhs, const T *zin, TZ *zout, const double *rdot, double *partials,
                 const int *done)
    {
        if (use_mf()) {
            MfView<T> v = mf_view<T>();
            mf_apply<T>(stream, v, zin, mf_Y<T>(), done);
            return mf_sweep<T, TR, TZ>(stream, v, mf_Y<T>(), zin, d, rhs, zout, rdot, partials, done);
        }
        return sell_sweep<T, TR, TZ>(stream, A.view<T>(), d, rhs, zin, zout, rdot, partials, done);
    }
    template <typename T>
    void pk_resid(const T *rhs, const T *z, T *res, const int *done)
    {
        if (use_mf()) {
            MfView<T> v = mf_view<T>();
            mf_apply<T>(stream, v, z, mf_Y<T>(), done);
            mf_resid<T>(stream, v, mf_Y<T>(), rhs, res, done);
            return;
        }
        sell_resid<T>(stream, A.view<T>(), rhs, z, res, done);
    }

    // kernel timing with HIP events on the handle's stream
    struct ProfRec {
        hipEvent_t a, b;
        int cat, tag;
    };
    bool prof_on = false;
    bool prof_apply_only = false;    // record whole preconditioner applications only
    int prof_tag = -1;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<ProfRec> prof;
    double prof_ms[AUX_PROF_NCAT] = {};
    int64_t prof_n[AUX_PROF_NCAT] = {};

    // ------------------------------------------------------------ memory
    void *dalloc(size_t bytes)
    {
        if (bytes == 0) bytes = 16;
        void *ptr = nullptr;
        if (dev.alloc) {
            ptr = dev.alloc(bytes, dev.ctx);
            if (!ptr) throw AuxError(AUX_ENOMEM, "device allocation callback failed");
        } else {
            hipError_t e = hipMalloc(&ptr, bytes);
            if (e != hipSuccess) throw AuxError(AUX_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        allocs.push_back(ptr);
        alloc_size.push_back(bytes);
        device_bytes += (int64_t)bytes;
        return ptr;
    }
    // (wait: first wait for the stream, which may still use the buffer)
    void dfree(void *ptr, bool wait = true)
    {
        for (size_t i = 0; i < allocs.size(); i++)
            if (allocs[i] == ptr) {
                if (wait) HIPCHECK(hipStreamSynchronize(stream));
                if (dev.free) dev.free(ptr, dev.ctx);
                else HIPCHECK(hipFree(ptr));
                device_bytes -= (int64_t)alloc_size[i];
                allocs.erase(allocs.begin() + i);
                alloc_size.erase(alloc_size.begin() + i);
                return;
            }
    }
    template <typename T>
    T *dnew(size_t n)
    {
        return (T *)dalloc(n * sizeof(T));
    }
    template <typename T>
    T *upload(const T *src, size_t n)
    {
        T *d = dnew<T>(n);
        if (n) HIPCHECK(hipMemcpy(d, src, n * sizeof(T), hipMemcpyHostToDevice));
        return d;
    }
    template <typename T>
    T *upload(const std::vector<T> &v)
    {
        return upload(v.data(), v.size());
    }
    static std::vector<float> to_f32(const std::vector<double> &v) { return std::vector<float>(v.begin(), v.end()); }
    // the P^k smoother's diagonal: omega / l1 (omega = 1: plain l1-Jacobi)
    std::vector<double> smoother_inv(const std::vector<double> &l1) const
    {
        std::vector<double> o(l1.size());
        for (size_t i = 0; i < l1.size(); i++) o[i] = opt.smoother_weight / l1[i];
        return o;
    }
    static std::vector<double> inverse(const std::vector<double> &v)
    {
        std::vector<double> o(v.size());
        for (size_t i = 0; i < v.size(); i++) o[i] = 1.0 / v[i];
        return o;
    }
    void drop_ell(DevOp &op)
    {
        for (void *b : {(void *)op.ell_off, (void *)op.ell_col, (void *)op.ell_v64, (void *)op.ell_v32}) dfree(b);
        op.ell_off = op.ell_col = nullptr;
        op.ell_v64 = nullptr;
        op.ell_v32 = nullptr;
        op.ell_lanes = 0;
        op.ell_stored = 0;
    }


    // Storage and lanes of one V-cycle operator: time one FP32 product
    // (two-source form when split > 0) for each candidate, CSR with 2-32
    // lanes per row and row-split ELL with 1-32 lanes per row, and keep the
    // fastest.  In the solve the operator's data has been evicted by the P^k
    // passes, so each timed launch follows a write of `flush` bytes that
    // clears the caches.  (T = double: the same for an FP64-only operator.)
    void tune_op(DevOp &op, int split, void *flush, size_t flush_bytes)
    {
        tune_op_t<float>(op, split, flush, flush_bytes);
    }
    template <typename T>
    void tune_op_t(DevOp &op, int split, void *flush, size_t flush_bytes)
    {
        if (!(std::is_same<T, float>::value ? (void *)op.v32 : (void *)op.v64) || op.n == 0) return;
        T *x = dnew<T>(std::max(op.m, 1)), *y = dnew<T>(op.n);
        HIPCHECK(hipMemsetAsync(x, 0, (size_t)std::max(op.m, 1) * sizeof(T), stream));
        const double avg = (double)op.nnz / op.n;
        hipEvent_t a = take_event(), b = take_event();
        auto measure = [&]() {
            auto run = [&]() {
                if (split > 0) csr_matvec2<T>(stream, op.view<T>(), x, x + split, split, y, nullptr);
                else csr_matvec<T>(stream, op.view<T>(), x, y, nullptr);
            };
            run();
            double total = 0.0;
            for (int i = 0; i < 3; i++) {
                HIPCHECK(hipMemsetAsync(flush, i + 1, flush_bytes, stream));
                HIPCHECK(hipEventRecord(a, stream));
                run();
                HIPCHECK(hipEventRecord(b, stream));
                HIPCHECK(hipEventSynchronize(b));
                float ms = 0.f;
                HIPCHECK(hipEventElapsedTime(&ms, a, b));
                total += ms;
            }
            return total;
        };
        double best = 1e300;
        int pick = op.lpr, pick_ell = 0;
        drop_ell(op);
        for (int lpr : {2, 4, 8, 16, 32}) {
            if (lpr > 4 * avg + 4) break;
            op.lpr = lpr;
            const double t = measure();
            if (t < best) {
                best = t;
                pick = lpr;
            }
        }
        op.lpr = pick;
        for (int lanes : {1, 2, 4, 8, 16, 32}) {
            if (lanes > 4 * avg + 4) break;
            set_ell(op, lanes);
            const double t = measure();
            if (t < best) {
                best = t;
                pick_ell = lanes;
            }
        }
        if (pick_ell > 0) set_ell(op, pick_ell);
        else drop_ell(op);
        ev_used -= 2;
        dfree(x);
        dfree(y);
    }

    // CSR with both precisions uploaded at once (composite operators)
    DevOp upload_op2(const Csr &c)
    {
        DevOp d = upload_op(c);
        d.v32 = upload(to_f32(c.val));
        return d;
    }

    DevOp upload_op(const Csr &c)
    {
        DevOp d;
        d.n = c.n;
        d.m = c.m;
        d.nnz = c.nnz();
        d.ptr = upload(c.ptr);
        d.col = upload(c.col);
        d.v64 = upload(c.val);
        d.lpr = pick_lpr(c.n ? (double)c.nnz() / c.n : 1.0);
        return d;
    }

    Csr IPi, IRi;                    // internal-order transfers (host, for the FP32 copies)
    std::vector<std::array<int, 2>> tuned_lanes;   // storage chosen at setup per level (down, up)
    std::vector<double> l1i;         // l1 norms in internal order

    DevSell upload_sell(const Sell &sl)
    {
        DevSell d;
        d.n = sl.n;
        d.nslices = sl.nslices;
        d.max_width = sl.max_width;
        d.stored = (int64_t)sl.val.size();
        for (int s = 0; s < sl.nslices; s++) {
            const int64_t entries = sl.slice_off[s + 1] - sl.slice_off[s];
            d.narrow_slices += sl.mode[s] == 0;
            d.index_bytes += sl.mode[s] == 0 ? 2 * entries + 4 * (entries / sl.slice) : 4 * entries;
        }
        d.slice_off = upload(sl.slice_off);
        d.mode = upload(sl.mode);
        d.base = upload(sl.base);
        d.off = upload(sl.off);
        d.wide = upload(sl.wide);
        d.v64 = upload(sl.val);
        return d;
    }

    void free_sell(DevSell &d)
    {
        for (void *b : {(void *)d.slice_off, (void *)d.mode, (void *)d.base, (void *)d.off, (void *)d.wide,
                        (void *)d.v64, (void *)d.v32})
            dfree(b);
        d = DevSell();
    }

    // mean time of a few products with a device layout, FP64 plus FP32 (the
    // autotuner's measure: the CG product and the preconditioner's passes)
    double time_sell(DevSell &d, const Sell &sl)
    {
        const int n = disc.ndof;
        d.v32 = upload(to_f32(sl.val));
        double *x = dnew<double>(n), *y = dnew<double>(n);
        float *xf = dnew<float>(n), *yf = dnew<float>(n), *bf = dnew<float>(n);
        HIPCHECK(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), stream));
        HIPCHECK(hipMemsetAsync(xf, 0, (size_t)n * sizeof(float), stream));
        HIPCHECK(hipMemsetAsync(bf, 0, (size_t)n * sizeof(float), stream));
        hipEvent_t a = take_event(), b = take_event();
        for (int i = 0; i < 3; i++) {              // untimed: first touches, clocks up
            sell_spmv64(stream, d.view<double>(), x, y, nullptr, nullptr);
            sell_resid<float>(stream, d.view<float>(), bf, xf, yf, nullptr);
        }
        HIPCHECK(hipEventRecord(a, stream));
        for (int i = 0; i < 5; i++) {
            sell_spmv64(stream, d.view<double>(), x, y, nullptr, nullptr);
            sell_resid<float>(stream, d.view<float>(), bf, xf, yf, nullptr);
        }
        HIPCHECK(hipEventRecord(b, stream));
        HIPCHECK(hipEventSynchronize(b));
        float ms = 0.f;
        HIPCHECK(hipEventElapsedTime(&ms, a, b));
        ev_used -= 2;
        for (void *p : {(void *)x, (void *)y, (void *)xf, (void *)yf, (void *)bf, (void *)d.v32}) dfree(p);
        d.v32 = nullptr;
        return ms / 5.0;
    }

    void upload_all()
    {
        // Device layout of A_h.  A fixed window if one is given; otherwise the
        // autotuner builds the candidates (rows sorted by length over the whole
        // operator, which on lattice-structured meshes groups nodes of one
        // type so a slice gathers nearly contiguous entries; and a 4096-row
        // window, which keeps locality on unstructured meshes), times a few
        // products with each on the device and keeps the faster.
        std::vector<std::pair<int, bool>> cands;
        std::vector<int> windows;
        if (opt.sell_window > 0) windows.push_back(opt.sell_window);
        else windows = {std::max(disc.ndof, 1), kSellWindow};
        for (int win : windows) {
            if (opt.sell_index16) cands.push_back({win, true});
            if (!opt.sell_index16 || opt.sell_window <= 0) cands.push_back({win, false});
        }
        double best = 1e300;
        int same_as_32 = -1;       // a window whose 16-bit build has no 16-bit slice
        for (auto [win, idx16] : cands) {
            Sell cand;
            if (!idx16 && win == same_as_32) continue;   // timed already, as the 32-bit form
            build_sell(disc.A, kSlice, win, idx16, cand);
            if (idx16 && cands.size() > 1 &&
                std::none_of(cand.mode.begin(), cand.mode.end(), [](int m) { return m == 0; })) {
                // no slice takes 16-bit offsets: the build is the 32-bit layout
                cand.base.clear();
                cand.off.clear();
                idx16 = false;
                same_as_32 = win;
            }
            DevSell d = upload_sell(cand);
            double ms = cands.size() > 1 ? time_sell(d, cand) : 0.0;
            tune_ms[(win == kSellWindow ? 2 : 0) + (idx16 ? 0 : 1)] = ms;
            if (ms < best) {
                if (A.v64) free_sell(A);
                best = ms;
                A = d;
                sell = std::move(cand);
                sell_window_used = win;
            } else {
                free_sell(d);
            }
        }
        perm = upload(sell.perm);
        IPi = permute_rows(disc.IP, sell.perm);
        IRi = transpose(IPi);
        IP = upload_op2(IPi);
        IR = upload_op(IRi);
        if (opt.cycle_lanes == 0) set_fixed(IPf, IPi);
        upload_coefficient_part(true);
        int n = disc.ndof;
        r = dnew<double>(n);
        z = dnew<double>(n);
        p = dnew<double>(n);
        q = dnew<double>(n);
        xi = dnew<double>(n);
        fi = dnew<double>(n);
        partials = dnew<double>(kMaxBlocks);
        scal = dnew<double>(8);
        istate = dnew<int>(4);
        HIPCHECK(hipHostMalloc((void **)&host_state, 4 * sizeof(int), hipHostMallocDefault));
        HIPCHECK(hipHostMalloc((void **)&host_scal, 8 * sizeof(double), hipHostMallocDefault));
        ensure_hist(std::max(opt.maxit, 16));
    }

    // the fixed-width slot form of an operator with 1 to 4 entries per row
    // (left unused otherwise)
    void set_fixed(FixedOp &f, const Csr &c)
    {
        int w = 0;
        for (int i = 0; i < c.n; i++) w = std::max(w, c.ptr[i + 1] - c.ptr[i]);
        if (w < 1 || w > 4) return;
        const size_t n = (size_t)c.n;
        std::vector<int> col(w * n, 0);
        std::vector<double> val(w * n, 0.0);
        for (size_t i = 0; i < n; i++)
            for (int e = c.ptr[i], k = 0; e < c.ptr[i + 1]; e++, k++) {
                col[k * n + i] = c.col[e];
                val[k * n + i] = c.val[e];
            }
        f.n = c.n;
        f.w = w;
        f.col = upload(col);
        f.v64 = upload(val);
        f.v32 = upload(to_f32(val));
    }

    // Storage of one operator by lanes code (> 0: row-split ELL with that
    // many lanes per row; <= 0: CSR with -code lanes per row)
    void set_storage(DevOp &op, int code)
    {
        if (code > 0) {
            set_ell(op, code);
        } else {
            drop_ell(op);
            op.lpr = -code;
        }
    }
    // the row-split ELL copy of an operator, built on the device from its
    // FP64 CSR (FP32 values the rounding of the FP64 ones)
    void set_ell(DevOp &op, int lanes)
    {
        drop_ell(op);
        DevMem mem{[this](size_t b) { return dalloc(b); }, [this](void *p) { dfree(p); }};
        DCsr c;
        c.n = op.n;
        c.m = op.m;
        c.nnz = (int)op.nnz;
        c.ptr = op.ptr;
        c.col = op.col;
        c.val = op.v64;
        DevEll e;
        ell_from_csr(stream, c, lanes, mem, e);
        op.ell_off = e.off;
        op.ell_col = e.col;
        op.ell_v64 = e.val;
        op.ell_v32 = dnew<float>((size_t)e.stored);
        to_f32_device(stream, e.stored, e.val, op.ell_v32);
        op.ell_stored = e.stored;
        op.ell_lanes = lanes;
    }

    // The levels, composite operators and coarse inverse of the pending
    // device build, taken over as they are (same arrays, CSR with the
    // rule-based lanes; FP32 copies of the composite operators made on the
    // device); the host copies are made when a host consumer needs them.
    void adopt_device_levels()
    {
        DevAmg &d = dev_built;
        const size_t L = d.A.size();
        auto take = [&](const DCsr &c) {
            DevOp o;
            o.n = c.n;
            o.m = c.m;
            o.nnz = c.nnz;
            o.ptr = c.ptr;
            o.col = c.col;
            o.v64 = c.val;
            o.lpr = pick_lpr(c.n ? (double)c.nnz / c.n : 1.0);
            return o;
        };
        auto with_f32 = [&](DevOp o) {
            o.v32 = dnew<float>((size_t)o.nnz);
            to_f32_device(stream, o.nnz, o.v64, o.v32);
            return o;
        };
        lev.assign(L, Lev());
        for (size_t l = 0; l < L; l++) {
            Lev &lv = lev[l];
            lv.A = take(d.A[l]);
            lv.l1 = d.l1[l];
            lv.dinv64 = dnew<double>((size_t)lv.A.n);
            reciprocal_device(stream, lv.A.n, lv.l1, lv.dinv64);
            if (l + 1 < L) {
                lv.P = take(d.P[l]);
                lv.R = take(d.R[l]);
                lv.cf = d.cf[l];
                if (opt.fuse_cycle) {
                    lv.down = with_f32(take(d.down[l]));
                    lv.up = with_f32(take(d.up[l]));
                }
            }
        }
        cinv64 = d.coarse_inv;
        dev_built = DevAmg();
        dev_built_ready = false;
        hier = Hierarchy();
        fused_host.clear();
        host_hier_stale = true;
    }

    // host copies of the levels and composite operators taken over from a
    // device build (exports, the batched forms)
    void ensure_host_hierarchy()
    {
        if (!host_hier_stale) return;
        DevAmg v;
        auto view = [](const DevOp &o) {
            DCsr c;
            c.n = o.n;
            c.m = o.m;
            c.nnz = (int)o.nnz;
            c.ptr = o.ptr;
            c.col = o.col;
            c.val = o.v64;
            return c;
        };
        const size_t L = lev.size();
        for (size_t l = 0; l < L; l++) {
            v.A.push_back(view(lev[l].A));
            v.l1.push_back(lev[l].l1);
            if (l + 1 < L) {
                v.P.push_back(view(lev[l].P));
                v.R.push_back(view(lev[l].R));
                v.cf.push_back(lev[l].cf);
                if (opt.fuse_cycle) {
                    v.down.push_back(view(lev[l].down));
                    v.up.push_back(view(lev[l].up));
                }
            }
        }
        v.coarse_inv = cinv64;
        v.ncoarse = L ? lev[L - 1].A.n : 0;
        download_amg(stream, v, hier, opt.fuse_cycle ? &fused_host : nullptr);
        host_hier_stale = false;
    }

    // Everything on the device that depends on the coefficient beyond A_h's
    // values, built from the host discretisation and hierarchy: the l1
    // diagonal, the AMG levels and coarse inverse, the composite cycle
    // operators, the dense sub-cycle and the fused restriction, with the
    // storage of the cycle's operators chosen again (first: I_P's as well).
    void upload_coefficient_part(bool first)
    {
        l1i.resize(disc.ndof);
        for (int i = 0; i < disc.ndof; i++) l1i[i] = disc.l1[sell.perm[i]];
        dinv64 = upload(smoother_inv(l1i));
        const bool adopted = dev_built_ready;
        if (adopted) {
            adopt_device_levels();
        } else {
            lev.resize(hier.levels.size());
            for (size_t l = 0; l < hier.levels.size(); l++) {
                const AmgLevel &hl = hier.levels[l];
                lev[l].A = upload_op(hl.A);
                lev[l].dinv64 = upload(inverse(hl.l1));
                if (l + 1 < hier.levels.size()) {
                    lev[l].P = upload_op(hl.P);
                    lev[l].R = upload_op(hl.R);
                }
            }
            cinv64 = upload(hier.coarse_inv);
        }
        if (opt.fuse_cycle && !lev.empty()) {
            if (!adopted) {
                if (!fused_pre) fused_host.resize(hier.levels.size());
                for (size_t l = 0; l + 1 < hier.levels.size(); l++) {
                    if (!fused_pre) fused_host[l] = fuse_level(hier.levels[l]);
                    lev[l].down = upload_op2(fused_host[l].down);
                    lev[l].up = upload_op2(fused_host[l].up);
                }
            }
            // the bottom of the cycle: each small level costs two launches
            // of dependent-load latency (about 5 us each) for well under a
            // microsecond of traffic; below the first level of at most
            // dense_cycle_rows rows the cycle is one dense product instead
            if (fused_pre) {
                if (dense_pre) {                   // formed on the device by the same rule
                    const size_t nd = (size_t)lev[dense_pre_first].A.n;
                    dcyc64 = dense_pre;
                    dcyc32 = dnew<float>(nd * nd);
                    to_f32_device(stream, (long long)(nd * nd), dcyc64, dcyc32);
                    dense_first = (size_t)dense_pre_first;
                    dense_pre = nullptr;
                }
            } else if (opt.dense_cycle_rows > 0)
                for (size_t l = 0; l + 1 < lev.size(); l++)
                    if (lev[l].A.n <= opt.dense_cycle_rows) {
                        const std::vector<double> T = dense_cycle(fused_host, hier, l);
                        dcyc64 = upload(T);
                        dcyc32 = upload(to_f32(T));
                        dense_first = l;
                        break;
                    }
            // the composite restriction depends on A_h's values through
            // I_R A_h on a pattern fixed by the mesh: built here once; a new
            // coefficient refreshes its values on the device (set_kappa)
            if (first) {
                RF_host = fuse_restriction(IRi, permute_symmetric(disc.A, sell.perm, sell.iperm));
                RF = upload_op2(RF_host);
            }
            // lanes per row of the large CSR passes, timed on the device
            // (with a fixed layout window every choice is rule-based)
            // (I_P has one or two entries per row: its rule-based two lanes
            // per row measured best in the solve).  A new coefficient keeps
            // the storage chosen at setup for each level index.
            if (opt.cycle_lanes != 0) {                // one storage for all of them
                const int code = opt.cycle_lanes;
                if (first) {
                    set_storage(RF, code);
                    set_storage(IP, code);
                }
                for (size_t l = 0; l + 1 < lev.size(); l++) {
                    set_storage(lev[l].down, code);
                    set_storage(lev[l].up, code);
                }
            } else if (opt.sell_window <= 0 && first) {
                const size_t fb = (size_t)512 << 20;    // twice the last-level cache
                void *flush = dalloc(fb);
                tune_op(RF, disc.ndof, flush, fb);
                if (!IPf.w) tune_op(IP, 0, flush, fb);
                tuned_lanes.clear();
                for (size_t l = 0; l + 1 < lev.size(); l++) {
                    if (lev[l].A.n < 8192) break;
                    tune_op(lev[l].down, 0, flush, fb);
                    tune_op(lev[l].up, lev[l].A.n, flush, fb);
                    tuned_lanes.push_back({lev[l].down.lanes_code(), lev[l].up.lanes_code()});
                }
                dfree(flush);
            } else if (opt.sell_window <= 0) {
                for (size_t l = 0; l + 1 < lev.size() && l < tuned_lanes.size(); l++) {
                    if (lev[l].A.n < 8192) break;
                    set_storage(lev[l].down, tuned_lanes[l][0]);
                    set_storage(lev[l].up, tuned_lanes[l][1]);
                }
            }
        }
        fused_pre = false;
    }

    SetupOptions amg_options() const
    {
        SetupOptions so;
        so.theta = opt.theta;
        so.coarse_max = opt.coarse_max;
        so.max_levels = opt.max_levels;
        so.seed = opt.pmis_seed;
        return so;
    }

    // The hierarchy of A_H (a device CSR in A_H's pattern) built on the
    // device with the host setup's arithmetic; host copies of the levels and
    // of the composite operators go to hier and fused_host (the host-side
    // consumers: uploads, layout choices, batched forms), and the dense
    // cycle stays on the device for upload_coefficient_part.
    // With adopt, the device arrays are kept for upload_coefficient_part to
    // take over and nothing is copied to the host.
    // The build's workspaces are released together at its end: a release
    // waits for the stream (the allocator need not be stream-ordered), and
    // one wait instead of one per workspace keeps the device busy.
    void device_hierarchy(const DCsr &AH, bool adopt = false)
    {
        auto t0 = std::chrono::steady_clock::now();
        std::vector<void *> spent;
        DevMem mem{[this](size_t b) { return dalloc(b); }, [&spent](void *p) { spent.push_back(p); }};
        auto release_spent = [&]() {
            if (!spent.empty()) HIPCHECK(hipStreamSynchronize(stream));
            for (void *p : spent) dfree(p, false);
            spent.clear();
        };
        DevAmg d;
        try {
            device_amg(stream, AH, amg_options(), opt.fuse_cycle != 0, opt.dense_cycle_rows, mem, d);
            release_spent();
            hier = Hierarchy();
            fused_host.clear();
            if (!adopt) download_amg(stream, d, hier, opt.fuse_cycle ? &fused_host : nullptr);
        } catch (...) {
            free_amg(mem, d);
            release_spent();
            throw;
        }
        dfree(dense_pre);
        dense_pre = d.dense;
        dense_pre_first = d.dense_first;
        d.dense = nullptr;
        fused_pre = opt.fuse_cycle != 0;
        if (adopt) {
            dev_built = d;
            dev_built_ready = true;
        } else {
            free_amg(mem, d);
            release_spent();
        }
        amg_seconds = seconds_since(t0);
    }

    // at setup: the host-assembled A_H through the device build
    void device_hierarchy_from_host()
    {
        DCsr AH;
        AH.n = AH.m = disc.AH.n;
        AH.nnz = (int)disc.AH.nnz();
        AH.ptr = upload(disc.AH.ptr);
        AH.col = upload(disc.AH.col);
        AH.val = upload(disc.AH.val);
        device_hierarchy(AH);
        for (void *b : {(void *)AH.ptr, (void *)AH.col, (void *)AH.val}) dfree(b);
    }

    void ensure_hist(int maxit)
    {
        if (maxit + 2 <= hist_cap) return;
        hist_cap = maxit + 2;
        hist = dnew<double>((size_t)3 * hist_cap);
    }

    void ensure_fp32()
    {
        if (child) child->ensure_fp32();
        if (fp32_ready) return;
        ensure_host_values();
        A.v32 = upload(to_f32(sell.val));
        if (!IP.v32) IP.v32 = upload(to_f32(IPi.val));
        IR.v32 = upload(to_f32(IRi.val));
        fp32_coefficient_part();
        fp32_ready = true;
    }
    // FP32 copies of the coefficient-dependent operators
    // (each the rounding of the FP64 array on the device)
    void fp32_coefficient_part()
    {
        auto f32 = [&](const double *a, size_t n) {
            float *b = dnew<float>(n);
            to_f32_device(stream, (long long)n, a, b);
            return b;
        };
        dinv32 = f32(dinv64, (size_t)disc.ndof);
        for (size_t l = 0; l < lev.size(); l++) {
            Lev &lv = lev[l];
            lv.A.v32 = f32(lv.A.v64, (size_t)lv.A.nnz);
            lv.dinv32 = f32(lv.dinv64, (size_t)lv.A.n);
            if (l + 1 < lev.size()) {
                lv.P.v32 = f32(lv.P.v64, (size_t)lv.P.nnz);
                lv.R.v32 = f32(lv.R.v64, (size_t)lv.R.nnz);
            }
        }
        if (!lev.empty()) cinv32 = f32(cinv64, (size_t)lev.back().A.n * lev.back().A.n);
    }

    template <typename T>
    Work<T> &work()
    {
        Work<T> *w;
        if constexpr (std::is_same<T, float>::value) w = &w32;
        else w = &w64;
        if (!w->ready) {
            int n = disc.ndof;
            w->za = dnew<T>(n);
            w->zb = dnew<T>(n);
            w->res = dnew<T>(n);
            if (std::is_same<T, float>::value) w->rT = dnew<T>(n);
            for (auto &L : lev) {
                w->b.push_back(dnew<T>(L.A.n));
                w->x.push_back(dnew<T>(L.A.n));
                w->r.push_back(dnew<T>(L.A.n));
                w->y.push_back(dnew<T>(L.A.n));
            }
            if (child) {
                w->nb = dnew<T>(child->disc.ndof);
                w->ne = dnew<T>(child->disc.ndof);
                child->work<T>();
            }
            w->ready = true;
        }
        return *w;
    }

    template <typename T>
    const T *dinv() const
    {
        if constexpr (std::is_same<T, float>::value) return dinv32;
        else return dinv64;
    }
    template <typename T>
    const T *ldinv(size_t l) const
    {
        if constexpr (std::is_same<T, float>::value) return lev[l].dinv32;
        else return lev[l].dinv64;
    }
    template <typename T>
    const T *cinv() const
    {
        if constexpr (std::is_same<T, float>::value) return cinv32;
        else return cinv64;
    }

    // ------------------------------------------------------------ timing
    hipEvent_t take_event()
    {
        if (ev_used == ev_pool.size()) {
            hipEvent_t e;
            HIPCHECK(hipEventCreate(&e));
            ev_pool.push_back(e);
        }
        return ev_pool[ev_used++];
    }
    int pbeg(int cat)
    {
        if (!prof_on || (prof_apply_only && cat != AUX_PROF_APPLY)) return -1;
        ProfRec rec{take_event(), take_event(), cat, prof_tag};
        HIPCHECK(hipEventRecord(rec.a, stream));
        prof.push_back(rec);
        return (int)prof.size() - 1;
    }
    void pend(int idx)
    {
        if (idx >= 0) HIPCHECK(hipEventRecord(prof[idx].b, stream));
    }
    // Fold recorded events into per-category sums.  In a CG solve, launch tag
    // j belongs to iteration j; launches of iterations enqueued after the
    // solve finished returned at once and are dropped.
    void prof_collect(int final_iter)
    {
        if (prof.empty()) return;
        HIPCHECK(hipStreamSynchronize(stream));
        for (const ProfRec &rec : prof) {
            bool ran = rec.tag <= 0 || (rec.cat == AUX_PROF_CG_SPMV ? rec.tag <= final_iter : rec.tag < final_iter);
            if (!ran) continue;
            float ms = 0.f;
            HIPCHECK(hipEventElapsedTime(&ms, rec.a, rec.b));
            prof_ms[rec.cat] += ms;
            prof_n[rec.cat] += 1;
        }
        prof.clear();
        ev_used = 0;
    }

    // ------------------------------------------------------------ preconditioner
    // one V(1,1) cycle from zero on level l; returns the device vector holding the result
    template <typename T>
    const T *dcyc() const
    {
        if constexpr (std::is_same<T, float>::value) return dcyc32;
        else return dcyc64;
    }

    template <typename T>
    const T *vcycle(size_t l, const int *done)
    {
        Work<T> &w = work<T>();
        hipStream_t s = stream;
        const Lev &L = lev[l];
        if (l + 1 == lev.size()) {
            dense_gemv<T>(s, L.A.n, cinv<T>(), w.b[l], w.x[l], done);
            return w.x[l];
        }
        if (opt.fuse_cycle && l == dense_first) {
            dense_gemv<T>(s, L.A.n, dcyc<T>(), w.b[l], w.y[l], done);
            return w.y[l];
        }
        if (opt.fuse_cycle) {
            // b' = P^T (I - A D^-1) b; recurse; y = (2 D^-1 - D^-1 A D^-1) b + (P - D^-1 A P) e
            csr_matvec<T>(s, L.down.view<T>(), w.b[l], w.b[l + 1], done);
            const T *e = vcycle<T>(l + 1, done);
            csr_matvec2<T>(s, L.up.view<T>(), w.b[l], e, L.A.n, w.y[l], done);
            return w.y[l];
        }
        DevCsrView Av = L.A.view<T>();
        csr_vpre<T>(s, Av, ldinv<T>(l), w.b[l], w.x[l], w.r[l], done);
        csr_matvec<T>(s, L.R.view<T>(), w.r[l], w.b[l + 1], done);
        const T *e = vcycle<T>(l + 1, done);
        csr_matvec_add<T>(s, L.P.view<T>(), e, w.x[l], done);
        csr_sweep<T>(s, Av, ldinv<T>(l), w.b[l], w.x[l], w.y[l], done);
        return w.y[l];
    }

    // zout = B rin (internal order).  With rz_partials, the last sweep also
    // writes the partial sums of rin . zout and the number of partials is
    // returned.
    // prepped: z = D^-1 r (and the FP32 copy of r) are already in w.za / w.rT
    template <typename T>
    int apply_B(const double *rin, double *zout, double *rz_partials, const int *done, bool prepped = false)
    {
        Work<T> &w = work<T>();
        hipStream_t s = stream;
        const T *d = dinv<T>();
        const int nu = opt.nu;
        T *rTbuf = std::is_same<T, float>::value ? w.rT : nullptr;
        T *zc = w.za, *zn = w.zb;
        int pb = pbeg(AUX_PROF_APPLY);
        // presmoothing: nu l1-Jacobi sweeps from z = 0 (the first is z = D^{-1} r)
        int pk = -1;
        if (!prepped) {
            pk = pbeg(AUX_PROF_PK_FIRST);
            vec_jacobi0<T>(s, disc.ndof, d, rin, zc, rTbuf, done);
            pend(pk);
        }
        const T *rT = rTbuf ? (const T *)rTbuf : (const T *)(const void *)rin;
        for (int k = 1; k < nu; k++) {
            pk = pbeg(AUX_PROF_PK_SWEEP);
            pk_sweep<T, T, T>(d, rT, zc, zn, nullptr, nullptr, done);
            pend(pk);
            std::swap(zc, zn);
        }
        coarse_correction<T>(rT, zc, done);
        // Step 3: nu postsmoothing sweeps; the last one writes the FP64 result
        for (int k = 1; k < nu; k++) {
            pk = pbeg(AUX_PROF_PK_SWEEP);
            pk_sweep<T, T, T>(d, rT, zc, zn, nullptr, nullptr, done);
            pend(pk);
            std::swap(zc, zn);
        }
        pk = pbeg(AUX_PROF_PK_LAST);
        int g = pk_sweep<T, double, double>(d, rin, zc, zout, rin, rz_partials, done);
        pend(pk);
        pend(pb);
        return g;
    }

    // Steps 1 and 2 of Algorithm 2.1 on z (rT the right-hand side in T):
    // r_H = I_R (r - A z), one AMG V-cycle, z += I_P e_H; with the
    // intermediate space (Remark 6.2) r_2 = I_2^T (r - A z), one application
    // of the P^2 handle's own preconditioner, z += I_2 e_2
    template <typename T>
    void coarse_correction(const T *rT, T *zc, const int *done)
    {
        Work<T> &w = work<T>();
        hipStream_t s = stream;
        if (child) {
            int pk = pbeg(AUX_PROF_PK_RESID);
            if (opt.fuse_cycle) {
                csr_matvec2<T>(s, RF2.view<T>(), rT, zc, disc.ndof, w.nb, done);
            } else {
                pk_resid<T>(rT, zc, w.res, done);
                csr_matvec<T>(s, I2Td.view<T>(), w.res, w.nb, done);
            }
            pend(pk);
            pk = pbeg(AUX_PROF_COARSE);
            child->stream = s;
            child->apply_inner<T>(w.nb, w.ne, done);
            csr_matvec_add<T>(s, I2d.view<T>(), w.ne, zc, done);
            pend(pk);
            return;
        }
        if (lev.empty()) return;
        int pk = pbeg(AUX_PROF_PK_RESID);
        if (opt.fuse_cycle) {
            // r_H = I_R r - (I_R A_h) z in one pass
            csr_matvec2<T>(s, RF.view<T>(), rT, zc, disc.ndof, w.b[0], done);
            pend(pk);
            pk = pbeg(AUX_PROF_COARSE);
        } else {
            pk_resid<T>(rT, zc, w.res, done);
            pend(pk);
            pk = pbeg(AUX_PROF_COARSE);
            csr_matvec<T>(s, IR.view<T>(), w.res, w.b[0], done);
        }
        const T *e0 = vcycle<T>(0, done);
        if (IPf.w) {
            const T *v;
            if constexpr (std::is_same<T, float>::value) v = IPf.v32;
            else v = IPf.v64;
            fixed_matvec_add<T>(s, IPf.n, IPf.w, IPf.col, v, e0, zc, done);
        } else {
            csr_matvec_add<T>(s, IP.view<T>(), e0, zc, done);
        }
        pend(pk);
    }

    // zout = B rin with both vectors in the working precision T and no
    // inner-product partials: this handle as the intermediate space of a
    // higher-order one (its stream set by the caller)
    template <typename T>
    void apply_inner(const T *rin, T *zout, const int *done)
    {
        Work<T> &w = work<T>();
        hipStream_t s = stream;
        const T *d = dinv<T>();
        T *zc = w.za, *zn = w.zb;
        vec_jacobi0_t<T>(s, disc.ndof, d, rin, zc, done);
        for (int k = 1; k < opt.nu; k++) {
            pk_sweep<T, T, T>(d, rin, zc, zn, nullptr, nullptr, done);
            std::swap(zc, zn);
        }
        coarse_correction<T>(rin, zc, done);
        for (int k = 1; k < opt.nu; k++) {
            pk_sweep<T, T, T>(d, rin, zc, zn, nullptr, nullptr, done);
            std::swap(zc, zn);
        }
        pk_sweep<T, T, T>(d, rin, zc, zout, nullptr, nullptr, done);
    }

    // the intermediate space's device data (after upload_all)
    void setup_nested()
    {
        I2i = renumber_cols(permute_rows(I2host, sell.perm), child->sell.iperm, child->disc.ndof);
        I2Ti = transpose(I2i);
        RF2_host = fuse_restriction(I2Ti, permute_symmetric(disc.A, sell.perm, sell.iperm));
        I2d = upload_op2(I2i);
        I2Td = upload_op2(I2Ti);
        RF2 = upload_op2(RF2_host);
    }

    int apply(const double *rin, double *zout, double *rz_partials, const int *done, bool prepped = false)
    {
        if (use_mf()) ensure_mf();
        if (opt.precision == AUX_MIXED) {
            ensure_fp32();
            return apply_B<float>(rin, zout, rz_partials, done, prepped);
        }
        return apply_B<double>(rin, zout, rz_partials, done, prepped);
    }

    // ------------------------------------------------------------ CG
    // Device buffers one CG solve reduces into and keeps its state in: the
    // handle's own (pcg_solve) or the file-scope scratch array (the
    // allocation-free pcg_solve_noalloc).
    struct CgBufs {
        double *partials;    // [kMaxBlocks] per-workgroup partial sums
        double *scal;        // [8] f.f, r0.r0, tol^2 f.f
        int *istate;         // [4] iteration, stop flag
        double *hist;        // rz, pq, rr, each [hist_cap]
        int hist_cap;
    };
    CgBufs own_cg() const { return {partials, scal, istate, hist, hist_cap}; }
    static CgState cg_state(const CgBufs &b, int maxit)
    {
        return {b.istate, b.istate + 1, b.hist, b.hist + b.hist_cap, b.hist + 2 * b.hist_cap, b.scal, maxit};
    }

    // one CG iteration: q = A p, alpha, x/r update, z = B r, beta, p update
    // (forming p inside the product, from gathered z and p, measured twice as
    // slow as the separate update pass)
    void cg_iteration(const CgState &st, double *part)
    {
        hipStream_t s = stream;
        int n = disc.ndof;
        int pk = pbeg(AUX_PROF_CG_SPMV);
        int g;
        if (use_mf()) {
            // q = A_h p by the element operator in FP64 (half the bytes of
            // the assembled product at P3), with the p . q part
            ensure_mf();
            MfView<double> v = mf_view<double>();
            mf_apply<double>(s, v, p, mf_Y64, st.done);
            g = mf_product<double>(s, v, mf_Y64, q, p, part, st.done);
        } else {
            g = sell_spmv64(s, A.view<double>(), p, q, part, st.done);
        }
        pend(pk);
        finish(s, part, g, FIN_PQ, nullptr, st);
        // the update also starts the preconditioner: z = D^-1 r
        if (opt.precision == AUX_MIXED) {
            ensure_fp32();
            Work<float> &w = work<float>();
            g = cg_update_prep<float>(s, n, xi, r, p, q, st, part, dinv32, w.za, w.rT);
        } else {
            Work<double> &w = work<double>();
            g = cg_update_prep<double>(s, n, xi, r, p, q, st, part, dinv64, w.za, nullptr);
        }
        finish(s, part, g, FIN_RR, nullptr, st);
        g = apply(r, z, part, st.done, true);
        finish(s, part, g, FIN_RZ, nullptr, st);
        cg_direction(s, n, z, p, st);
    }

    // Cached graph of one CG iteration; recaptured when anything its kernels
    // depend on by value changes (precision, operator, iteration limit, block
    // width).  Capture runs on a private stream of default priority.
    struct GraphCache {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        int key[4] = {-1, -1, -1, -1};
        void drop()
        {
            if (exec) hipGraphExecDestroy(exec);
            if (graph) hipGraphDestroy(graph);
            exec = nullptr;
            graph = nullptr;
        }
    };
    hipStream_t cap_stream = nullptr;
    GraphCache g_single, g_batch;

    template <typename Body>
    hipGraphExec_t captured(GraphCache &gc, const int key[4], Body body)
    {
        if (gc.exec && std::equal(key, key + 4, gc.key)) return gc.exec;
        gc.drop();
        if (!cap_stream) HIPCHECK(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
        hipStream_t keep = stream;
        stream = cap_stream;
        HIPCHECK(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
        body();
        hipError_t e = hipStreamEndCapture(cap_stream, &gc.graph);
        stream = keep;
        HIPCHECK(e);
        HIPCHECK(hipGraphInstantiate(&gc.exec, gc.graph, nullptr, nullptr, 0));
        std::copy(key, key + 4, gc.key);
        return gc.exec;
    }

    hipGraphExec_t iteration_graph(const CgState &st)
    {
        // make every buffer the iteration touches exist before capture
        if (use_mf()) ensure_mf();
        if (opt.precision == AUX_MIXED) {
            ensure_fp32();
            work<float>();
        } else {
            work<double>();
        }
        // two iterations per graph: half the gaps between graph launches
        const int key[4] = {opt.precision, opt.op, st.maxit, 1};
        return captured(g_single, key, [&]() {
            cg_iteration(st, partials);
            cg_iteration(st, partials);
        });
    }

    void drop_graph()
    {
        g_single.drop();
        g_batch.drop();
    }

    int pcg(const double *f, double *u, double tol, int maxit, aux_solve_info *info)
    {
        if (maxit <= 0) maxit = opt.maxit;
        ensure_hist(maxit);
        return pcg_run(own_cg(), f, u, tol, maxit, info, opt.graph && !prof_on);
    }

    // The CG solve on the given buffers.  use_graph: replay two iterations
    // per captured graph (bound to the handle's own buffers); otherwise every
    // launch is enqueued directly, and nothing is allocated on this path once
    // the preconditioner's data for the current precision and operator exist.
    int pcg_run(const CgBufs &cb, const double *f, double *u, double tol, int maxit, aux_solve_info *info,
                bool use_graph)
    {
        auto t0 = std::chrono::steady_clock::now();
        hipStream_t s = stream;
        int n = disc.ndof;
        double *partials = cb.partials, *scal = cb.scal;
        int *istate = cb.istate;
        CgState st = cg_state(cb, maxit);
        vec_gather(s, n, perm, f, fi);
        vec_gather(s, n, perm, u, xi);
        sell_residual64(s, A.view<double>(), fi, xi, r);
        int g = vec_dot(s, n, fi, fi, partials);
        finish(s, partials, g, FIN_PLAIN, scal + 0, st);
        g = vec_dot(s, n, r, r, partials);
        finish(s, partials, g, FIN_PLAIN, scal + 1, st);
        cg_init(s, st, tol * tol);
        prof_tag = 0;
        g = apply(r, z, partials, st.done);
        finish(s, partials, g, FIN_RZ, nullptr, st);
        cg_direction(s, n, z, p, st);

        // two CG iterations as a HIP graph (its kernels have fixed arguments:
        // the iteration index and the stopping state live in device memory,
        // and iterations past the stop return at once); not used while kernel
        // timing records events
        hipGraphExec_t gexec = use_graph ? iteration_graph(st) : nullptr;
        int issued = 0, iter = 0, done = 0, chunk = 2;
        bool first_check = true;
        while (true) {
            for (int c = 0; c < chunk && issued < maxit;) {
                if (gexec) {
                    prof_tag = issued + 1;
                    HIPCHECK(hipGraphLaunch(gexec, s));
                    issued += 2;
                    c += 2;
                } else {
                    prof_tag = issued + 1;
                    cg_iteration(st, partials);
                    issued++;
                    c++;
                }
            }
            // one round trip per check: the status, the r.r values of the last
            // three issued iterations (unless the solve stopped, every issued
            // iteration ran, so they are those of iterations iter-2..iter) and,
            // on the first check, the stopping target, all into pinned memory
            HIPCHECK(hipMemcpyAsync(host_state, istate, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
            const int win = std::min(issued, maxit);
            if (win >= 2)
                HIPCHECK(hipMemcpyAsync(host_scal, st.rr + win - 2, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
            if (first_check)
                HIPCHECK(hipMemcpyAsync(host_scal + 3, st.scal + 2, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHECK(hipStreamSynchronize(s));
            first_check = false;
            iter = host_state[0];
            done = host_state[1];
            if (done || issued >= maxit) break;
            // predict the remaining iterations from the observed contraction
            chunk = 2;
            if (iter >= 2 && iter == win) {
                const double *rr = host_scal, target = host_scal[3];
                if (rr[2] > 0 && rr[0] > rr[2] && target > 0) {
                    double rate = std::sqrt(rr[2] / rr[0]);
                    double need = std::log(target / rr[2]) / std::log(rate);
                    chunk = (int)std::ceil(std::max(1.0, std::min(need, 16.0)));
                }
            }
        }
        vec_scatter(s, n, perm, xi, u);
        prof_tag = -1;
        prof_collect(iter);
        if (opt.true_residual) {
            // ||f - A_h u||_2 of the returned iterate (one more product)
            sell_residual64(s, A.view<double>(), fi, xi, r);
            const int g2 = vec_dot(s, n, r, r, partials);
            finish(s, partials, g2, FIN_PLAIN, scal + 3, st);
            HIPCHECK(hipMemcpyAsync(host_scal + 6, scal + 3, sizeof(double), hipMemcpyDeviceToHost, s));
        }
        HIPCHECK(hipMemcpyAsync(host_scal + 4, st.rr + iter, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipMemcpyAsync(host_scal + 5, scal + 0, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        const double rrv = host_scal[4], ffv = host_scal[5];
        last_rr = st.rr;
        last_iters = iter;
        last_ff = ffv;
        int status = AUX_OK;
        if (done == 2 || (done == 0 && issued >= maxit)) status = AUX_ENOTCONV;
        else if (done == 3) status = AUX_EBREAKDOWN;
        else if (done == 4) status = AUX_ENAN;
        if (info) {
            info->iterations = iter;
            info->status = status;
            info->rel_residual = ffv > 0 ? std::sqrt(rrv / ffv) : 0.0;
            info->seconds = seconds_since(t0);
            info->true_rel_residual = !opt.true_residual ? -1.0 : ffv > 0 ? std::sqrt(host_scal[6] / ffv) : 0.0;
        }
        return status;
    }

    // ------------------------------------------------------------ FGMRES
    // Flexible GMRES(m) (the Krylov method of the paper's Sec. 6.1; Saad's
    // flexible variant): basis V (m+1 vectors) and preconditioned vectors Z
    // (m) in HBM, the Hessenberg matrix and its Givens rotations on the host.
    static constexpr int kHs = kMaxRestart + 1;   // stride of the coefficient slots
    struct Fgm {
        int m = 0;
        size_t len = 0;           // vector length the basis holds
        double *V = nullptr, *Z = nullptr, *part = nullptr;
        double *dh = nullptr;     // [0, kHs) first pass, [kHs, 2 kHs) second pass, [2 kHs] w.w, then y
    } fg;
    double *fg_host = nullptr;    // pinned mirror of fg.dh

    void ensure_fgmres(int m, size_t len)
    {
        if (fg.m < m || fg.len < len) {
            dfree(fg.V);
            dfree(fg.Z);
            fg.m = std::max(fg.m, m);
            fg.len = std::max(fg.len, len);
            fg.V = dnew<double>((size_t)(fg.m + 1) * fg.len);
            fg.Z = dnew<double>((size_t)fg.m * fg.len);
        }
        if (!fg.part) {
            fg.part = dnew<double>((size_t)kKrylovBlocks * kHs);
            fg.dh = dnew<double>(4 * (size_t)kHs);
            HIPCHECK(hipHostMalloc((void **)&fg_host, 4 * kHs * sizeof(double), hipHostMallocDefault));
        }
    }

    // y = A_h x in FP64 by the operator of the solve
    void op_product(const double *x, double *y)
    {
        if (use_mf()) {
            ensure_mf();
            MfView<double> v = mf_view<double>();
            mf_apply<double>(stream, v, x, mf_Y64, nullptr);
            mf_product<double>(stream, v, mf_Y64, y, nullptr, nullptr, nullptr);
        } else {
            sell_spmv64(stream, A.view<double>(), x, y, nullptr, nullptr);
        }
    }

    // A system for the flexible GMRES core, on device vectors of length len
    // in the handle's internal layout.
    struct KrylovSystem {
        size_t len;
        std::function<void(const double *, double *)> prec;                        // z = M v
        std::function<void(const double *, double *)> op;                          // w = F z
        std::function<void(const double *, const double *, double *)> residual;    // r = b - F x
    };

    int fgmres(const double *b, double *x, double tol, int m, int maxit, double *history, aux_solve_info *info)
    {
        auto t0 = std::chrono::steady_clock::now();
        const int n = disc.ndof;
        if (use_mf()) ensure_mf();
        vec_gather(stream, n, perm, b, fi);
        vec_gather(stream, n, perm, x, xi);
        KrylovSystem K{(size_t)n, [&](const double *v, double *z) { apply(v, z, nullptr, nullptr); },
                       [&](const double *z, double *w) { op_product(z, w); },
                       [&](const double *bb, const double *xx, double *r) {
                           sell_residual64(stream, A.view<double>(), bb, xx, r);
                       }};
        const int status = fgmres_core(K, fi, xi, tol, m, maxit, history, info);
        vec_scatter(stream, n, perm, xi, x);
        HIPCHECK(hipStreamSynchronize(stream));
        prof_collect(0);
        if (info) info->seconds = seconds_since(t0);
        return status;
    }

    // Flexible GMRES(m) on F x = b (internal layout, x updated in place):
    // returns the status and fills info except its time.
    int fgmres_core(const KrylovSystem &K, const double *b, double *x, double tol, int m, int maxit, double *history,
                    aux_solve_info *info)
    {
        if (maxit <= 0) maxit = opt.maxit;
        hipStream_t s = stream;
        const size_t len = K.len;
        const int n = (int)len;
        const long long ld = (long long)len;
        ensure_fgmres(m, len);
        double *V = fg.V, *Z = fg.Z, *hh = fg_host;
        double *h1 = fg.dh, *h2 = fg.dh + kHs, *nrm = fg.dh + 2 * kHs, *yd = fg.dh + 2 * kHs + 1;
        // v_0 <- r = b - F x (unnormalised) and ||r||
        auto residual_norm = [&]() {
            K.residual(b, x, V);
            multi_dot(s, n, 1, V, ld, V, fg.part, nrm);
            HIPCHECK(hipMemcpyAsync(hh + 2 * kHs, nrm, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHECK(hipStreamSynchronize(s));
            return std::sqrt(hh[2 * kHs]);
        };
        double beta = residual_norm();
        const double r0 = beta;
        if (history) history[0] = r0;
        int it = 0, status = AUX_ENOTCONV;
        std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
        auto Hc = [&](int i, int j) -> double & { return H[(size_t)i * m + j]; };
        if (!std::isfinite(beta)) status = AUX_ENAN;
        else if (beta == 0.0) status = AUX_OK;
        while (status == AUX_ENOTCONV && it < maxit) {
            scale_unit(s, n, V, nrm, V);
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            int jend = 0;
            bool stop = false;
            for (int j = 0; j < m && it < maxit; j++) {
                double *vj = V + j * ld, *zj = Z + j * ld, *w = V + (j + 1) * ld;
                K.prec(vj, zj);
                K.op(zj, w);
                // classical Gram-Schmidt, once (PETSc's default for its
                // GMRES) or twice (option gram_schmidt)
                multi_dot(s, n, j + 1, V, ld, w, fg.part, h1);
                if (opt.gram_schmidt == 2) {
                    multi_axpy(s, n, j + 1, V, ld, h1, -1.0, w, nullptr, nullptr);
                    multi_dot(s, n, j + 1, V, ld, w, fg.part, h2);
                    multi_axpy(s, n, j + 1, V, ld, h2, -1.0, w, fg.part, nrm);
                } else {
                    multi_axpy(s, n, j + 1, V, ld, h1, -1.0, w, fg.part, nrm);
                }
                scale_unit(s, n, w, nrm, w);
                HIPCHECK(hipMemcpyAsync(hh, h1, (size_t)(j + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
                if (opt.gram_schmidt == 2)
                    HIPCHECK(hipMemcpyAsync(hh + kHs, h2, (size_t)(j + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
                else
                    for (int i = 0; i <= j; i++) hh[kHs + i] = 0.0;
                HIPCHECK(hipMemcpyAsync(hh + 2 * kHs, nrm, sizeof(double), hipMemcpyDeviceToHost, s));
                HIPCHECK(hipStreamSynchronize(s));
                for (int i = 0; i <= j; i++) Hc(i, j) = hh[i] + hh[kHs + i];
                const double hn = std::sqrt(hh[2 * kHs]);
                Hc(j + 1, j) = hn;
                // the rotations so far on the new column, then a new one that
                // zeroes its subdiagonal entry; g stays Q^T beta e_1
                for (int i = 0; i < j; i++) {
                    const double u0 = Hc(i, j), u1 = Hc(i + 1, j);
                    Hc(i, j) = cs[i] * u0 + sn[i] * u1;
                    Hc(i + 1, j) = cs[i] * u1 - sn[i] * u0;
                }
                const double dj = Hc(j, j), ej = Hc(j + 1, j), rad = std::sqrt(dj * dj + ej * ej);
                cs[j] = rad > 0.0 ? dj / rad : 1.0;
                sn[j] = rad > 0.0 ? ej / rad : 0.0;
                Hc(j, j) = rad;
                Hc(j + 1, j) = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] *= cs[j];
                it++;
                jend = j + 1;
                const double est = std::fabs(g[j + 1]);
                if (history) history[it] = est;
                if (!std::isfinite(est)) {
                    status = AUX_ENAN;
                    stop = true;
                    break;
                }
                if (est <= tol * r0) {
                    status = AUX_OK;
                    stop = true;
                    break;
                }
                if (hn == 0.0) break;   // the space holds the solution
            }
            if (status == AUX_ENAN) break;
            // y = R^-1 g (upper triangular), x += Z y
            for (int i = jend - 1; i >= 0; i--) {
                double t = g[i];
                for (int k = i + 1; k < jend; k++) t -= Hc(i, k) * y[k];
                y[i] = t / Hc(i, i);
            }
            std::copy(y.begin(), y.begin() + jend, hh + 2 * kHs + 1);
            HIPCHECK(hipMemcpyAsync(yd, hh + 2 * kHs + 1, (size_t)jend * sizeof(double), hipMemcpyHostToDevice, s));
            multi_axpy(s, n, jend, Z, ld, yd, 1.0, x, nullptr, nullptr);
            beta = residual_norm();   // the true residual; also v_0 of the next cycle
            if (stop) break;
            if (!std::isfinite(beta)) status = AUX_ENAN;
            else if (beta == 0.0) status = AUX_OK;
        }
        if (info) {
            info->iterations = it;
            info->status = status;
            info->rel_residual = r0 > 0.0 ? beta / r0 : 0.0;
        }
        return status;
    }

    // ------------------------------------------------------------ Stokes
    // Hood-Taylor P^k-P^{k-1} Stokes system (Sec. 5) on the handle's mesh,
    //   F = [A  B^T; B  0],  A = diag(A_h, A_h, A_h),
    // with the block triangular preconditioner (Sec. 5, Q_t)
    //   Q_t = [A  B^T; 0  -S]^{-1},  S replaced by the pressure mass matrix
    // M_p and A^{-1} by the auxiliary-space preconditioner B per component:
    //   y_p = -M_p^{-1} r_p  (diagonal PCG from zero to a relative 1e-6, at
    //   most 200 steps),  y_c = B (r_c - (B^T y_p)_c).
    // Internal layout of a Stokes vector: the three velocity components, each
    // in the internal dof order, then the pressure in its key order.
    static constexpr double kMassTol = 1e-6;
    static constexpr int kMassMaxit = 200;
    struct StokesData {
        bool host_ready = false, ready = false;
        int np = 0;
        Csr B, Mp;                   // host, external numbering
        std::vector<int32_t> pkeys;  // [np][k-1] pressure node keys
        DevOp Bi, BTi, M;            // FP64 device operators, internal velocity order
        double *mdinv = nullptr;     // 1 / diag(M_p)
        double *mx = nullptr, *mr = nullptr, *mz = nullptr, *mp = nullptr, *mq = nullptr;
        double *t3 = nullptr;        // velocity scratch [3 n_h]
        double *bi = nullptr, *xi = nullptr;   // internal right-hand side and iterate
        double *part = nullptr, *scal = nullptr, *hist = nullptr;
        int *istate = nullptr;
        int *host_state = nullptr;   // pinned: iterations, stop flag
        int mass_chunk = 8;          // mass-CG steps enqueued before the first check
        int64_t mass_solves = 0, mass_steps = 0;
    } sk;

    void stokes_host()
    {
        if (sk.host_ready) return;
        try {
            build_stokes(disc, sk.B, sk.Mp, sk.pkeys);
        } catch (const std::invalid_argument &e) {
            throw AuxError(AUX_EINVAL, e.what());
        }
        sk.np = sk.B.n;
        sk.host_ready = true;
    }

    void stokes_setup()
    {
        stokes_host();
        if (sk.ready || host_only) return;
        const int n = disc.ndof, np = sk.np;
        std::vector<int> map3((size_t)3 * n);
        for (int c = 0; c < 3; c++)
            for (int i = 0; i < n; i++) map3[(size_t)c * n + i] = c * n + sell.iperm[i];
        Csr Bi = renumber_cols(sk.B, map3, 3 * n), BTi = transpose(Bi);
        sk.Bi = upload_op(Bi);
        sk.BTi = upload_op(BTi);
        sk.M = upload_op(sk.Mp);
        // storage of B and B^T (FP64 products), timed as the V-cycle's
        if (opt.sell_window <= 0) {
            const size_t fb = (size_t)512 << 20;
            void *flush = dalloc(fb);
            tune_op_t<double>(sk.Bi, 0, flush, fb);
            tune_op_t<double>(sk.BTi, 0, flush, fb);
            dfree(flush);
        }
        std::vector<double> dinv(np, 0.0);
        for (int i = 0; i < np; i++)
            for (int e = sk.Mp.ptr[i]; e < sk.Mp.ptr[i + 1]; e++)
                if (sk.Mp.col[e] == i) dinv[i] = 1.0 / sk.Mp.val[e];
        sk.mdinv = upload(dinv);
        for (double **v : {&sk.mx, &sk.mr, &sk.mz, &sk.mp, &sk.mq}) *v = dnew<double>(np);
        sk.t3 = dnew<double>((size_t)3 * n);
        sk.bi = dnew<double>((size_t)3 * n + np);
        sk.xi = dnew<double>((size_t)3 * n + np);
        sk.part = dnew<double>(2 * (size_t)kMaxBlocks);
        sk.scal = dnew<double>(8);
        sk.hist = dnew<double>(3 * (size_t)(kMassMaxit + 2));
        sk.istate = (int *)dnew<double>(2);
        HIPCHECK(hipHostMalloc((void **)&sk.host_state, 2 * sizeof(int), hipHostMallocDefault));
        host_bufs.push_back(sk.host_state);
        sk.ready = true;
    }

    size_t stokes_len() const { return (size_t)3 * disc.ndof + sk.np; }

    // sk.mx = M_p^{-1} b (device b [n_p]) by diagonal PCG from zero, stopped
    // at ||r|| <= 1e-6 ||b|| or 200 steps.  The steps run with their state in
    // device memory, five launches each (product, p.q, update, r.r and r.z,
    // direction); the host enqueues as many as the last solve took (plus
    // one) and then two at a time until the stop flag is set.  Returns the
    // step count.
    // count steps of the mass-matrix CG, enqueued on the handle's stream
    void mass_steps(int count, const CgState &st)
    {
        hipStream_t s = stream;
        const DevCsrView Mv = sk.M.view<double>();
        for (int c = 0; c < count; c++) {
            int g = mass_product(s, Mv, sk.mp, sk.mq, sk.part, st);
            finish(s, sk.part, g, FIN_PQ, nullptr, st);
            g = mass_update(s, sk.np, sk.mx, sk.mr, sk.mp, sk.mq, sk.mdinv, sk.mz, sk.part, st);
            mass_finish(s, sk.part, g, st);
            cg_direction(s, sk.np, sk.mz, sk.mp, st);
        }
    }

    int mass_solve(const double *b)
    {
        hipStream_t s = stream;
        const int np = sk.np;
        CgState st = cg_state(CgBufs{sk.part, sk.scal, sk.istate, sk.hist, kMassMaxit + 2}, kMassMaxit);
        double *part_rz = sk.part + kMaxBlocks;
        int g = mass_start(s, np, b, sk.mdinv, sk.mx, sk.mr, sk.mz, sk.part);
        finish(s, sk.part, g, FIN_PLAIN, sk.scal + 0, st);
        finish(s, sk.part, g, FIN_PLAIN, sk.scal + 1, st);
        cg_init(s, st, kMassTol * kMassTol);
        finish(s, part_rz, g, FIN_RZ, nullptr, st);
        cg_direction(s, np, sk.mz, sk.mp, st);
        int issued = 0, chunk = sk.mass_chunk;
        while (true) {
            const int cnt = std::min(chunk, kMassMaxit - issued);
            mass_steps(cnt, st);
            issued += cnt;
            HIPCHECK(hipMemcpyAsync(sk.host_state, sk.istate, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHECK(hipStreamSynchronize(s));
            if (sk.host_state[1] || issued >= kMassMaxit) break;
            chunk = 2;
        }
        const int steps = sk.host_state[0];
        sk.mass_chunk = std::max(2, steps + 1);
        sk.mass_solves++;
        sk.mass_steps += steps;
        return steps;
    }

    // y = F x (internal layout)
    void stokes_product(const double *x, double *y)
    {
        const size_t n = disc.ndof;
        for (int c = 0; c < 3; c++) op_product(x + c * n, y + c * n);
        csr_matvec_add<double>(stream, sk.BTi.view<double>(), x + 3 * n, y, nullptr);   // y_u += B^T x_p
        csr_matvec<double>(stream, sk.Bi.view<double>(), x, y + 3 * n, nullptr);        // y_p = B x_u
    }

    // y = Q_t r (internal layout)
    void stokes_qt(const double *r, double *y)
    {
        const size_t n = disc.ndof, nu = 3 * n;
        mass_solve(r + nu);                                   // mx = M_p^{-1} r_p
        vec_negate(stream, sk.np, sk.mx, y + nu);             // y_p = -M_p^{-1} r_p
        HIPCHECK(hipMemcpyAsync(sk.t3, r, nu * sizeof(double), hipMemcpyDeviceToDevice, stream));
        csr_matvec_add<double>(stream, sk.BTi.view<double>(), sk.mx, sk.t3, nullptr);   // r_u - B^T y_p
        for (int c = 0; c < 3; c++) apply(sk.t3 + c * n, y + c * n, nullptr, nullptr);
    }

    // external <-> internal Stokes vectors
    void stokes_in(const double *ext, double *in)
    {
        const size_t n = disc.ndof;
        for (int c = 0; c < 3; c++) vec_gather(stream, (int)n, perm, ext + c * n, in + c * n);
        HIPCHECK(hipMemcpyAsync(in + 3 * n, ext + 3 * n, (size_t)sk.np * sizeof(double), hipMemcpyDeviceToDevice,
                                stream));
    }
    void stokes_out(const double *in, double *ext)
    {
        const size_t n = disc.ndof;
        for (int c = 0; c < 3; c++) vec_scatter(stream, (int)n, perm, in + c * n, ext + c * n);
        HIPCHECK(hipMemcpyAsync(ext + 3 * n, in + 3 * n, (size_t)sk.np * sizeof(double), hipMemcpyDeviceToDevice,
                                stream));
    }

    void stokes_prepare()
    {
        stokes_setup();
        if (use_mf()) ensure_mf();
        if (opt.precision == AUX_MIXED) ensure_fp32();
    }

    void stokes_operator_external(const double *x, double *y)
    {
        stokes_prepare();
        stokes_in(x, sk.bi);
        stokes_product(sk.bi, sk.xi);
        stokes_out(sk.xi, y);
    }

    void stokes_qt_external(const double *r, double *y)
    {
        stokes_prepare();
        stokes_in(r, sk.bi);
        stokes_qt(sk.bi, sk.xi);
        stokes_out(sk.xi, y);
    }

    int stokes_fgmres(const double *b, double *x, double tol, int m, int maxit, double *history, aux_solve_info *info)
    {
        auto t0 = std::chrono::steady_clock::now();
        stokes_prepare();
        stokes_in(b, sk.bi);
        stokes_in(x, sk.xi);
        const size_t len = stokes_len();
        KrylovSystem K{len, [&](const double *v, double *z) { stokes_qt(v, z); },
                       [&](const double *z, double *w) { stokes_product(z, w); },
                       [&](const double *bb, const double *xx, double *r) {
                           stokes_product(xx, r);
                           sub_from(stream, (int)len, bb, r);
                       }};
        const int status = fgmres_core(K, sk.bi, sk.xi, tol, m, maxit, history, info);
        stokes_out(sk.xi, x);
        HIPCHECK(hipStreamSynchronize(stream));
        if (info) info->seconds = seconds_since(t0);
        return status;
    }

    // ------------------------------------------------------------ batched order
    // The block kernels gather an NR-word block row for every entry, so their
    // speed depends on the gathered rows staying in a die's L2.  With
    // batch_order = 1 they run in a dof order of their own: the dofs along
    // the Morton curve of their node positions (so any run of rows is a
    // compact region), rows sorted by length within windows of kBatchWindow
    // rows (short slices), and each die takes a contiguous range of A_h's
    // slices balanced by stored entries (its gathers stay in one region).
    // At P2 64^3 with 32 columns this halves the bytes the block products
    // fetch past L2 (FP64 product 8.9 -> 4.2 GB per launch, L2 hits 30 ->
    // 62 %) without making them faster (L2 misses do not bound them; each
    // entry still gathers an NR-word block row through L1).
    // batch_order = 0 (default) keeps the single-vector order (round-robin
    // slices).
    static constexpr int kBatchWindow = 2048;
    static constexpr int kDies = 8;
    struct BOrder {
        bool ready = false;
        std::vector<int> perm;           // batched row -> external dof
        std::vector<int> from_single;    // single-vector internal row -> batched row
        DevSell A;
        int *die_off = nullptr;          // [kDies + 1] slice ranges, or null (round-robin)
        int *perm_d = nullptr;
        double *dinv64 = nullptr;
        float *dinv32 = nullptr;
        Csr Am;                          // A_h in the Morton order (host, until the tiles are built)
        std::vector<int> m2b;            // Morton position -> batched row
    } bo;

    void ensure_border()
    {
        ensure_host_values();
        if (bo.ready) return;
        ensure_fp32();
        const int n = disc.ndof;
        if (!opt.batch_order) {
            // the single-vector layout as it is
            bo.perm = sell.perm;
            bo.from_single.resize(n);
            std::iota(bo.from_single.begin(), bo.from_single.end(), 0);
            bo.A = A;
            bo.perm_d = perm;
            bo.dinv64 = dinv64;
            bo.dinv32 = dinv32;
            bo.Am = disc.A;
            bo.m2b = sell.iperm;
            bo.ready = true;
            return;
        }
        std::vector<double> pos((size_t)3 * n);
        for (int i = 0; i < n; i++)
            for (int c = 0; c < 3; c++) {
                double t = 0.0;
                for (int p = 0; p < disc.k; p++) t += disc.xyz[3 * (size_t)disc.keys[(size_t)i * disc.k + p] + c];
                pos[3 * (size_t)i + c] = t / disc.k;
            }
        const std::vector<int> mo = morton_order(pos, n);     // Morton position -> external dof
        std::vector<int> imo(n);
        for (int r = 0; r < n; r++) imo[mo[r]] = r;
        bo.Am = permute_symmetric(disc.A, mo, imo);
        Sell sl;
        build_sell(bo.Am, kSlice, kBatchWindow, false, sl);
        bo.perm.resize(n);
        for (int r = 0; r < n; r++) bo.perm[r] = mo[sl.perm[r]];
        bo.m2b = sl.iperm;
        std::vector<int> iperm(n);
        for (int r = 0; r < n; r++) iperm[bo.perm[r]] = r;
        bo.from_single.resize(n);
        for (int i = 0; i < n; i++) bo.from_single[i] = iperm[sell.perm[i]];
        bo.A = upload_sell(sl);
        bo.A.v32 = upload(to_f32(sl.val));
        // die ranges of equal stored entries
        std::vector<int> off(kDies + 1, 0);
        const double total = (double)sl.slice_off[sl.nslices];
        int d = 1;
        for (int sidx = 0; sidx < sl.nslices && d < kDies; sidx++)
            while (d < kDies && (double)sl.slice_off[sidx + 1] >= total * d / kDies) off[d++] = sidx + 1;
        while (d <= kDies) off[d++] = sl.nslices;
        bo.die_off = upload(off);
        bo.perm_d = upload(bo.perm);
        std::vector<double> l1b(n);
        for (int r = 0; r < n; r++) l1b[r] = disc.l1[bo.perm[r]];
        bo.dinv64 = upload(smoother_inv(l1b));
        bo.dinv32 = upload(to_f32(smoother_inv(l1b)));
        if (!opt.batch_tiles) {
            bo.Am = Csr();
            bo.m2b.clear();
        }
        bo.ready = true;
    }
    template <typename T>
    DevSellView bview() const
    {
        DevSellView v = bo.A.view<T>();
        v.die_off = bo.die_off;
        return v;
    }
    template <typename T>
    const T *bdinv() const
    {
        if constexpr (std::is_same<T, float>::value) return bo.dinv32;
        else return bo.dinv64;
    }

    // ------------------------------------------------------------ batched CG
    struct Batch {
        int nr = 0, hist_cap = 0;
        double *X = nullptr, *R = nullptr, *Z = nullptr, *P = nullptr, *Q = nullptr, *F = nullptr;
        double *partials = nullptr, *ff = nullptr, *rr0 = nullptr, *tol2ff = nullptr, *hist = nullptr;
        int *ist = nullptr;            // k, all_done, iter[nr], done[nr]
        int layout32 = -1, layout64 = -1;   // tile size index of the block products, -1 slices
        int *host = nullptr;           // pinned copy of ist
        Work<double> w64;
        Work<float> w32;
    } bt;

    void ensure_batch(int nr, int maxit)
    {
        int n = disc.ndof;
        ensure_fp32();
        ensure_border();
        if (bt.nr != nr) {
            release_batch();
            bt.nr = nr;
            size_t blk = (size_t)n * nr;
            bt.X = dnew<double>(blk);
            bt.R = dnew<double>(blk);
            bt.Z = dnew<double>(blk);
            bt.P = dnew<double>(blk);
            bt.Q = dnew<double>(blk);
            bt.F = dnew<double>(blk);
            bt.partials = dnew<double>((size_t)kMaxBlocks * nr);
            bt.ff = dnew<double>(nr);
            bt.rr0 = dnew<double>(nr);
            bt.tol2ff = dnew<double>(nr);
            bt.ist = dnew<int>(2 + 2 * (size_t)nr);
            HIPCHECK(hipHostMalloc((void **)&bt.host, (2 + 2 * (size_t)nr) * sizeof(int), hipHostMallocDefault));
            host_bufs.push_back(bt.host);
            tune_batch_layout();
        }
        if (maxit + 2 > bt.hist_cap) {
            dfree(bt.hist);
            bt.hist_cap = maxit + 2;
            bt.hist = dnew<double>((size_t)3 * bt.hist_cap * nr);
        }
    }

    // The batched autotuner: for the current block width, time the block
    // products of A_h with 64-row slices and with each tile size whose LDS
    // fits (an FP32 sweep for the preconditioner, an FP64 product for CG) and
    // keep the fastest per precision.
    double time_block(const std::function<void()> &f)
    {
        hipEvent_t a = take_event(), b = take_event();
        f();
        HIPCHECK(hipEventRecord(a, stream));
        for (int i = 0; i < 3; i++) f();
        HIPCHECK(hipEventRecord(b, stream));
        HIPCHECK(hipEventSynchronize(b));
        float ms = 0.f;
        HIPCHECK(hipEventElapsedTime(&ms, a, b));
        ev_used -= 2;
        return ms;
    }

    void tune_batch_layout()
    {
        bt.layout32 = bt.layout64 = -1;
        // 0: slices; with a fixed layout window every choice is rule-based (slices)
        if (!opt.batch_tiles || (opt.batch_tiles == 1 && opt.sell_window > 0)) return;
        ensure_tiles();
        if (opt.batch_tiles == 2) {                    // the largest tile whose LDS fits
            for (int k = 0; k < kTileSizes; k++) {
                if (btile_lds(tiles[k].view<float>(), bt.nr, 4)) bt.layout32 = k;
                if (btile_lds(tiles[k].view<double>(), bt.nr, 8)) bt.layout64 = k;
            }
            return;
        }
        ensure_fp32();
        const int nr = bt.nr;
        const size_t blk = (size_t)disc.ndof * nr;
        float *z0 = dnew<float>(blk), *z1 = dnew<float>(blk), *rh = dnew<float>(blk);
        HIPCHECK(hipMemsetAsync(z0, 0, blk * sizeof(float), stream));
        HIPCHECK(hipMemsetAsync(rh, 0, blk * sizeof(float), stream));
        HIPCHECK(hipMemsetAsync(bt.P, 0, blk * sizeof(double), stream));
        double best32 = time_block([&]() {
            bsell_sweep<float, float, float>(stream, nr, bview<float>(), bo.dinv32, rh, z0, z1, nullptr, nullptr, nullptr);
        });
        double best64 = time_block([&]() { bsell_spmv64(stream, nr, bview<double>(), bt.P, bt.Q, nullptr, nullptr); });
        for (int k = 0; k < kTileSizes; k++) {
            if (btile_lds(tiles[k].view<float>(), nr, 4)) {
                double ms = time_block([&]() {
                    btile_sweep<float, float, float>(stream, nr, tiles[k].view<float>(), bo.dinv32, rh, z0, z1,
                                                     nullptr, nullptr, nullptr);
                });
                if (ms < best32) {
                    best32 = ms;
                    bt.layout32 = k;
                }
            }
            if (btile_lds(tiles[k].view<double>(), nr, 8)) {
                double ms = time_block(
                    [&]() { btile_spmv64(stream, nr, tiles[k].view<double>(), bt.P, bt.Q, nullptr, nullptr); });
                if (ms < best64) {
                    best64 = ms;
                    bt.layout64 = k;
                }
            }
        }
        dfree(z0);
        dfree(z1);
        dfree(rh);
    }

    // device buffers of the current block width (the pinned status copy
    // stays with the handle)
    void release_batch()
    {
        g_batch.drop();
        for (double *b : {bt.X, bt.R, bt.Z, bt.P, bt.Q, bt.F, bt.partials, bt.ff, bt.rr0, bt.tol2ff, bt.hist})
            dfree(b);
        dfree(bt.ist);
        release_work(bt.w64);
        release_work(bt.w32);
        bt = Batch();
    }

    template <typename T>
    void release_work(Work<T> &w)
    {
        for (T *b : {w.za, w.zb, w.res, w.rT, w.nb, w.ne}) dfree(b);
        for (auto *v : {&w.b, &w.x, &w.r, &w.y})
            for (T *b : *v) dfree(b);
        w = Work<T>();
    }

    template <typename T>
    Work<T> &bwork()
    {
        Work<T> *w;
        if constexpr (std::is_same<T, float>::value) w = &bt.w32;
        else w = &bt.w64;
        if (!w->ready) {
            size_t n = (size_t)disc.ndof * bt.nr;
            w->za = dnew<T>(n);
            w->zb = dnew<T>(n);
            w->res = dnew<T>(n);
            if (std::is_same<T, float>::value) w->rT = dnew<T>(n);
            for (auto &L : lev) {
                size_t m = (size_t)L.A.n * bt.nr;
                w->b.push_back(dnew<T>(m));
                w->x.push_back(dnew<T>(m));
                w->r.push_back(dnew<T>(m));
                w->y.push_back(dnew<T>(m));
            }
            w->ready = true;
        }
        return *w;
    }

    BCgState bstate(int maxit)
    {
        int nr = bt.nr;
        return {bt.ist, bt.ist + 2, bt.ist + 2 + nr, bt.ist + 1, bt.hist, bt.hist + (size_t)bt.hist_cap * nr,
                bt.hist + (size_t)2 * bt.hist_cap * nr, bt.tol2ff, maxit};
    }

    // Operators of the V-cycle and the transfers for the block kernels:
    // row-permuted sliced ELL (rows sorted by length within 4096-row windows,
    // results written back to the original rows), FP64 and FP32 values.
    struct BOp {
        DevSell m;
        int *perm = nullptr;
        // level matrices only: the values of A D^-1 (D = diag of the l1
        // norms), formed in FP64 and rounded once, in the same layout, so
        // the pre-smoothing residual b - A D^-1 b gathers b alone
        double *s64 = nullptr;
        float *s32 = nullptr;
        int unroll = 1;          // slots in flight per lane in the block kernels
        template <typename T>
        DevSellView view() const { return m.view<T>(); }
        template <typename T>
        DevSellView scaled_view() const
        {
            DevSellView v = m.view<T>();
            v.val = std::is_same<T, float>::value ? (const void *)s32 : (const void *)s64;
            return v;
        }
    };
    std::vector<BOp> bA, bP, bR;
    BOp bIP, bIR, bRF;
    bool bops_ready = false;

    // A_h as row tiles (16, 32 and 64 consecutive original rows) for the
    // block products; a launch uses the largest tile whose LDS fits
    static constexpr int kTileSizes = 3;
    DevTiles tiles[kTileSizes];
    bool tiles_ready = false;

    void ensure_tiles()
    {
        if (tiles_ready || !opt.batch_tiles) return;
        const int sizes[kTileSizes] = {16, 32, 64};
        for (int k = 0; k < kTileSizes; k++) {
            Tiles h;
            build_tiles(bo.Am, bo.m2b, sizes[k], h);
            DevTiles &d = tiles[k];
            d.n = h.n;
            d.tile = h.tile;
            d.ntiles = h.ntiles;
            d.max_cols = h.max_cols;
            d.max_entries = h.max_entries;
            d.rows = upload(h.rows);
            d.row_ptr = upload(h.row_ptr);
            d.col_off = upload(h.col_off);
            d.ucols = upload(h.ucols);
            d.lidx = upload(h.lidx);
            d.v64 = upload(h.val);
            d.v32 = upload(to_f32(h.val));
        }
        tiles_ready = true;
        bo.Am = Csr();
        bo.m2b.clear();
    }

    // tile layout the batched autotuner chose for values of type T at the
    // current block width, or null (slice kernels)
    template <typename T>
    const DevTiles *tiles_for(int nr) const
    {
        const int k = std::is_same<T, float>::value ? bt.layout32 : bt.layout64;
        if (!tiles_ready || k < 0 || bt.nr != nr) return nullptr;
        return &tiles[k];
    }

    static constexpr double kLongRow = 8.0;   // mean entries per row
    static constexpr int kFewSlices = 512;
    BOp upload_bop(const Csr &op)
    {
        Sell sl;
        build_sell(op, kSlice, kSellWindow, false, sl, false);
        BOp b;
        b.m = upload_sell(sl);
        b.m.v32 = upload(to_f32(sl.val));
        b.perm = upload(sl.perm);
        // long rows (level matrices, restrictions) take the unrolled kernels,
        // and so do small operators, whose few slices leave the chip idle and
        // make every pass latency-bound; the short rows (a few entries) of
        // the large prolongations do not
        const bool long_rows = (double)op.col.size() >= kLongRow * op.n;
        b.unroll = op.n > 0 && (long_rows || sl.nslices < kFewSlices) ? 4 : 1;
        return b;
    }

    void ensure_bops()
    {
        ensure_host_values();
        ensure_host_hierarchy();
        if (bops_ready) return;
        const size_t L = hier.levels.size();
        bA.resize(L);
        bP.resize(L);
        bR.resize(L);
        // The block kernels are bound by the bytes gathered per entry
        // (NR words each), where the composite level operators' scattered
        // coarse-row gathers cost more than the two extra passes save; they
        // keep the four-pass cycle and fuse only the restricted residual.
        for (size_t l = 0; l < L; l++) {
            const AmgLevel &hl = hier.levels[l];
            if (l + 1 == L) continue;                 // coarsest: dense inverse
            bA[l] = upload_bop(hl.A);
            Csr ad = hl.A;
            for (size_t e = 0; e < ad.val.size(); e++) ad.val[e] /= hl.l1[ad.col[e]];
            Sell sl;
            build_sell(ad, kSlice, kSellWindow, false, sl, false);
            bA[l].s64 = upload(sl.val);
            bA[l].s32 = upload(to_f32(sl.val));
            bP[l] = upload_bop(hl.P);
            bR[l] = upload_bop(hl.R);
        }
        if (L) {
            ensure_border();
            // P^k rows / columns in the batched order
            bIP = upload_bop(permute_rows(disc.IP, bo.perm));
            if (opt.fuse_cycle) bRF = upload_bop(renumber_cols(RF_host, bo.from_single, disc.ndof));
            else bIR = upload_bop(renumber_cols(IRi, bo.from_single, disc.ndof));
        }
        bops_ready = true;
    }

    template <typename T>
    const T *bvcycle(size_t l, const int *all_done)
    {
        Work<T> &w = bwork<T>();
        hipStream_t s = stream;
        const int nr = bt.nr;
        const Lev &L = lev[l];
        if (l + 1 == lev.size()) {
            bdense<T>(s, nr, L.A.n, cinv<T>(), w.b[l], w.x[l], all_done);
            return w.x[l];
        }
        if (l == dense_first) {
            bdense<T>(s, nr, L.A.n, dcyc<T>(), w.b[l], w.y[l], all_done);
            return w.y[l];
        }
        const BOp &A_ = bA[l], &P_ = bP[l], &R_ = bR[l];
        blevel_vpre<T>(s, nr, A_.scaled_view<T>(), A_.unroll, A_.perm, ldinv<T>(l), w.b[l], w.x[l], w.r[l], all_done);
        blevel_matvec<T>(s, nr, R_.view<T>(), R_.unroll, R_.perm, w.r[l], w.b[l + 1], false, all_done);
        const T *e = bvcycle<T>(l + 1, all_done);
        blevel_matvec<T>(s, nr, P_.view<T>(), P_.unroll, P_.perm, e, w.x[l], true, all_done);
        blevel_sweep<T>(s, nr, A_.view<T>(), A_.unroll, A_.perm, ldinv<T>(l), w.b[l], w.x[l], w.y[l], all_done);
        return w.y[l];
    }

    // Zout = B Rin for the nr columns of a block (internal order)
    template <typename T>
    int bapply_B(const double *Rin, T *Zout, double *rz_partials, const int *all_done, bool prepped = false)
    {
        Work<T> &w = bwork<T>();
        hipStream_t s = stream;
        const int nr = bt.nr;
        DevSellView Av = bview<T>();
        const DevTiles *tl = tiles_for<T>(nr);
        const T *d = bdinv<T>();
        const int nu = opt.nu;
        T *rTbuf = std::is_same<T, float>::value ? w.rT : nullptr;
        T *zc = w.za, *zn = w.zb;
        int pb = pbeg(AUX_PROF_APPLY);
        int pk = -1;
        if (!prepped) {
            pk = pbeg(AUX_PROF_PK_FIRST);
            bjacobi0<T>(s, nr, disc.ndof, d, Rin, zc, rTbuf, all_done);
            pend(pk);
        }
        const T *rT = rTbuf ? (const T *)rTbuf : (const T *)(const void *)Rin;
        for (int k = 1; k < nu; k++) {
            pk = pbeg(AUX_PROF_PK_SWEEP);
            if (tl) btile_sweep<T, T, T>(s, nr, tl->view<T>(), d, rT, zc, zn, nullptr, nullptr, all_done);
            else bsell_sweep<T, T, T>(s, nr, Av, d, rT, zc, zn, nullptr, nullptr, all_done);
            pend(pk);
            std::swap(zc, zn);
        }
        if (!lev.empty()) {
            pk = pbeg(AUX_PROF_PK_RESID);
            if (opt.fuse_cycle) {
                blevel_matvec2<T>(s, nr, bRF.view<T>(), bRF.unroll, bRF.perm, rT, zc, disc.ndof, w.b[0], all_done);
                pend(pk);
                pk = pbeg(AUX_PROF_COARSE);
            } else {
                if (tl) btile_resid<T>(s, nr, tl->view<T>(), rT, zc, w.res, all_done);
                else bsell_resid<T>(s, nr, Av, rT, zc, w.res, all_done);
                pend(pk);
                pk = pbeg(AUX_PROF_COARSE);
                blevel_matvec<T>(s, nr, bIR.view<T>(), bIR.unroll, bIR.perm, w.res, w.b[0], false, all_done);
            }
            const T *e0 = bvcycle<T>(0, all_done);
            blevel_matvec<T>(s, nr, bIP.view<T>(), bIP.unroll, bIP.perm, e0, zc, true, all_done);
            pend(pk);
        }
        for (int k = 1; k < nu; k++) {
            pk = pbeg(AUX_PROF_PK_SWEEP);
            if (tl) btile_sweep<T, T, T>(s, nr, tl->view<T>(), d, rT, zc, zn, nullptr, nullptr, all_done);
            else bsell_sweep<T, T, T>(s, nr, Av, d, rT, zc, zn, nullptr, nullptr, all_done);
            pend(pk);
            std::swap(zc, zn);
        }
        pk = pbeg(AUX_PROF_PK_LAST);
        int g = tl ? btile_sweep<T, double, T>(s, nr, tl->view<T>(), d, Rin, zc, Zout, Rin, rz_partials, all_done)
                   : bsell_sweep<T, double, T>(s, nr, Av, d, Rin, zc, Zout, Rin, rz_partials, all_done);
        pend(pk);
        pend(pb);
        return g;
    }

    // Z = B R into the z block.  In mixed mode the last sweep's values are
    // FP32 results, so the block is kept in FP32 (in the FP64 block's memory):
    // the same values with half the bytes written and read back.
    int bapply(const double *Rin, double *rz_partials, const int *all_done, bool prepped = false)
    {
        ensure_bops();
        if (opt.precision == AUX_MIXED) {
            ensure_fp32();
            return bapply_B<float>(Rin, (float *)bt.Z, rz_partials, all_done, prepped);
        }
        return bapply_B<double>(Rin, bt.Z, rz_partials, all_done, prepped);
    }
    // P = Z + beta P from the z block of the current precision
    void bdirection(const BCgState &st)
    {
        if (opt.precision == AUX_MIXED) bcg_direction(stream, bt.nr, disc.ndof, (const float *)bt.Z, bt.P, st);
        else bcg_direction(stream, bt.nr, disc.ndof, (const double *)bt.Z, bt.P, st);
    }

    // one lock-step iteration of every column: Q = A P, alpha, X/R update,
    // Z = B R, beta, P update (columns that stopped are left unchanged)
    void bcg_iteration(const BCgState &st)
    {
        hipStream_t s = stream;
        const int nr = bt.nr, n = disc.ndof;
        DevSellView A64 = bview<double>();
        int pk = pbeg(AUX_PROF_CG_SPMV);
        const DevTiles *tl = tiles_for<double>(nr);
        int g = tl ? btile_spmv64(s, nr, tl->view<double>(), bt.P, bt.Q, bt.partials, st.all_done)
                   : bsell_spmv64(s, nr, A64, bt.P, bt.Q, bt.partials, st.all_done);
        pend(pk);
        bfinish(s, nr, bt.partials, g, FIN_PQ, nullptr, st);
        // the update also starts the preconditioner: Z = D^-1 R
        if (opt.precision == AUX_MIXED) {
            ensure_fp32();
            Work<float> &w = bwork<float>();
            g = bcg_update_prep<float>(s, nr, n, bt.X, bt.R, bt.P, bt.Q, st, bt.partials, bo.dinv32, w.za, w.rT);
        } else {
            Work<double> &w = bwork<double>();
            g = bcg_update_prep<double>(s, nr, n, bt.X, bt.R, bt.P, bt.Q, st, bt.partials, bo.dinv64, w.za, nullptr);
        }
        bfinish(s, nr, bt.partials, g, FIN_RR, nullptr, st);
        g = bapply(bt.R, bt.partials, st.all_done, true);
        bfinish(s, nr, bt.partials, g, FIN_RZ, nullptr, st);
        bdirection(st);
    }

    int pcg_batched(const double *Fext, double *Uext, int nrhs, double tol, int maxit, aux_solve_info *infos)
    {
        auto t0 = std::chrono::steady_clock::now();
        if (maxit <= 0) maxit = opt.maxit;
        int nr = 8;
        while (nr < nrhs) nr *= 2;
        if ((uint64_t)disc.ndof * nr * sizeof(double) > (uint64_t(1) << 32))
            throw AuxError(AUX_EINVAL, "block of n_h x " + std::to_string(nr) +
                                           " doubles exceeds 4 GiB; solve fewer right-hand sides per call");
        ensure_batch(nr, maxit);
        hipStream_t s = stream;
        const int n = disc.ndof;
        BCgState st = bstate(maxit);
        const int *all_done = st.all_done;
        DevSellView A64 = bview<double>();
        bgather(s, nr, n, nrhs, bo.perm_d, Fext, bt.F);
        bgather(s, nr, n, nrhs, bo.perm_d, Uext, bt.X);
        if (const DevTiles *tl = tiles_for<double>(nr)) btile_residual64(s, nr, tl->view<double>(), bt.F, bt.X, bt.R);
        else bsell_residual64(s, nr, A64, bt.F, bt.X, bt.R);
        int g = bvec_dot(s, nr, n, bt.F, bt.F, bt.partials);
        bfinish(s, nr, bt.partials, g, FIN_PLAIN, bt.ff, st);
        g = bvec_dot(s, nr, n, bt.R, bt.R, bt.partials);
        bfinish(s, nr, bt.partials, g, FIN_PLAIN, bt.rr0, st);
        bcg_init(s, nr, st, tol * tol, bt.ff, bt.rr0);
        prof_tag = 0;
        g = bapply(bt.R, bt.partials, all_done);
        bfinish(s, nr, bt.partials, g, FIN_RZ, nullptr, st);
        bdirection(st);
        // lock-step iterations, replayed as a HIP graph when not profiling
        hipGraphExec_t gexec = nullptr;
        if (opt.graph && !prof_on) {
            ensure_bops();
            if (opt.precision == AUX_MIXED) {
                ensure_fp32();
                bwork<float>();
            } else {
                bwork<double>();
            }
            const int key[4] = {opt.precision, 0, maxit, nr};
            gexec = captured(g_batch, key, [&]() { bcg_iteration(st); });
        }
        int issued = 0, chunk = 2;
        int *h = bt.host;
        while (true) {
            for (int c = 0; c < chunk && issued < maxit; c++, issued++) {
                prof_tag = issued + 1;
                if (gexec) HIPCHECK(hipGraphLaunch(gexec, s));
                else bcg_iteration(st);
            }
            HIPCHECK(hipMemcpyAsync(h, bt.ist, (2 + 2 * (size_t)nr) * sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHECK(hipStreamSynchronize(s));
            if (h[1] || issued >= maxit) break;
            chunk = 4;
        }
        bscatter(s, nr, n, nrhs, bo.perm_d, bt.X, Uext);
        int last = 0;
        for (int c = 0; c < nrhs; c++) last = std::max(last, h[2 + c]);
        prof_tag = -1;
        prof_collect(last);
        std::vector<double> ff(nr), rr((size_t)bt.hist_cap * nr);
        HIPCHECK(hipMemcpy(ff.data(), bt.ff, nr * sizeof(double), hipMemcpyDeviceToHost));
        HIPCHECK(hipMemcpy(rr.data(), st.rr, rr.size() * sizeof(double), hipMemcpyDeviceToHost));
        int worst = AUX_OK;
        double secs = seconds_since(t0);
        for (int c = 0; c < nrhs; c++) {
            int it = h[2 + c], d = h[2 + nr + c];
            int status = AUX_OK;
            if (d == 2 || d == 0) status = AUX_ENOTCONV;
            else if (d == 3) status = AUX_EBREAKDOWN;
            else if (d == 4) status = AUX_ENAN;
            if (status != AUX_OK && (worst == AUX_OK || status < worst)) worst = status;
            if (infos) {
                infos[c].iterations = it;
                infos[c].status = status;
                double r2 = rr[(size_t)it * nr + c];
                infos[c].rel_residual = ff[c] > 0 ? std::sqrt(r2 / ff[c]) : 0.0;
                infos[c].seconds = secs;
            }
        }
        return worst;
    }

    // ------------------------------------------------------------ block CG
    // O'Leary's block preconditioned CG on the batched block buffers: with
    // gamma = Z^T R and delta = P^T A P, alpha = delta^{-1} gamma,
    // X += P alpha, R -= A P alpha, Z = B R, beta = gamma^{-1} gamma_new,
    // P = Z + P beta.  The nrhs x nrhs Cholesky solves run on the host from
    // one pinned copy of each Gram matrix per step; the padded columns of the
    // block (zero right-hand sides) get zero rows and columns in alpha and
    // beta, so they stay zero.
    struct BlockCg {
        double *gram_part = nullptr, *G = nullptr, *coef = nullptr, *colsum = nullptr;
        double *host = nullptr;        // pinned: gram [nr*nr], coef [nr*nr], colsum [nr]
        int nr = 0;
    } bk;

    void ensure_block(int nr)
    {
        if (bk.nr == nr) return;
        dfree(bk.gram_part);
        dfree(bk.G);
        dfree(bk.coef);
        dfree(bk.colsum);
        bk.gram_part = dnew<double>((size_t)kBlockGramParts * nr * nr);
        bk.G = dnew<double>((size_t)nr * nr);
        bk.coef = dnew<double>((size_t)nr * nr);
        bk.colsum = dnew<double>((size_t)nr);
        if (!bk.host) {
            HIPCHECK(hipHostMalloc((void **)&bk.host, (2 * 64 * 64 + 64) * sizeof(double), hipHostMallocDefault));
            host_bufs.push_back(bk.host);
        }
        bk.nr = nr;
    }

    // Cholesky of the leading s x s block of M (row-major, stride nr) in place
    static bool host_cholesky(int s, int nr, double *M)
    {
        for (int j = 0; j < s; j++) {
            double d = M[j * nr + j];
            for (int p = 0; p < j; p++) d -= M[j * nr + p] * M[j * nr + p];
            if (!(d > 0.0) || !std::isfinite(d)) return false;
            d = std::sqrt(d);
            M[j * nr + j] = d;
            for (int i = j + 1; i < s; i++) {
                double t = M[i * nr + j];
                for (int p = 0; p < j; p++) t -= M[i * nr + p] * M[j * nr + p];
                M[i * nr + j] = t / d;
            }
        }
        return true;
    }
    // C = M^{-1} Y on the leading s x s blocks (L the Cholesky factor of M),
    // every other entry of C zero
    static void host_cholesky_solve(int s, int nr, const double *L, const double *Y, double *C)
    {
        std::fill(C, C + (size_t)nr * nr, 0.0);
        for (int c = 0; c < s; c++) {
            for (int i = 0; i < s; i++) {
                double t = Y[i * nr + c];
                for (int p = 0; p < i; p++) t -= L[i * nr + p] * C[p * nr + c];
                C[i * nr + c] = t / L[i * nr + i];
            }
            for (int i = s - 1; i >= 0; i--) {
                double t = C[i * nr + c];
                for (int p = i + 1; p < s; p++) t -= L[p * nr + i] * C[p * nr + c];
                C[i * nr + c] = t / L[i * nr + i];
            }
        }
    }

    // Gram matrix U^T V of the block (U the z block in its precision or an
    // FP64 block) into host memory
    void block_gram_host(const void *U, bool u_f32, const double *V, double *host_out)
    {
        const int nr = bt.nr, n = disc.ndof;
        if (u_f32) block_gram<float>(stream, nr, n, (const float *)U, V, bk.gram_part, bk.G);
        else block_gram<double>(stream, nr, n, (const double *)U, V, bk.gram_part, bk.G);
        HIPCHECK(hipMemcpyAsync(host_out, bk.G, (size_t)nr * nr * sizeof(double), hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
    }

    // per-column squared norms of an FP64 block into host memory
    void block_colnorms_host(const double *Y, double *host_out)
    {
        const int nr = bt.nr, n = disc.ndof;
        BCgState st = bstate(1);
        int g = bvec_dot(stream, nr, n, Y, Y, bt.partials);
        bfinish(stream, nr, bt.partials, g, FIN_PLAIN, bk.colsum, st);
        HIPCHECK(hipMemcpyAsync(host_out, bk.colsum, nr * sizeof(double), hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
    }

    int block_pcg(const double *Fext, double *Uext, int nrhs, double tol, int maxit, aux_solve_info *infos)
    {
        auto t0 = std::chrono::steady_clock::now();
        if (maxit <= 0) maxit = opt.maxit;
        int nr = 8;
        while (nr < nrhs) nr *= 2;
        if (nr > 64) throw AuxError(AUX_EINVAL, "block CG takes at most 64 right-hand sides");
        if ((uint64_t)disc.ndof * nr * sizeof(double) > (uint64_t(1) << 32))
            throw AuxError(AUX_EINVAL, "block of n_h x " + std::to_string(nr) +
                                           " doubles exceeds 4 GiB; solve fewer right-hand sides per call");
        ensure_batch(nr, 1);
        ensure_block(nr);
        ensure_bops();
        const bool mixed = opt.precision == AUX_MIXED;
        if (mixed) ensure_fp32();
        hipStream_t s = stream;
        const int n = disc.ndof;
        DevSellView A64 = bview<double>();
        const DevTiles *tl = tiles_for<double>(nr);
        bgather(s, nr, n, nrhs, bo.perm_d, Fext, bt.F);
        bgather(s, nr, n, nrhs, bo.perm_d, Uext, bt.X);
        if (tl) btile_residual64(s, nr, tl->view<double>(), bt.F, bt.X, bt.R);
        else bsell_residual64(s, nr, A64, bt.F, bt.X, bt.R);
        double *gam = bk.host, *tmp = bk.host + 64 * 64, *cols = bk.host + 2 * 64 * 64;
        std::vector<double> ff(nr), rr(nr), gcur((size_t)nr * nr), coef((size_t)nr * nr);
        block_colnorms_host(bt.F, cols);
        std::copy(cols, cols + nr, ff.begin());
        block_colnorms_host(bt.R, cols);
        std::copy(cols, cols + nr, rr.begin());
        auto status_of = [&]() {
            bool ok = true;
            for (int c = 0; c < nrhs; c++) {
                if (!std::isfinite(rr[c])) return 3;
                if (ff[c] > 0.0 && !(rr[c] <= tol * tol * ff[c])) ok = false;
            }
            return ok ? 0 : 1;
        };
        int it = 0, status = status_of();
        prof_tag = 0;
        if (status == 1) {
            // Z = B R, gamma = Z^T R, P = Z
            bapply(bt.R, nullptr, nullptr);
            block_gram_host(bt.Z, mixed, bt.R, gam);
            std::copy(gam, gam + (size_t)nr * nr, gcur.begin());
            if (mixed) block_direction<float>(s, nr, n, (const float *)bt.Z, bt.P, nullptr, true);
            else block_direction<double>(s, nr, n, bt.Z, bt.P, nullptr, true);
            while (it < maxit) {
                prof_tag = it + 1;
                // Q = A P; delta = P^T Q; alpha = delta^{-1} gamma
                int pk = pbeg(AUX_PROF_CG_SPMV);
                if (tl) btile_spmv64(s, nr, tl->view<double>(), bt.P, bt.Q, nullptr, nullptr);
                else bsell_spmv64(s, nr, A64, bt.P, bt.Q, nullptr, nullptr);
                pend(pk);
                block_gram_host(bt.P, false, bt.Q, tmp);
                if (!host_cholesky(nrhs, nr, tmp)) {
                    status = 2;
                    break;
                }
                host_cholesky_solve(nrhs, nr, tmp, gcur.data(), coef.data());
                std::copy(coef.begin(), coef.end(), tmp);
                HIPCHECK(hipMemcpyAsync(bk.coef, tmp, (size_t)nr * nr * sizeof(double), hipMemcpyHostToDevice, s));
                // X += P alpha, R -= Q alpha, r.r per column, Z0 = D^-1 R
                int g;
                if (mixed) {
                    Work<float> &w = bwork<float>();
                    g = block_update<float>(s, nr, n, bt.X, bt.R, bt.P, bt.Q, bk.coef, bt.partials, bo.dinv32, w.za,
                                            w.rT);
                } else {
                    Work<double> &w = bwork<double>();
                    g = block_update<double>(s, nr, n, bt.X, bt.R, bt.P, bt.Q, bk.coef, bt.partials, bo.dinv64, w.za,
                                             nullptr);
                }
                BCgState st = bstate(1);
                bfinish(s, nr, bt.partials, g, FIN_PLAIN, bk.colsum, st);
                HIPCHECK(hipMemcpyAsync(cols, bk.colsum, nr * sizeof(double), hipMemcpyDeviceToHost, s));
                HIPCHECK(hipStreamSynchronize(s));
                std::copy(cols, cols + nr, rr.begin());
                it++;
                status = status_of();
                if (status != 1) break;
                // Z = B R (its first sweep came with the update); beta =
                // gamma^{-1} gamma_new; P = Z + P beta
                bapply(bt.R, nullptr, nullptr, true);
                block_gram_host(bt.Z, mixed, bt.R, gam);
                std::copy(gcur.begin(), gcur.end(), tmp);
                if (!host_cholesky(nrhs, nr, tmp)) {
                    status = 2;
                    break;
                }
                host_cholesky_solve(nrhs, nr, tmp, gam, coef.data());
                std::copy(gam, gam + (size_t)nr * nr, gcur.begin());
                std::copy(coef.begin(), coef.end(), tmp);
                HIPCHECK(hipMemcpyAsync(bk.coef, tmp, (size_t)nr * nr * sizeof(double), hipMemcpyHostToDevice, s));
                if (mixed) block_direction<float>(s, nr, n, (const float *)bt.Z, bt.P, bk.coef, false);
                else block_direction<double>(s, nr, n, bt.Z, bt.P, bk.coef, false);
            }
        }
        bscatter(s, nr, n, nrhs, bo.perm_d, bt.X, Uext);
        prof_tag = -1;
        prof_collect(it + 1);
        HIPCHECK(hipStreamSynchronize(s));
        const int code = status == 0 ? AUX_OK : status == 2 ? AUX_EBREAKDOWN : status == 3 ? AUX_ENAN : AUX_ENOTCONV;
        const double secs = seconds_since(t0);
        if (infos)
            for (int c = 0; c < nrhs; c++) {
                infos[c].iterations = it;
                infos[c].status = code;
                infos[c].rel_residual = ff[c] > 0 ? std::sqrt(rr[c] / ff[c]) : 0.0;
                infos[c].seconds = secs;
            }
        return code;
    }

    // ------------------------------------------------------------ new coefficient
    // A new per-tet kappa on the same mesh (aux_set_kappa).  The device
    // assembles A_h into its sliced-ELL slots (FP64 and FP32), its l1 norms,
    // A_H and the matrix-free weights, repeating the host assembly's
    // arithmetic in its order (bitwise equal); the host keeps copies of the
    // values for its own use and builds the AMG hierarchy of the new A_H,
    // then the coefficient-dependent device data are rebuilt.  What depends
    // on the mesh alone (dof numbering, patterns, layouts, I_P, the tet
    // metrics and each entry's list of element-matrix contributions) is kept.
    struct AsmMaps {
        bool ready = false;
        int *a_ptr = nullptr, *a_idx = nullptr, *a_pos = nullptr, *a_rowptr = nullptr, *a_col = nullptr;
        int *h_ptr = nullptr, *h_idx = nullptr;
        int *h_rowptr = nullptr, *h_col = nullptr;   // A_H's pattern
    } asmd;
    // after a coefficient update the host copies of A_h (CSR and sliced-ELL
    // values) and of the composite restriction's values are fetched from
    // the device only when a host-side consumer needs them
    std::vector<int> a_pos_host;     // sliced-ELL slot of each CSR entry of A_h
    bool host_vals_stale = false;
    void ensure_host_values()
    {
        if (!host_vals_stale) return;
        HIPCHECK(hipMemcpyAsync(sell.val.data(), A.v64, sell.val.size() * sizeof(double), hipMemcpyDeviceToHost,
                                stream));
        if (RF.ptr)
            HIPCHECK(hipMemcpyAsync(RF_host.val.data(), RF.v64, RF_host.val.size() * sizeof(double),
                                    hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
        for (size_t e = 0; e < disc.A.val.size(); e++) disc.A.val[e] = sell.val[a_pos_host[e]];
        host_vals_stale = false;
    }

    void ensure_assembly_maps()
    {
        if (asmd.ready) return;
        ensure_adjoint();                          // tet metrics, kappa, reference tables on the device
        const int n = disc.ndof, nt = disc.nt;
        std::vector<int> ptr, idx;
        assembly_map(disc.A, nt, disc.nloc, disc.tet_dof.data(), ptr, idx);
        asmd.a_ptr = upload(ptr);
        asmd.a_idx = upload(idx);
        std::vector<int> pos(disc.A.col.size());
        for (int r = 0; r < n; r++) {
            const int sl = r / kSlice, lane = r % kSlice, i = sell.perm[r];
            for (int e = disc.A.ptr[i], j = 0; e < disc.A.ptr[i + 1]; e++, j++)
                pos[e] = sell.slice_off[sl] + j * kSlice + lane;
        }
        asmd.a_pos = upload(pos);
        a_pos_host = std::move(pos);
        asmd.a_rowptr = upload(disc.A.ptr);
        asmd.a_col = upload(disc.A.col);
        std::vector<int> vmap((size_t)nt * 4);
        for (size_t q = 0; q < vmap.size(); q++) vmap[q] = disc.vert_dof[disc.tets[q]];
        assembly_map(disc.AH, nt, 4, vmap.data(), ptr, idx);
        asmd.h_ptr = upload(ptr);
        asmd.h_idx = upload(idx);
        asmd.h_rowptr = upload(disc.AH.ptr);
        asmd.h_col = upload(disc.AH.col);
        asmd.ready = true;
    }

    void free_op(DevOp &op)
    {
        drop_ell(op);
        for (void *b : {(void *)op.ptr, (void *)op.col, (void *)op.v64, (void *)op.v32}) dfree(b);
        op = DevOp();
    }

    // every device buffer built from the coefficient-dependent operators
    void release_coefficient_part()
    {
        drop_graph();
        dfree(dinv64);
        dfree(dinv32);
        dinv64 = nullptr;
        dinv32 = nullptr;
        for (Lev &L : lev) {
            for (DevOp *op : {&L.A, &L.P, &L.R, &L.down, &L.up}) free_op(*op);
            for (void *b : {(void *)L.dinv64, (void *)L.dinv32, (void *)L.l1, (void *)L.cf}) dfree(b);
        }
        lev.clear();
        host_hier_stale = false;
        if (dev_built_ready) {                     // a build never taken over (an error in between)
            DevMem mem{[this](size_t b) { return dalloc(b); }, [this](void *p) { dfree(p); }};
            free_amg(mem, dev_built);
            dev_built_ready = false;
        }
        for (void *b : {(void *)cinv64, (void *)cinv32, (void *)dcyc64, (void *)dcyc32}) dfree(b);
        cinv64 = dcyc64 = nullptr;
        cinv32 = dcyc32 = nullptr;
        dense_first = SIZE_MAX;
        fused_host.clear();
        dfree(dense_pre);
        dense_pre = nullptr;
        fused_pre = false;
        release_work(w64);
        release_work(w32);
        // batched forms: rebuilt on their next use
        release_batch();
        auto free_bop = [&](BOp &b) {
            free_sell(b.m);
            for (void *q : {(void *)b.perm, (void *)b.s64, (void *)b.s32}) dfree(q);
            b = BOp();
        };
        for (std::vector<BOp> *v : {&bA, &bP, &bR})
            for (BOp &b : *v) free_bop(b);
        bA.clear();
        bP.clear();
        bR.clear();
        for (BOp *b : {&bIP, &bIR, &bRF}) free_bop(*b);
        bops_ready = false;
        for (DevTiles &d : tiles) {
            for (void *q : {(void *)d.rows, (void *)d.row_ptr, (void *)d.col_off, (void *)d.ucols, (void *)d.lidx,
                            (void *)d.v64, (void *)d.v32})
                dfree(q);
            d = DevTiles();
        }
        tiles_ready = false;
        if (opt.batch_order && bo.ready) {
            free_sell(bo.A);
            for (void *q : {(void *)bo.die_off, (void *)bo.perm_d, (void *)bo.dinv64, (void *)bo.dinv32}) dfree(q);
        }
        bo = BOrder();
    }

    void set_kappa(const double *kap)
    {
        const int nt = disc.nt, nl = disc.nloc, n = disc.ndof;
        for (int t = 0; t < nt; t++)
            if (!(kap[t] > 0.0) || !std::isfinite(kap[t])) throw AuxError(AUX_EINVAL, "kappa must be positive and finite");
        ensure_fp32();                             // A_h's FP32 slots are refreshed with the FP64 ones
        ensure_assembly_maps();
        hipStream_t s = stream;
        HIPCHECK(hipMemcpyAsync(kappa_d, kap, (size_t)nt * sizeof(double), hipMemcpyHostToDevice, s));
        const size_t nnzA = disc.A.col.size(), nnzH = disc.AH.col.size();
        double *Ke = dnew<double>((size_t)nt * nl * nl);
        double *aval = dnew<double>(nnzA), *l1e = dnew<double>(n), *hval = dnew<double>(std::max<size_t>(nnzH, 1));
        element_matrices(s, nt, nl, G, kappa_d, Mtab, Ke);
        gather_entries(s, (long long)nnzA, asmd.a_ptr, asmd.a_idx, Ke, nullptr, aval, asmd.a_pos, A.v64, A.v32);
        row_l1(s, n, asmd.a_rowptr, aval, l1e);
        if (nnzH) gather_entries(s, (long long)nnzH, asmd.h_ptr, asmd.h_idx, G, kappa_d, hval, nullptr, nullptr, nullptr);
        if (mf_ready) mf_weights(s, nt, G, kappa_d, mf_w64, mf_w32);
        // the composite restriction's block -I_R A_h, in place (same pattern)
        if (RF.ptr)
            restrict_values(s, RF.n, n, RF.ptr, RF.col, IR.ptr, IR.col, IR.v64, asmd.a_rowptr, asmd.a_col, aval, perm,
                            RF.v64, RF.v32, RF.ell_lanes, RF.ell_off, RF.ell_v64, RF.ell_v32);
        if (RF2.ptr)
            restrict_values(s, RF2.n, n, RF2.ptr, RF2.col, I2Td.ptr, I2Td.col, I2Td.v64, asmd.a_rowptr, asmd.a_col,
                            aval, perm, RF2.v64, RF2.v32, RF2.ell_lanes, RF2.ell_off, RF2.ell_v64, RF2.ell_v32);
        // host copies of the l1 norms and A_H now; those of A_h and of the
        // composite restriction when a host-side consumer needs them
        HIPCHECK(hipMemcpyAsync(disc.l1.data(), l1e, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s));
        if (nnzH) HIPCHECK(hipMemcpyAsync(disc.AH.val.data(), hval, nnzH * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        host_vals_stale = true;
        for (void *b : {(void *)Ke, (void *)aval, (void *)l1e}) dfree(b);
        disc.kappa.assign(kap, kap + nt);
        // the hierarchy of the new A_H and everything built from it
        coef_ready = false;
        release_coefficient_part();
        hier = Hierarchy();
        if (child) child->set_kappa(kap);
        if (disc.nH > 0 && !child) {
            if (opt.amg_setup) {
                DCsr AH;
                AH.n = AH.m = disc.nH;
                AH.nnz = (int)nnzH;
                AH.ptr = asmd.h_rowptr;
                AH.col = asmd.h_col;
                AH.val = hval;
                device_hierarchy(AH, true);
            } else {
                auto t0 = std::chrono::steady_clock::now();
                build_hierarchy(disc.AH, amg_options(), hier);
                amg_seconds = seconds_since(t0);
            }
        }
        dfree(hval);
        upload_coefficient_part(false);
        if (fp32_ready) fp32_coefficient_part();
        work<double>();
        if (opt.precision == AUX_MIXED) work<float>();
        HIPCHECK(hipStreamSynchronize(s));
        coef_ready = true;
    }

    void apply_external(const double *rext, double *zext)
    {
        int n = disc.ndof;
        vec_gather(stream, n, perm, rext, fi);
        apply(fi, z, nullptr, nullptr);
        vec_scatter(stream, n, perm, z, zext);
    }

    void matvec_external(const double *x, double *y)
    {
        int n = disc.ndof;
        vec_gather(stream, n, perm, x, fi);
        sell_spmv64(stream, A.view<double>(), fi, q, nullptr, nullptr);
        vec_scatter(stream, n, perm, q, y);
    }

    void ensure_adjoint()
    {
        if (G) return;
        int nt = disc.nt;
        std::vector<double> g((size_t)nt * 16);
        for (int t = 0; t < nt; t++) {
            const int *v = &disc.tets[4 * (size_t)t];
            double Gt[4][4];
            tet_metric(&disc.xyz[3 * (size_t)v[0]], &disc.xyz[3 * (size_t)v[1]], &disc.xyz[3 * (size_t)v[2]],
                       &disc.xyz[3 * (size_t)v[3]], Gt);
            for (int pq = 0; pq < 16; pq++) g[(size_t)t * 16 + pq] = Gt[pq / 4][pq % 4];
        }
        G = upload(g);
        kappa_d = upload(disc.kappa);
        Mtab = upload(stiffness_tables(disc.k));
        tet_dof_d = upload(disc.tet_dof);
    }

    void release()
    {
        if (child) {
            child->release();
            delete child;
            child = nullptr;
        }
        if (!host_only) {
            if (stream) hipStreamSynchronize(stream);
            else hipDeviceSynchronize();
        }
        drop_graph();
        if (cap_stream) hipStreamDestroy(cap_stream);
        cap_stream = nullptr;
        for (void *ptr : allocs) {
            if (dev.free) dev.free(ptr, dev.ctx);
            else hipFree(ptr);
        }
        allocs.clear();
        alloc_size.clear();
        for (hipEvent_t e : ev_pool) hipEventDestroy(e);
        ev_pool.clear();
        if (host_state) hipHostFree(host_state);
        host_state = nullptr;
        if (host_scal) hipHostFree(host_scal);
        host_scal = nullptr;
        if (fg_host) hipHostFree(fg_host);
        fg_host = nullptr;
        for (void *ptr : host_bufs) hipHostFree(ptr);
        host_bufs.clear();
    }
};

namespace {

template <typename F>
int guarded(F &&f)
{
    try {
        g_error.clear();
        return f();
    } catch (const AuxError &e) {
        g_error = e.what();
        return e.code;
    } catch (const std::invalid_argument &e) {
        g_error = e.what();
        return AUX_EINVAL;
    } catch (const std::bad_alloc &) {
        g_error = "host allocation failed";
        return AUX_ENOMEM;
    } catch (const std::exception &e) {
        g_error = e.what();
        return AUX_EINVAL;
    }
}

// fields a solve fills only when asked for
void init_infos(aux_solve_info *info, int n)
{
    if (info)
        for (int i = 0; i < n; i++) info[i].true_rel_residual = -1.0;
}

// coef: the call needs the coefficient-dependent device data, which a
// coefficient update that failed after releasing them leaves missing
void need_device(const aux_handle *h, bool coef = true)
{
    if (!h) throw AuxError(AUX_EINVAL, "null handle");
    if (h->host_only) throw AuxError(AUX_ESTATE, "handle was set up host-only");
    if (coef && !h->coef_ready)
        throw AuxError(AUX_ESTATE, "the last aux_set_kappa failed: set a coefficient again before solving");
}

void set_dev(const aux_handle *h) { HIPCHECK(hipSetDevice(h->device)); }

}  // namespace

extern "C" {

void aux_default_options(aux_options *o)
{
    if (!o) return;
    o->nu = 2;
    o->theta = 0.8;
    o->coarse_max = 100;
    o->max_levels = 25;
    o->pmis_seed = 0;
    o->precision = AUX_FP64;
    o->maxit = 1000;
    o->host_only = 0;
    o->op = AUX_OP_ASSEMBLED;
    o->sell_window = 0;
    o->graph = 1;
    o->sell_index16 = 1;
    o->fuse_cycle = 1;
    o->batch_tiles = 1;
    o->cycle_lanes = 0;
    o->dense_cycle_rows = 2048;
    o->batch_order = 0;
    o->amg_setup = 1;
    o->aux_space = 1;
    o->smoother_weight = 1.0;
    o->true_residual = 0;
    o->gram_schmidt = 1;
}

int aux_setup(const aux_mesh *mesh, int order, const double *kappa, const aux_options *opt, const aux_device *dev,
              aux_handle **out)
{
    return guarded([&]() {
        if (!mesh || !out) throw AuxError(AUX_EINVAL, "null mesh or output pointer");
        *out = nullptr;
        auto t0 = std::chrono::steady_clock::now();
        aux_options o;
        aux_default_options(&o);
        if (opt) o = *opt;
        if (o.nu < 1 || o.nu > 16) throw AuxError(AUX_EINVAL, "nu must be in [1, 16]");
        if (!(o.theta > 0.0 && o.theta < 1.0)) throw AuxError(AUX_EINVAL, "theta must be in (0, 1)");
        if (o.coarse_max < 1 || o.max_levels < 1 || o.max_levels > 32)
            throw AuxError(AUX_EINVAL, "bad coarse_max or max_levels");
        if (o.precision != AUX_FP64 && o.precision != AUX_MIXED) throw AuxError(AUX_EINVAL, "bad precision");
        if (o.op != AUX_OP_ASSEMBLED && o.op != AUX_OP_MATFREE) throw AuxError(AUX_EINVAL, "bad operator kind");
        if (o.sell_window < 0) throw AuxError(AUX_EINVAL, "sell_window must be >= 0");
        for (int flag : {o.graph, o.sell_index16, o.fuse_cycle, o.host_only, o.batch_order, o.amg_setup,
                         o.true_residual})
            if (flag != 0 && flag != 1) throw AuxError(AUX_EINVAL, "a boolean option is not 0 or 1");
        if (o.batch_tiles < 0 || o.batch_tiles > 2) throw AuxError(AUX_EINVAL, "batch_tiles must be 0, 1 or 2");
        if (o.aux_space != 1 && o.aux_space != 2) throw AuxError(AUX_EINVAL, "aux_space must be 1 or 2");
        if (o.gram_schmidt != 1 && o.gram_schmidt != 2) throw AuxError(AUX_EINVAL, "gram_schmidt must be 1 or 2");
        if (!std::isfinite(o.smoother_weight) || o.smoother_weight == 0.0)
            throw AuxError(AUX_EINVAL, "smoother_weight must be finite and nonzero");
        if (o.dense_cycle_rows < 0 || o.dense_cycle_rows > 8192)
            throw AuxError(AUX_EINVAL, "dense_cycle_rows must be in [0, 8192]");
        {
            const int a = o.cycle_lanes < 0 ? -o.cycle_lanes : o.cycle_lanes;
            if (a != 0 && a != 1 && a != 2 && a != 4 && a != 8 && a != 16 && a != 32)
                throw AuxError(AUX_EINVAL, "cycle_lanes must be 0 or +-1, 2, 4, 8, 16, 32");
        }
        if (o.maxit < 1) o.maxit = 1000;
        auto *h = new aux_handle();
        try {
            h->opt = o;
            h->host_only = o.host_only != 0;
            if (dev) h->dev = *dev;
            h->stream = (hipStream_t)h->dev.stream;
            build_discretization(h->disc, mesh->n_vertices, mesh->xyz, mesh->n_tets, mesh->tets, order, kappa);
            if (h->disc.ndof == 0) throw AuxError(AUX_EINVAL, "mesh has no interior degrees of freedom");
            if (o.aux_space == 2) {
                // the intermediate space: the P^2 problem on the same mesh,
                // with the P^1 auxiliary space and the assembled operator
                if (order < 3) throw AuxError(AUX_EINVAL, "aux_space 2 needs order 3 or 4");
                aux_options co = o;
                co.aux_space = 1;
                co.op = AUX_OP_ASSEMBLED;
                const int rc = aux_setup(mesh, 2, kappa, &co, dev, &h->child);
                if (rc != AUX_OK) throw AuxError(rc, "intermediate P2 space: " + g_error);
                h->I2host = p2_transfer(h->disc, h->child->disc);
            }
            const bool dev_amg = !h->host_only && o.amg_setup == 1 && h->disc.nH > 0 && !h->child;
            if (h->disc.nH > 0 && !dev_amg && !h->child) {
                auto t1 = std::chrono::steady_clock::now();
                build_hierarchy(h->disc.AH, h->amg_options(), h->hier);
                h->amg_seconds = seconds_since(t1);
            }
            if (!h->host_only) {
                HIPCHECK(hipGetDevice(&h->device));
                scratch_address(h->device);
                if (dev_amg) h->device_hierarchy_from_host();
                h->upload_all();
                if (h->child) h->setup_nested();
                if (o.precision == AUX_MIXED) h->ensure_fp32();
                h->work<double>();
                if (o.precision == AUX_MIXED) h->work<float>();
                if (o.op == AUX_OP_MATFREE) h->ensure_mf();
                HIPCHECK(hipDeviceSynchronize());
            }
            h->setup_seconds = seconds_since(t0);
        } catch (...) {
            h->release();
            delete h;
            throw;
        }
        *out = h;
        return AUX_OK;
    });
}

int aux_destroy(aux_handle *h)
{
    if (!h) return AUX_OK;
    return guarded([&]() {
        if (!h->host_only) set_dev(h);
        h->release();
        delete h;
        return AUX_OK;
    });
}

int aux_set_stream(aux_handle *h, void *stream)
{
    return guarded([&]() {
        need_device(h, false);
        h->stream = (hipStream_t)stream;
        if (h->child) h->child->stream = (hipStream_t)stream;
        return AUX_OK;
    });
}

int aux_set_precision(aux_handle *h, int precision)
{
    return guarded([&]() {
        need_device(h);
        if (precision != AUX_FP64 && precision != AUX_MIXED) throw AuxError(AUX_EINVAL, "bad precision");
        set_dev(h);
        h->opt.precision = precision;
        if (h->child) h->child->opt.precision = precision;
        if (precision == AUX_MIXED) {
            h->ensure_fp32();
            h->work<float>();
        }
        return AUX_OK;
    });
}

int aux_set_operator(aux_handle *h, int op)
{
    return guarded([&]() {
        need_device(h);
        if (op != AUX_OP_ASSEMBLED && op != AUX_OP_MATFREE) throw AuxError(AUX_EINVAL, "bad operator kind");
        set_dev(h);
        h->opt.op = op;
        if (op == AUX_OP_MATFREE) h->ensure_mf();
        return AUX_OK;
    });
}

int aux_get_info(const aux_handle *h, aux_info *info)
{
    return guarded([&]() {
        if (!h || !info) throw AuxError(AUX_EINVAL, "null argument");
        std::memset(info, 0, sizeof(*info));
        const Discretization &d = h->disc;
        info->n_h = d.ndof;
        info->n_H = d.nH;
        info->n_tets = d.nt;
        info->nnz_A = d.A.nnz();
        info->nnz_AH = d.AH.nnz();
        info->nnz_IP = d.IP.nnz();
        info->order = d.k;
        // sizes from the device levels when their host copies are not made
        const bool dev = h->host_hier_stale;
        const size_t L = dev ? h->lev.size() : h->hier.levels.size();
        info->levels = (int)L;
        info->ncoarse = dev ? (L ? h->lev[L - 1].A.n : 0) : h->hier.ncoarse;
        info->precision = h->opt.precision;
        double tot = 0.0;
        for (size_t l = 0; l < L && l < 32; l++) {
            const int64_t nnz = dev ? h->lev[l].A.nnz : h->hier.levels[l].A.nnz();
            info->level_rows[l] = dev ? h->lev[l].A.n : h->hier.levels[l].A.n;
            info->level_nnz[l] = nnz;
            info->level_nnz_P[l] = l + 1 < L ? (dev ? h->lev[l].P.nnz : h->hier.levels[l].P.nnz()) : 0;
            tot += (double)nnz;
        }
        info->op_complexity = d.A.nnz() ? (d.A.nnz() + tot) / (double)d.A.nnz() : 0.0;
        info->amg_complexity = d.AH.nnz() ? tot / (double)d.AH.nnz() : 0.0;
        info->setup_seconds = h->setup_seconds;
        info->device_bytes = h->device_bytes;
        info->stored_A = h->A.stored;
        info->sell_window = h->sell_window_used;
        info->sell_slices = h->A.nslices;
        info->sell_narrow_slices = h->A.narrow_slices;
        info->sell_index_bytes = h->A.index_bytes;
        for (int c = 0; c < 4; c++) info->sell_tune_ms[c] = h->tune_ms[c];
        info->nnz_restrict = h->RF_host.nnz();
        info->batch_tile_rows[0] = h->bt.layout32 >= 0 ? h->tiles[h->bt.layout32].tile : 0;
        info->batch_tile_rows[1] = h->bt.layout64 >= 0 ? h->tiles[h->bt.layout64].tile : 0;
        if (dev) {
            for (size_t l = 0; l + 1 < L && l < 32; l++) {
                info->level_nnz_down[l] = h->lev[l].down.nnz;
                info->level_nnz_up[l] = h->lev[l].up.nnz;
            }
        } else {
            for (size_t l = 0; l < h->fused_host.size() && l < 32; l++) {
                info->level_nnz_down[l] = h->fused_host[l].down.nnz();
                info->level_nnz_up[l] = h->fused_host[l].up.nnz();
            }
        }
        info->dense_cycle_level = h->dense_first == SIZE_MAX ? -1 : (int32_t)h->dense_first;
        info->amg_setup_seconds = h->amg_seconds;
        info->aux_space = h->child ? 2 : 1;
        info->sell_split = h->A.split() ? 1 : 0;
        info->lanes_restrict = h->RF.n ? h->RF.lanes_code() : 0;
        info->lanes_prolong = h->IPf.w ? 0 : h->IP.lanes_code();
        for (size_t l = 0; l + 1 < h->lev.size() && l < 32; l++) {
            info->lanes_down[l] = h->lev[l].down.n ? h->lev[l].down.lanes_code() : 0;
            info->lanes_up[l] = h->lev[l].up.n ? h->lev[l].up.lanes_code() : 0;
        }
        return AUX_OK;
    });
}

int aux_dof_keys(const aux_handle *h, int32_t *keys)
{
    return guarded([&]() {
        if (!h || !keys) throw AuxError(AUX_EINVAL, "null argument");
        std::memcpy(keys, h->disc.keys.data(), h->disc.keys.size() * sizeof(int32_t));
        return AUX_OK;
    });
}

int aux_dof_xyz(const aux_handle *h, double *xyz)
{
    return guarded([&]() {
        if (!h || !xyz) throw AuxError(AUX_EINVAL, "null argument");
        const Discretization &d = h->disc;
        for (int i = 0; i < d.ndof; i++)
            for (int c = 0; c < 3; c++) {
                double s = 0.0;
                for (int p = 0; p < d.k; p++) s += d.xyz[3 * (size_t)d.keys[(size_t)i * d.k + p] + c];
                xyz[3 * (size_t)i + c] = s / d.k;
            }
        return AUX_OK;
    });
}

int aux_qpoints_per_tet(const aux_handle *h) { return h ? load_rule_points(h->disc.k) : AUX_EINVAL; }

int aux_qpoints(const aux_handle *h, int32_t t0, int32_t t1, double *xyzq)
{
    return guarded([&]() {
        if (!h || !xyzq || t0 < 0 || t1 > h->disc.nt || t0 > t1) throw AuxError(AUX_EINVAL, "bad tet range");
        quadrature_points(h->disc, t0, t1, xyzq);
        return AUX_OK;
    });
}

int aux_load_accumulate(const aux_handle *h, int32_t t0, int32_t t1, const double *fq, double *b)
{
    return guarded([&]() {
        if (!h || !fq || !b || t0 < 0 || t1 > h->disc.nt || t0 > t1) throw AuxError(AUX_EINVAL, "bad tet range");
        accumulate_load(h->disc, t0, t1, fq, b);
        return AUX_OK;
    });
}

int aux_export_csr(const aux_handle *h, int which, int level, int64_t *shape, int32_t *ptr, int32_t *col, double *val)
{
    return guarded([&]() {
        if (!h || !shape) throw AuxError(AUX_EINVAL, "null argument");
        if ((which == 3 || which == 4 || which == 7 || which == 8) && h->host_hier_stale) {
            set_dev(h);
            const_cast<aux_handle *>(h)->ensure_host_hierarchy();
        }
        const Csr *c = nullptr;
        int nl = (int)h->hier.levels.size();
        switch (which) {
        case 0:
            if (!h->host_only) {
                set_dev(h);
                const_cast<aux_handle *>(h)->ensure_host_values();
            }
            c = &h->disc.A;
            break;
        case 1: c = &h->disc.AH; break;
        case 2: c = &h->disc.IP; break;
        case 3: if (level >= 0 && level < nl) c = &h->hier.levels[level].A; break;
        case 4: if (level >= 0 && level + 1 < nl) c = &h->hier.levels[level].P; break;
        case 5: if (h->sk.host_ready) c = &h->sk.B; break;
        case 6: if (h->sk.host_ready) c = &h->sk.Mp; break;
        case 7:
            if (level >= 0 && level + 1 < nl && (size_t)level < h->fused_host.size()) c = &h->fused_host[level].down;
            break;
        case 8:
            if (level >= 0 && level + 1 < nl && (size_t)level < h->fused_host.size()) c = &h->fused_host[level].up;
            break;
        case 9: if (h->child) c = &h->I2host; break;
        default: break;
        }
        if (!c) throw AuxError(AUX_EINVAL, "no such matrix");
        shape[0] = c->n;
        shape[1] = c->m;
        shape[2] = c->nnz();
        if (ptr) {
            std::memcpy(ptr, c->ptr.data(), c->ptr.size() * sizeof(int32_t));
            std::memcpy(col, c->col.data(), c->col.size() * sizeof(int32_t));
            std::memcpy(val, c->val.data(), c->val.size() * sizeof(double));
        }
        return AUX_OK;
    });
}

int aux_export_cf(const aux_handle *h, int level, int32_t *cf)
{
    return guarded([&]() {
        if (h && h->host_hier_stale) {
            set_dev(h);
            const_cast<aux_handle *>(h)->ensure_host_hierarchy();
        }
        if (!h || !cf || level < 0 || level + 1 >= (int)h->hier.levels.size())
            throw AuxError(AUX_EINVAL, "no splitting on this level");
        const auto &v = h->hier.levels[level].cf;
        std::memcpy(cf, v.data(), v.size() * sizeof(int32_t));
        return AUX_OK;
    });
}

int aux_set_kappa(aux_handle *h, const double *kappa)
{
    return guarded([&]() {
        need_device(h, false);
        if (!kappa) throw AuxError(AUX_EINVAL, "null kappa");
        set_dev(h);
        auto t0 = std::chrono::steady_clock::now();
        h->set_kappa(kappa);
        HIPCHECK(hipGetLastError());
        h->setup_seconds = seconds_since(t0);
        return AUX_OK;
    });
}

int aux_apply(aux_handle *h, const double *r, double *z)
{
    return guarded([&]() {
        need_device(h);
        if (!r || !z) throw AuxError(AUX_EINVAL, "null vector");
        set_dev(h);
        h->apply_external(r, z);
        HIPCHECK(hipGetLastError());
        return AUX_OK;
    });
}

int pcg_solve(aux_handle *h, const double *f, double *u, double tol, int maxit, aux_solve_info *info)
{
    return guarded([&]() {
        need_device(h);
        if (!f || !u) throw AuxError(AUX_EINVAL, "null vector");
        if (!(tol >= 0.0)) throw AuxError(AUX_EINVAL, "tol must be >= 0");
        init_infos(info, 1);
        set_dev(h);
        int st = h->pcg(f, u, tol, maxit, info);
        HIPCHECK(hipGetLastError());
        return st;
    });
}

int pcg_solve_noalloc(aux_handle *h, const double *f, double *u, double tol, int maxit, aux_solve_info *info)
{
    return guarded([&]() {
        need_device(h);
        if (!f || !u) throw AuxError(AUX_EINVAL, "null vector");
        if (!(tol >= 0.0)) throw AuxError(AUX_EINVAL, "tol must be >= 0");
        if (maxit <= 0) maxit = h->opt.maxit;
        if (maxit + 2 > kNoAllocHist)
            throw AuxError(AUX_EINVAL, "maxit exceeds the limit of the allocation-free solve (" +
                                           std::to_string(kNoAllocHist - 2) + ")");
        init_infos(info, 1);
        set_dev(h);
        // everything the solve reads must already exist (built by aux_setup,
        // aux_set_precision and aux_set_operator): nothing is allocated here
        const bool mixed = h->opt.precision == AUX_MIXED;
        if ((mixed && (!h->fp32_ready || !h->w32.ready)) || (!mixed && !h->w64.ready) ||
            (h->use_mf() && !h->mf_ready))
            throw AuxError(AUX_ESTATE, "preconditioner data for the current precision or operator not built");
        double *base = scratch_address(h->device);
        aux_handle::CgBufs cb{base + kScratchPartials, base + kScratchScal, (int *)(base + kScratchState),
                              base + kScratchHist, kNoAllocHist};
        // kernel timing would create events: not recorded by this call
        const bool prof = h->prof_on;
        h->prof_on = false;
        int st;
        try {
            st = h->pcg_run(cb, f, u, tol, maxit, info, false);
        } catch (...) {
            h->prof_on = prof;
            throw;
        }
        h->prof_on = prof;
        HIPCHECK(hipGetLastError());
        return st;
    });
}

int pcg_solve_block(aux_handle *h, const double *F, double *U, int nrhs, double tol, int maxit,
                    aux_solve_info *infos)
{
    return guarded([&]() {
        need_device(h);
        if (!F || !U) throw AuxError(AUX_EINVAL, "null block");
        if (nrhs < 1 || nrhs > 64) throw AuxError(AUX_EINVAL, "nrhs must be in [1, 64]");
        if (!(tol >= 0.0)) throw AuxError(AUX_EINVAL, "tol must be >= 0");
        if (h->child) throw AuxError(AUX_EINVAL, "block solves use the P^1 auxiliary space (aux_space 1)");
        init_infos(infos, nrhs);
        set_dev(h);
        int st = h->block_pcg(F, U, nrhs, tol, maxit, infos);
        HIPCHECK(hipGetLastError());
        return st;
    });
}

int pcg_solve_batched(aux_handle *h, const double *F, double *U, int nrhs, double tol, int maxit,
                      aux_solve_info *infos)
{
    return guarded([&]() -> int {
        need_device(h);
        if (!F || !U) throw AuxError(AUX_EINVAL, "null block");
        if (nrhs < 1 || nrhs > 64) throw AuxError(AUX_EINVAL, "nrhs must be in [1, 64]");
        if (!(tol >= 0.0)) throw AuxError(AUX_EINVAL, "tol must be >= 0");
        if (h->child) throw AuxError(AUX_EINVAL, "batched solves use the P^1 auxiliary space (aux_space 1)");
        init_infos(infos, nrhs);
        set_dev(h);
        int st = h->pcg_batched(F, U, nrhs, tol, maxit, infos);
        HIPCHECK(hipGetLastError());
        return st;
    });
}

int fgmres_solve(aux_handle *h, const double *b, double *x, double tol, int restart, int maxit, double *history,
                 aux_solve_info *info)
{
    return guarded([&]() {
        need_device(h);
        if (!b || !x) throw AuxError(AUX_EINVAL, "null vector");
        if (!(tol >= 0.0)) throw AuxError(AUX_EINVAL, "tol must be >= 0");
        if (restart < 1 || restart > auxp::kMaxRestart) throw AuxError(AUX_EINVAL, "restart must be in [1, 128]");
        init_infos(info, 1);
        set_dev(h);
        int st = h->fgmres(b, x, tol, restart, maxit, history, info);
        HIPCHECK(hipGetLastError());
        return st;
    });
}

int aux_stokes_setup(aux_handle *h, int32_t *n_p)
{
    return guarded([&]() {
        if (!h) throw AuxError(AUX_EINVAL, "null handle");
        if (!h->host_only) set_dev(h);
        h->stokes_setup();
        if (!h->host_only) HIPCHECK(hipGetLastError());
        if (n_p) *n_p = h->sk.np;
        return AUX_OK;
    });
}

int aux_stokes_pressure_keys(const aux_handle *h, int32_t *keys)
{
    return guarded([&]() {
        if (!h || !keys) throw AuxError(AUX_EINVAL, "null argument");
        if (!h->sk.host_ready) throw AuxError(AUX_ESTATE, "call aux_stokes_setup first");
        std::memcpy(keys, h->sk.pkeys.data(), h->sk.pkeys.size() * sizeof(int32_t));
        return AUX_OK;
    });
}

int stokes_apply_operator(aux_handle *h, const double *x, double *y)
{
    return guarded([&]() {
        need_device(h);
        if (!x || !y) throw AuxError(AUX_EINVAL, "null vector");
        set_dev(h);
        h->stokes_operator_external(x, y);
        HIPCHECK(hipGetLastError());
        return AUX_OK;
    });
}

int stokes_apply_qt(aux_handle *h, const double *r, double *z, int32_t *mass_steps)
{
    return guarded([&]() {
        need_device(h);
        if (!r || !z) throw AuxError(AUX_EINVAL, "null vector");
        set_dev(h);
        const int64_t before = h->sk.mass_steps;
        h->stokes_qt_external(r, z);
        HIPCHECK(hipGetLastError());
        if (mass_steps) *mass_steps = (int32_t)(h->sk.mass_steps - before);
        return AUX_OK;
    });
}

int stokes_fgmres_solve(aux_handle *h, const double *b, double *x, double tol, int restart, int maxit,
                        double *history, aux_solve_info *info)
{
    return guarded([&]() {
        need_device(h);
        if (!b || !x) throw AuxError(AUX_EINVAL, "null vector");
        if (!(tol >= 0.0)) throw AuxError(AUX_EINVAL, "tol must be >= 0");
        if (restart < 1 || restart > auxp::kMaxRestart) throw AuxError(AUX_EINVAL, "restart must be in [1, 128]");
        init_infos(info, 1);
        set_dev(h);
        int st = h->stokes_fgmres(b, x, tol, restart, maxit, history, info);
        HIPCHECK(hipGetLastError());
        return st;
    });
}

int aux_matvec(aux_handle *h, const double *x, double *y)
{
    return guarded([&]() {
        need_device(h);
        if (!x || !y) throw AuxError(AUX_EINVAL, "null vector");
        set_dev(h);
        h->matvec_external(x, y);
        HIPCHECK(hipGetLastError());
        return AUX_OK;
    });
}

int aux_kappa_grad(aux_handle *h, const double *u, const double *lam, double *g)
{
    return guarded([&]() {
        need_device(h);
        if (!u || !lam || !g) throw AuxError(AUX_EINVAL, "null vector");
        set_dev(h);
        h->ensure_adjoint();
        kappa_grad(h->stream, h->disc.nt, h->disc.nloc, h->tet_dof_d, h->G, h->kappa_d, h->Mtab, u, lam, g);
        HIPCHECK(hipGetLastError());
        return AUX_OK;
    });
}

int aux_profile(aux_handle *h, int enable)
{
    return guarded([&]() {
        need_device(h, false);
        set_dev(h);
        if (enable < 0 || enable > 2) throw AuxError(AUX_EINVAL, "enable must be 0, 1 or 2");
        h->prof_collect(1 << 30);
        h->prof_on = enable != 0;
        h->prof_apply_only = enable == 2;
        for (int c = 0; c < AUX_PROF_NCAT; c++) {
            h->prof_ms[c] = 0.0;
            h->prof_n[c] = 0;
        }
        return AUX_OK;
    });
}

int aux_profile_read(aux_handle *h, int category, int64_t *launches, double *ms)
{
    return guarded([&]() {
        need_device(h, false);
        if (category < 0 || category >= AUX_PROF_NCAT || !launches || !ms)
            throw AuxError(AUX_EINVAL, "bad profile category");
        set_dev(h);
        h->prof_collect(1 << 30);
        *launches = h->prof_n[category];
        *ms = h->prof_ms[category];
        return AUX_OK;
    });
}

const char *aux_last_error(void) { return g_error.c_str(); }

int aux_residual_history(aux_handle *h, double *hist, int32_t max_len, int32_t *len)
{
    return guarded([&]() {
        need_device(h, false);
        if (!len) throw AuxError(AUX_EINVAL, "null length");
        if (h->last_iters < 0 || !h->last_rr) throw AuxError(AUX_ESTATE, "no single-vector CG solve yet");
        const int n = h->last_iters + 1;
        *len = n;
        if (hist && max_len > 0) {
            const int m = std::min(n, (int)max_len);
            std::vector<double> rr((size_t)m);
            set_dev(h);
            HIPCHECK(hipMemcpyAsync(rr.data(), h->last_rr, (size_t)m * sizeof(double), hipMemcpyDeviceToHost,
                                    h->stream));
            HIPCHECK(hipStreamSynchronize(h->stream));
            for (int k = 0; k < m; k++) hist[k] = h->last_ff > 0 ? std::sqrt(rr[k] / h->last_ff) : 0.0;
        }
        return AUX_OK;
    });
}

}  // extern "C"
