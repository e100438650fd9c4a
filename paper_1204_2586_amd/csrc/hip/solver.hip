// Device side of the solver: upload of the setup data, the preconditioner
// B (Algorithm 2.1 with presmoothing, Remark 2.1) and preconditioned CG,
// behind the C ABI declared in include/aux.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "../host/setup.hpp"
#include "aux.h"
#include "kernels.hpp"

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

struct DevOp {
    int n = 0, m = 0;
    int64_t nnz = 0;
    int *ptr = nullptr, *col = nullptr;
    double *v64 = nullptr;
    float *v32 = nullptr;
    int lpr = 1;
    template <typename T>
    DevCsrView view() const
    {
        return {n, ptr, col, std::is_same<T, float>::value ? (const void *)v32 : (const void *)v64, lpr};
    }
};

template <typename T>
struct Work {
    bool ready = false;
    T *za = nullptr, *zb = nullptr, *res = nullptr, *rT = nullptr;
    std::vector<T *> b, x, r, y;
};

double seconds_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct aux_handle {
    Discretization disc;
    Hierarchy hier;
    aux_options opt{};
    aux_device dev{};
    bool host_only = false;
    int device = 0;
    hipStream_t stream = nullptr;
    double setup_seconds = 0.0;
    int64_t device_bytes = 0;
    std::vector<void *> allocs;

    DevOp A, IP, IR;
    double *dinv64 = nullptr;
    float *dinv32 = nullptr;
    struct Lev {
        DevOp A, P, R;
        double *dinv64 = nullptr;
        float *dinv32 = nullptr;
    };
    std::vector<Lev> lev;
    double *cinv64 = nullptr;
    float *cinv32 = nullptr;
    bool fp32_ready = false;

    Work<double> w64;
    Work<float> w32;

    // CG buffers
    double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
    double *partials = nullptr;
    unsigned int *counter = nullptr;
    double *scal = nullptr;      // [0] f.f, [1] r0.r0, [2] tol2bb
    int *istate = nullptr;       // [0] iter, [1] done
    double *hist = nullptr;      // rz, pq, rr each [hist_cap]
    int hist_cap = 0;
    int *host_state = nullptr;   // pinned: iter, done
    double *host_scal = nullptr; // pinned

    // adjoint data
    double *G = nullptr, *kappa_d = nullptr, *Mtab = nullptr;
    int *tet_dof_d = nullptr;

    // kernel timing with HIP events on the handle's stream
    struct ProfRec {
        hipEvent_t a, b;
        int cat, tag;
    };
    bool prof_on = false;
    int prof_tag = -1;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<ProfRec> prof;
    double prof_ms[AUX_PROF_NCAT] = {};
    int64_t prof_n[AUX_PROF_NCAT] = {};

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
        if (!prof_on) return -1;
        ProfRec r{take_event(), take_event(), cat, prof_tag};
        HIPCHECK(hipEventRecord(r.a, stream));
        prof.push_back(r);
        return (int)prof.size() - 1;
    }
    void pend(int idx)
    {
        if (idx >= 0) HIPCHECK(hipEventRecord(prof[idx].b, stream));
    }
    // fold the recorded events into the per-category sums; launches of CG
    // iteration tags that never ran (enqueued after convergence) are dropped
    void prof_collect(int final_iter)
    {
        if (prof.empty()) return;
        HIPCHECK(hipStreamSynchronize(stream));
        for (const ProfRec &r : prof) {
            bool ran = r.tag < 0 || r.tag == 0 ||
                       (r.cat == AUX_PROF_CG_SPMV ? r.tag <= final_iter : r.tag < final_iter);
            if (!ran) continue;
            float ms = 0.f;
            HIPCHECK(hipEventElapsedTime(&ms, r.a, r.b));
            prof_ms[r.cat] += ms;
            prof_n[r.cat] += 1;
        }
        prof.clear();
        ev_used = 0;
    }

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
        device_bytes += (int64_t)bytes;
        return ptr;
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
    static std::vector<float> to_f32(const std::vector<double> &v)
    {
        return std::vector<float>(v.begin(), v.end());
    }
    static std::vector<double> inverse(const std::vector<double> &v)
    {
        std::vector<double> o(v.size());
        for (size_t i = 0; i < v.size(); i++) o[i] = 1.0 / v[i];
        return o;
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
    void op_fp32(DevOp &d, const Csr &c) { d.v32 = upload(to_f32(c.val)); }

    void upload_all()
    {
        A = upload_op(disc.A);
        dinv64 = upload(inverse(disc.l1));
        IP = upload_op(disc.IP);
        IR = upload_op(disc.IR);
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
        int n = disc.ndof;
        r = dnew<double>(n);
        z = dnew<double>(n);
        p = dnew<double>(n);
        q = dnew<double>(n);
        partials = dnew<double>(kMaxBlocks);
        counter = dnew<unsigned int>(4);
        HIPCHECK(hipMemset(counter, 0, 4 * sizeof(unsigned int)));
        scal = dnew<double>(8);
        istate = dnew<int>(4);
        HIPCHECK(hipHostMalloc((void **)&host_state, 4 * sizeof(int), hipHostMallocDefault));
        HIPCHECK(hipHostMalloc((void **)&host_scal, 8 * sizeof(double), hipHostMallocDefault));
        ensure_hist(std::max(opt.maxit, 16));
    }

    void ensure_hist(int maxit)
    {
        if (maxit + 2 <= hist_cap) return;
        hist_cap = maxit + 2;
        hist = dnew<double>((size_t)3 * hist_cap);
    }

    void ensure_fp32()
    {
        if (fp32_ready) return;
        op_fp32(A, disc.A);
        dinv32 = upload(to_f32(inverse(disc.l1)));
        op_fp32(IP, disc.IP);
        op_fp32(IR, disc.IR);
        for (size_t l = 0; l < hier.levels.size(); l++) {
            const AmgLevel &hl = hier.levels[l];
            op_fp32(lev[l].A, hl.A);
            lev[l].dinv32 = upload(to_f32(inverse(hl.l1)));
            if (l + 1 < hier.levels.size()) {
                op_fp32(lev[l].P, hl.P);
                op_fp32(lev[l].R, hl.R);
            }
        }
        cinv32 = upload(to_f32(hier.coarse_inv));
        fp32_ready = true;
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

    // one V(1,1) cycle from zero on level l; returns the device vector holding the result
    template <typename T>
    const T *vcycle(size_t l, const int *done)
    {
        Work<T> &w = work<T>();
        hipStream_t s = stream;
        const Lev &L = lev[l];
        if (l + 1 == lev.size()) {
            launch_dense_gemv<T>(s, L.A.n, cinv<T>(), w.b[l], w.x[l], done);
            return w.x[l];
        }
        DevCsrView Av = L.A.view<T>();
        launch_vpre<T>(s, Av, ldinv<T>(l), w.b[l], w.x[l], w.r[l], done);
        launch_matvec<T>(s, L.R.view<T>(), w.r[l], w.b[l + 1], done);
        const T *e = vcycle<T>(l + 1, done);
        launch_matvec_add<T>(s, L.P.view<T>(), e, w.x[l], done);
        Reduce none{nullptr, nullptr, nullptr, nullptr};
        launch_sweep<T, T, T>(s, Av, ldinv<T>(l), w.b[l], w.x[l], w.y[l], nullptr, none, done);
        return w.y[l];
    }

    // zout = B r; with red.out, also r.zout into red.out[*red.index]
    template <typename T>
    void apply_B(const double *rin, double *zout, const Reduce &red, const int *done)
    {
        Work<T> &w = work<T>();
        hipStream_t s = stream;
        DevCsrView Av = A.view<T>();
        const T *d = dinv<T>();
        const int nu = opt.nu;
        T *rTbuf = std::is_same<T, float>::value ? w.rT : nullptr;
        T *zc = w.za, *zn = w.zb;
        Reduce none{nullptr, nullptr, nullptr, nullptr};
        // presmoothing: nu l1-Jacobi sweeps from z = 0 (the first two fused)
        int pb = pbeg(AUX_PROF_APPLY);
        int pk = pbeg(AUX_PROF_PK_FIRST);
        if (nu >= 2) launch_first2<T>(s, Av, d, rin, zc, rTbuf, done);
        else launch_jacobi0<T>(s, disc.ndof, d, rin, zc, rTbuf, done);
        pend(pk);
        const T *rT = rTbuf ? (const T *)rTbuf : (const T *)(const void *)rin;
        for (int k = 2; k < nu; k++) {
            pk = pbeg(AUX_PROF_PK_SWEEP);
            launch_sweep<T, T, T>(s, Av, d, rT, zc, zn, nullptr, none, done);
            pend(pk);
            std::swap(zc, zn);
        }
        // Step 1: r_H = I_R (r - A z), one AMG V-cycle; Step 2: z += I_P e_H
        if (!lev.empty()) {
            pk = pbeg(AUX_PROF_PK_RESID);
            launch_resid<T>(s, Av, rT, zc, w.res, done);
            pend(pk);
            pk = pbeg(AUX_PROF_COARSE);
            launch_matvec<T>(s, IR.view<T>(), w.res, w.b[0], done);
            const T *e0 = vcycle<T>(0, done);
            launch_matvec_add<T>(s, IP.view<T>(), e0, zc, done);
            pend(pk);
        }
        // Step 3: nu postsmoothing sweeps; the last one writes the FP64 result
        for (int k = 1; k < nu; k++) {
            pk = pbeg(AUX_PROF_PK_SWEEP);
            launch_sweep<T, T, T>(s, Av, d, rT, zc, zn, nullptr, none, done);
            pend(pk);
            std::swap(zc, zn);
        }
        pk = pbeg(AUX_PROF_PK_LAST);
        launch_sweep<T, double, double>(s, Av, d, rin, zc, zout, rin, red, done);
        pend(pk);
        pend(pb);
    }

    void apply(const double *rin, double *zout, const Reduce &red, const int *done)
    {
        if (opt.precision == AUX_MIXED) {
            ensure_fp32();
            apply_B<float>(rin, zout, red, done);
        } else {
            apply_B<double>(rin, zout, red, done);
        }
    }

    CgState cg_state()
    {
        return {istate, istate + 1, hist, hist + hist_cap, hist + 2 * hist_cap, scal + 2, 0};
    }

    int pcg(const double *f, double *u, double tol, int maxit, aux_solve_info *info)
    {
        auto t0 = std::chrono::steady_clock::now();
        if (maxit <= 0) maxit = opt.maxit;
        ensure_hist(maxit);
        hipStream_t s = stream;
        int n = disc.ndof;
        CgState st = cg_state();
        st.maxit = maxit;
        Reduce rf{partials, counter, scal, nullptr};
        DevCsrView A64 = A.view<double>();
        launch_residual64(s, A64, f, u, r);
        launch_dot64(s, n, f, f, Reduce{partials, counter, scal + 0, nullptr});
        launch_dot64(s, n, r, r, Reduce{partials, counter, scal + 1, nullptr});
        launch_cg_init(s, st, tol * tol, scal + 0, scal + 1);
        Reduce rz{partials, counter, st.rz, st.iter};
        Reduce pq{partials, counter, st.pq, st.iter};
        prof_tag = 0;
        apply(r, z, rz, st.done);
        launch_cg_check_rz(s, st);
        launch_cg_direction(s, n, z, p, st);
        (void)rf;

        int issued = 0, iter = 0, done = 0;
        int chunk = 2;
        std::vector<double> rr_host;
        while (true) {
            for (int c = 0; c < chunk && issued < maxit; c++, issued++) {
                prof_tag = issued + 1;
                int pk = pbeg(AUX_PROF_CG_SPMV);
                launch_spmv64(s, A64, p, q, pq, st.done);
                pend(pk);
                launch_cg_check_pq(s, st);
                launch_cg_update(s, n, u, r, p, q, st, Reduce{partials, counter, nullptr, nullptr});
                apply(r, z, rz, st.done);
                launch_cg_check_rz(s, st);
                launch_cg_direction(s, n, z, p, st);
            }
            HIPCHECK(hipMemcpyAsync(host_state, istate, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHECK(hipStreamSynchronize(s));
            iter = host_state[0];
            done = host_state[1];
            if (done || issued >= maxit) break;
            // predict the remaining iterations from the observed contraction
            std::vector<double> rr(iter + 1);
            HIPCHECK(hipMemcpy(rr.data(), st.rr, (iter + 1) * sizeof(double), hipMemcpyDeviceToHost));
            double target = 0.0;
            HIPCHECK(hipMemcpy(&target, st.tol2bb, sizeof(double), hipMemcpyDeviceToHost));
            chunk = 2;
            if (iter >= 2 && rr[iter] > 0 && rr[iter - 2] > rr[iter] && target > 0) {
                double rate = std::sqrt(rr[iter] / rr[iter - 2]);          // per iteration, squared norm
                double need = std::log(target / rr[iter]) / std::log(rate);
                chunk = (int)std::ceil(std::max(1.0, std::min(need, 16.0)));
            }
        }
        prof_tag = -1;
        prof_collect(iter);
        double rrv = 0.0, ffv = 0.0;
        HIPCHECK(hipMemcpy(&rrv, st.rr + iter, sizeof(double), hipMemcpyDeviceToHost));
        HIPCHECK(hipMemcpy(&ffv, scal + 0, sizeof(double), hipMemcpyDeviceToHost));
        int status = AUX_OK;
        if (done == 2 || (done == 0 && issued >= maxit)) status = AUX_ENOTCONV;
        else if (done == 3) status = AUX_EBREAKDOWN;
        else if (done == 4) status = AUX_ENAN;
        if (info) {
            info->iterations = iter;
            info->status = status;
            info->rel_residual = ffv > 0 ? std::sqrt(rrv / ffv) : 0.0;
            info->seconds = seconds_since(t0);
        }
        return status;
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
        if (!host_only) {
            if (stream) hipStreamSynchronize(stream);
            else hipDeviceSynchronize();
        }
        for (void *ptr : allocs) {
            if (dev.free) dev.free(ptr, dev.ctx);
            else hipFree(ptr);
        }
        allocs.clear();
        for (hipEvent_t e : ev_pool) hipEventDestroy(e);
        ev_pool.clear();
        if (host_state) hipHostFree(host_state);
        if (host_scal) hipHostFree(host_scal);
        host_state = nullptr;
        host_scal = nullptr;
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

void need_device(const aux_handle *h)
{
    if (!h) throw AuxError(AUX_EINVAL, "null handle");
    if (h->host_only) throw AuxError(AUX_ESTATE, "handle was set up host-only");
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
        if (o.maxit < 1) o.maxit = 1000;
        auto *h = new aux_handle();
        try {
            h->opt = o;
            h->host_only = o.host_only != 0;
            if (dev) h->dev = *dev;
            h->stream = (hipStream_t)h->dev.stream;
            build_discretization(h->disc, mesh->n_vertices, mesh->xyz, mesh->n_tets, mesh->tets, order, kappa);
            SetupOptions so;
            so.theta = o.theta;
            so.coarse_max = o.coarse_max;
            so.max_levels = o.max_levels;
            so.seed = o.pmis_seed;
            if (h->disc.nH > 0) build_hierarchy(h->disc.AH, so, h->hier);
            if (!h->host_only) {
                HIPCHECK(hipGetDevice(&h->device));
                h->upload_all();
                if (o.precision == AUX_MIXED) h->ensure_fp32();
                h->work<double>();
                if (o.precision == AUX_MIXED) h->work<float>();
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
        need_device(h);
        h->stream = (hipStream_t)stream;
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
        if (precision == AUX_MIXED) {
            h->ensure_fp32();
            h->work<float>();
        }
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
        info->levels = (int)h->hier.levels.size();
        info->ncoarse = h->hier.ncoarse;
        info->precision = h->opt.precision;
        double tot = 0.0;
        for (size_t l = 0; l < h->hier.levels.size() && l < 32; l++) {
            info->level_rows[l] = h->hier.levels[l].A.n;
            info->level_nnz[l] = h->hier.levels[l].A.nnz();
            tot += (double)h->hier.levels[l].A.nnz();
        }
        info->op_complexity = d.A.nnz() ? (d.A.nnz() + tot) / (double)d.A.nnz() : 0.0;
        info->amg_complexity = d.AH.nnz() ? tot / (double)d.AH.nnz() : 0.0;
        info->setup_seconds = h->setup_seconds;
        info->device_bytes = h->device_bytes;
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
        const Csr *c = nullptr;
        int nl = (int)h->hier.levels.size();
        switch (which) {
        case 0: c = &h->disc.A; break;
        case 1: c = &h->disc.AH; break;
        case 2: c = &h->disc.IP; break;
        case 3: if (level >= 0 && level < nl) c = &h->hier.levels[level].A; break;
        case 4: if (level >= 0 && level + 1 < nl) c = &h->hier.levels[level].P; break;
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
        if (!h || !cf || level < 0 || level + 1 >= (int)h->hier.levels.size())
            throw AuxError(AUX_EINVAL, "no splitting on this level");
        const auto &v = h->hier.levels[level].cf;
        std::memcpy(cf, v.data(), v.size() * sizeof(int32_t));
        return AUX_OK;
    });
}

int aux_apply(aux_handle *h, const double *r, double *z)
{
    return guarded([&]() {
        need_device(h);
        if (!r || !z) throw AuxError(AUX_EINVAL, "null vector");
        set_dev(h);
        h->apply(r, z, Reduce{nullptr, nullptr, nullptr, nullptr}, nullptr);
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
        set_dev(h);
        int st = h->pcg(f, u, tol, maxit, info);
        HIPCHECK(hipGetLastError());
        return st;
    });
}

int pcg_solve_batched(aux_handle *h, const double *F, double *U, int nrhs, double tol, int maxit,
                      aux_solve_info *infos)
{
    return guarded([&]() -> int {
        need_device(h);
        (void)F; (void)U; (void)nrhs; (void)tol; (void)maxit; (void)infos;
        throw AuxError(AUX_ESTATE, "batched solve not built yet");
    });
}

int aux_matvec(aux_handle *h, const double *x, double *y)
{
    return guarded([&]() {
        need_device(h);
        if (!x || !y) throw AuxError(AUX_EINVAL, "null vector");
        set_dev(h);
        launch_spmv64(h->stream, h->A.view<double>(), x, y, Reduce{nullptr, nullptr, nullptr, nullptr}, nullptr);
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
        launch_kappa_grad(h->stream, h->disc.nt, h->disc.nloc, h->tet_dof_d, h->G, h->kappa_d, h->Mtab, u, lam, g);
        HIPCHECK(hipGetLastError());
        return AUX_OK;
    });
}

int aux_profile(aux_handle *h, int enable)
{
    return guarded([&]() {
        need_device(h);
        set_dev(h);
        h->prof_collect(1 << 30);
        h->prof_on = enable != 0;
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
        need_device(h);
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

}  // extern "C"
