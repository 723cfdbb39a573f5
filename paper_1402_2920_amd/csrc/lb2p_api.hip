// lb2p_api.hip -- host side of the C ABI declared in include/lb2p.h.
//
// A context owns two population buffers (A: read by the next step, B: written
// by it), the per-site fields of items 1-11 and a few scalars used by the
// implicit solve's stop rule.  Kernels are instantiated per lattice (D2Q21,
// D3Q59) and storage form (F64, F32, BF16, F16); F64 computes in FP64, the
// others in FP32.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/lb2p.h"
#include "kernels.hpp"

using namespace lb2p;

namespace {

constexpr double kPi = 3.14159265358979323846;

// Positivity windows of the shell weights (Sec. III, App. B), computed at
// create time from the weight polynomials by bisection.
template <int Q>
double min_weight(double s)
{
    double w[8];
    shell_weights<Q, double>(s, w);
    double m = w[0];
    for (int k = 1; k < Lattice<Q>::NSHELL; ++k) m = std::fmin(m, w[k]);
    return m;
}

EosParams make_eos(const lb2p_eos& e)
{
    EosParams p;
    p.rho1 = e.rho1;
    p.rho3 = 2.0 * e.rho2 - e.rho1;
    p.inv_delta_pi = kPi / (e.rho2 - e.rho1);
    p.A = e.A;
    p.cs2_1 = e.cs2_rho1;
    p.a_delta_over_pi = e.A * (e.rho2 - e.rho1) / kPi;
    return p;
}

template <int Q>
lb2p_status check_eos(const lb2p_params& p)
{
    const lb2p_eos& e = p.eos;
    if (!(e.rho2 > e.rho1) || !(e.rho1 > 0.0) || !(e.A >= 0.0) || !(e.cs2_rho1 > 0.0))
        return LB2P_EINVAL;
    const int d = Lattice<Q>::D;
    // weights positive for every c_s^2 the EOS takes: [c1, c1 exp(2 A D/pi)]
    const double lo = e.cs2_rho1, hi = e.cs2_rho1 * std::exp(2.0 * e.A * (e.rho2 - e.rho1) / kPi);
    const int n = 2000;
    for (int k = 0; k <= n; ++k) {
        const double s = lo + (hi - lo) * k / n;
        if (!(min_weight<Q>(s) > 0.0)) return LB2P_EEOS;
    }
    // two-phase region and positive bulk viscosity, sampled on (rho1, rho3)
    const double rho3 = 2.0 * e.rho2 - e.rho1;
    bool two_phase = false;
    for (int k = 1; k < 20000; ++k) {
        const double r = e.rho1 + (rho3 - e.rho1) * k / 20000.0;
        const double psi = e.A * std::sin(kPi * (r - e.rho1) / (e.rho2 - e.rho1));
        if (psi < -1.0 / r) two_phase = true;
        if (!(psi < (2.0 / d) / r)) return LB2P_EEOS;
    }
    if (!two_phase && e.A > 0.0) return LB2P_EEOS;
    return LB2P_OK;
}

}  // namespace

struct lb2p_ctx {
    lb2p_params prm;
    int Q = 0, D = 0;
    Geom g{};
    Coef cf{};
    DevScale ds{};
    hipStream_t stream = nullptr;
    size_t elem = 0;      // bytes per stored population
    size_t rsize = 0;     // bytes per field element
    void* A = nullptr;
    void* B = nullptr;
    void* fields = nullptr;
    void* rho = nullptr; void* j0 = nullptr; void* f = nullptr; void* j0p = nullptr;
    void* u = nullptr; void* jt0 = nullptr; void* jt1 = nullptr; void* q = nullptr;
    void* X = nullptr; void* T = nullptr; void* Y = nullptr; void* Xi = nullptr; void* Sig = nullptr;
    double* partial = nullptr;
    long long nblk = 0;
    void* scratch = nullptr;   // scalars
    int* flags = nullptr;
    unsigned long long* res = nullptr;
    unsigned long long* jscale = nullptr;
    int* done_at = nullptr;
    SolveInfo* info = nullptr;
    double* sums = nullptr;
    void* host = nullptr;      // pinned readback area
    dim3 block, grid;
    bool initialized = false;
    bool have_prev = false;
    bool sigma_valid = false;
    lb2p_status sticky = LB2P_OK;
    int last_iters = 0;
    // optional per-kernel-class event timing (lb2p_profile_*)
    bool prof = false;
    struct Pending { hipEvent_t a, b; int kid; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    double prof_ms[LB2P_NKERNEL] = {0};
    long long prof_n[LB2P_NKERNEL] = {0};
};

namespace {

#define HIPCHK(expr)                                   \
    do {                                               \
        hipError_t _e = (expr);                        \
        if (_e != hipSuccess) return LB2P_EHIP;        \
    } while (0)

void choose_launch(lb2p_ctx* c)
{
    int bx = c->g.nx >= 256 ? 256 : (c->g.nx >= 128 ? 128 : 64);
    int by = 256 / bx;
    c->block = dim3(bx, by, 1);
    c->grid = dim3((c->g.nx + bx - 1) / bx, (c->g.ny + by - 1) / by, c->g.nz);
    c->nblk = (long long)c->grid.x * c->grid.y * c->grid.z;
}

hipEvent_t prof_event(lb2p_ctx* c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Bracket one launch of kernel class `kid` with events on the context stream.
struct ProfScope {
    lb2p_ctx* c;
    int kid;
    hipEvent_t a = nullptr;
    ProfScope(lb2p_ctx* cc, int k) : c(cc), kid(k)
    {
        if (c->prof) {
            a = prof_event(c);
            if (a) (void)hipEventRecord(a, c->stream);
        }
    }
    ~ProfScope()
    {
        if (c->prof && a) {
            hipEvent_t b = prof_event(c);
            if (b) {
                (void)hipEventRecord(b, c->stream);
                c->pending.push_back({a, b, kid});
            }
        }
    }
};

// Resolve recorded events into per-class totals (synchronises the stream).
void prof_collect(lb2p_ctx* c)
{
    if (c->pending.empty()) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto& p : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->prof_ms[p.kid] += ms;
            c->prof_n[p.kid] += 1;
        }
        c->pool.push_back(p.a);
        c->pool.push_back(p.b);
    }
    c->pending.clear();
}

struct HostScratch {
    int done_at;
    int flags;
    SolveInfo info;
    double sums[4];
    double resid;
    double jscale;
};

// ---- typed dispatch -------------------------------------------------------

template <int Q, class R, class S>
struct Impl {
    static void launch_init(lb2p_ctx* c)
    {
        hipLaunchKernelGGL((k_init<Q, R, S>), c->grid, c->block, 0, c->stream, c->g, c->cf, c->ds,
                           (const R*)c->rho, (const R*)c->u, (S*)c->A);
    }

    static void launch_moments(lb2p_ctx* c, bool write_fields)
    {
        {
            ProfScope _ps(c, LB2P_K_MOMENTS);
            hipLaunchKernelGGL((k_moments<Q, R, S>), c->grid, c->block, 0, c->stream, c->g, c->ds,
                               (const S*)c->A, write_fields ? (R*)c->rho : (R*)c->X,
                               write_fields ? (R*)c->j0 : (R*)c->T, c->partial, c->flags);
        }
    }

    // Items 1-8; returns false on a HIP error.  iters/converged in c->host.
    static lb2p_status solve(lb2p_ctx* c)
    {
        const lb2p_params& p = c->prm;
        const int max_it = p.fixed_iter > 0 ? p.fixed_iter : p.max_iter;
        hipLaunchKernelGGL(k_reset_ctl, dim3((max_it + 255) / 256 + 1), dim3(256), 0, c->stream,
                           c->res, max_it, c->jscale, c->done_at);
        launch_moments(c, true);
        const R* prev = nullptr;
        if (p.warm_start && c->have_prev) {
            // previous final iterate, moved into jt0 (same element, same thread)
            HostScratch* hs = (HostScratch*)c->host;
            prev = (const R*)(hs->info.final_buf ? c->jt1 : c->jt0);
        }
        {
            ProfScope _ps(c, LB2P_K_FORCE);
            hipLaunchKernelGGL((k_force<Q, R>), c->grid, c->block, 0, c->stream, c->g, c->cf,
                               (const R*)c->rho, (const R*)c->j0, (R*)c->f, (R*)c->j0p, (R*)c->u,
                               prev, (R*)c->jt0, c->jscale);
        }
        IterCtl ic{c->res, c->jscale, c->done_at, p.fixed_iter > 0 ? -1.0 : p.tol};
        const int every = p.check_every > 0 ? p.check_every : 4;
        HostScratch* hs = (HostScratch*)c->host;
        int launched = 0;
        for (int it = 0; it < max_it; ++it) {
            R* jold = (R*)((it & 1) ? c->jt1 : c->jt0);
            R* jnew = (R*)((it & 1) ? c->jt0 : c->jt1);
            {
                ProfScope _ps(c, LB2P_K_ITER_Q);
                hipLaunchKernelGGL((k_iter_q<Q, R>), c->grid, c->block, 0, c->stream, c->g, c->cf, ic,
                                   it, (const R*)c->rho, (const R*)c->u, (R*)c->q);
            }
            {
                ProfScope _ps(c, LB2P_K_ITER_JT);
                hipLaunchKernelGGL((k_iter_jt<Q, R>), c->grid, c->block, 0, c->stream, c->g, ic, it,
                                   (const R*)c->rho, (const R*)c->q, (const R*)c->j0p,
                                   (const R*)jold, jnew, (R*)c->u);
            }
            launched = it + 1;
            if (p.fixed_iter <= 0 && (launched % every) == 0 && launched < max_it) {
                HIPCHK(hipMemcpyAsync(&hs->done_at, c->done_at, sizeof(int), hipMemcpyDeviceToHost,
                                      c->stream));
                HIPCHK(hipStreamSynchronize(c->stream));
                if (hs->done_at >= 0) break;
            }
        }
        hipLaunchKernelGGL(k_iter_finish, dim3(1), dim3(64), 0, c->stream, ic, launched, c->info);
        HIPCHK(hipGetLastError());
        if (p.fixed_iter <= 0) {
            HIPCHK(hipMemcpyAsync(&hs->info, c->info, sizeof(SolveInfo), hipMemcpyDeviceToHost,
                                  c->stream));
            HIPCHK(hipMemcpyAsync(&hs->flags, c->flags, sizeof(int), hipMemcpyDeviceToHost,
                                  c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            c->last_iters = hs->info.iters;
            if (!hs->info.converged && c->sticky == LB2P_OK) c->sticky = LB2P_ENOCONV;
            if (hs->flags) c->sticky = LB2P_ENONFINITE;
        } else {
            // the final buffer index is known without a readback
            hs->info.final_buf = max_it & 1;
            hs->info.iters = max_it;
            hs->info.converged = 1;
            c->last_iters = max_it;
        }
        c->have_prev = true;
        return LB2P_OK;
    }

    static lb2p_status step(lb2p_ctx* c)
    {
        lb2p_status st = solve(c);
        if (st != LB2P_OK) return st;
        {
            ProfScope _ps(c, LB2P_K_CLOSURE1);
            hipLaunchKernelGGL((k_closure1<Q, R>), c->grid, c->block, 0, c->stream, c->g, c->cf,
                               (const SolveInfo*)c->info, (const R*)c->rho, (const R*)c->u,
                               (const R*)c->jt0, (const R*)c->jt1, (R*)c->X, (R*)c->T, (R*)c->Y,
                               (R*)c->Xi);
        }
        {
            ProfScope _ps(c, LB2P_K_CLOSURE2);
            hipLaunchKernelGGL((k_closure2<Q, R>), c->grid, c->block, 0, c->stream, c->g, c->cf,
                               (const R*)c->rho, (const R*)c->u, (const R*)c->X, (const R*)c->T,
                               (const R*)c->Y, (R*)c->Sig);
        }
        {
            ProfScope _ps(c, LB2P_K_COLLIDE);
            hipLaunchKernelGGL((k_collide<Q, R, S>), c->grid, c->block, 0, c->stream, c->g, c->cf,
                               c->ds, (const SolveInfo*)c->info, (const S*)c->A, (S*)c->B,
                               (const R*)c->rho, (const R*)c->u, (const R*)c->f, (const R*)c->jt0,
                               (const R*)c->jt1, (const R*)c->Sig, (const R*)c->Xi);
        }
        HIPCHK(hipGetLastError());
        std::swap(c->A, c->B);
        c->sigma_valid = true;
        return LB2P_OK;
    }

    static void export_pop(lb2p_ctx* c, double* out)
    {
        hipLaunchKernelGGL((k_export<Q, S>), c->grid, c->block, 0, c->stream, c->g, c->ds,
                           (const S*)c->A, out);
    }
    static void import_pop(lb2p_ctx* c, const double* in)
    {
        hipLaunchKernelGGL((k_import<Q, S>), c->grid, c->block, 0, c->stream, c->g, c->ds, in,
                           (S*)c->A);
    }
};

template <int Q, class F>
auto by_storage(lb2p_ctx* c, F&& fn)
{
    switch (c->prm.storage) {
        case LB2P_STORE_F64: return fn(Impl<Q, double, double>{});
        case LB2P_STORE_F32: return fn(Impl<Q, float, float>{});
        case LB2P_STORE_BF16: return fn(Impl<Q, float, __bf16>{});
        default: return fn(Impl<Q, float, _Float16>{});
    }
}

template <class F>
auto dispatch(lb2p_ctx* c, F&& fn)
{
    if (c->Q == 59) return by_storage<59>(c, fn);
    return by_storage<21>(c, fn);
}

size_t storage_bytes(int storage)
{
    switch (storage) {
        case LB2P_STORE_F64: return 8;
        case LB2P_STORE_F32: return 4;
        default: return 2;
    }
}

// Copy a field [ncomp][N] of type R to a caller buffer of dtype.
lb2p_status copy_out(lb2p_ctx* c, const void* src, int ncomp, void* dst, int dtype, int on_device)
{
    const long long n = (long long)ncomp * c->g.N;
    const bool same = (dtype == LB2P_DTYPE_F64) == (c->rsize == 8);
    const size_t out_elem = dtype == LB2P_DTYPE_F64 ? 8 : 4;
    const void* from = src;
    void* tmp = nullptr;
    if (!same) {
        HIPCHK(hipMallocAsync(&tmp, n * out_elem, c->stream));
        const int tb = 256;
        const long long nb = (n + tb - 1) / tb;
        if (c->rsize == 8)
            hipLaunchKernelGGL((k_convert<double, float>), dim3((unsigned)nb), dim3(tb), 0, c->stream,
                               (const double*)src, (float*)tmp, n);
        else
            hipLaunchKernelGGL((k_convert<float, double>), dim3((unsigned)nb), dim3(tb), 0, c->stream,
                               (const float*)src, (double*)tmp, n);
        from = tmp;
    }
    HIPCHK(hipMemcpyAsync(dst, from, n * out_elem,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    if (tmp) HIPCHK(hipFreeAsync(tmp, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return LB2P_OK;
}

// Copy a caller buffer [ncomp][N] of dtype into a field of type R.
lb2p_status copy_in(lb2p_ctx* c, const void* src, int ncomp, void* dst, int dtype, int on_device)
{
    const long long n = (long long)ncomp * c->g.N;
    const bool same = (dtype == LB2P_DTYPE_F64) == (c->rsize == 8);
    const size_t in_elem = dtype == LB2P_DTYPE_F64 ? 8 : 4;
    if (same) {
        HIPCHK(hipMemcpyAsync(dst, src, n * in_elem,
                              on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        return LB2P_OK;
    }
    void* tmp = nullptr;
    HIPCHK(hipMallocAsync(&tmp, n * in_elem, c->stream));
    HIPCHK(hipMemcpyAsync(tmp, src, n * in_elem,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
    const int tb = 256;
    const long long nb = (n + tb - 1) / tb;
    if (c->rsize == 8)
        hipLaunchKernelGGL((k_convert<float, double>), dim3((unsigned)nb), dim3(tb), 0, c->stream,
                           (const float*)tmp, (double*)dst, n);
    else
        hipLaunchKernelGGL((k_convert<double, float>), dim3((unsigned)nb), dim3(tb), 0, c->stream,
                           (const double*)tmp, (float*)dst, n);
    HIPCHK(hipFreeAsync(tmp, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return LB2P_OK;
}

void free_ctx(lb2p_ctx* c)
{
    if (!c) return;
    if (c->A) (void)hipFree(c->A);
    if (c->B) (void)hipFree(c->B);
    if (c->fields) (void)hipFree(c->fields);
    if (c->partial) (void)hipFree(c->partial);
    if (c->scratch) (void)hipFree(c->scratch);
    if (c->host) (void)hipHostFree(c->host);
    for (auto& p : c->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : c->pool) (void)hipEventDestroy(e);
    delete c;
}

}  // namespace

extern "C" {

const char* lb2p_strerror(lb2p_status st)
{
    switch (st) {
        case LB2P_OK: return "ok";
        case LB2P_EINVAL: return "invalid argument";
        case LB2P_EEOS: return "equation of state not admissible";
        case LB2P_ENOCONV: return "correction-current iteration did not converge";
        case LB2P_ENONFINITE: return "non-finite density";
        case LB2P_ENOMEM: return "out of device memory";
        case LB2P_EHIP: return "HIP runtime error";
        case LB2P_ESTATE: return "call out of order";
    }
    return "unknown status";
}

lb2p_status lb2p_velocities(int lattice, int* c_out, int* q_out)
{
    if (lattice != LB2P_D2Q21 && lattice != LB2P_D3Q59) return LB2P_EINVAL;
    const VelSet& v = lattice == LB2P_D3Q59 ? kD3Q59 : kD2Q21;
    if (q_out) *q_out = v.q;
    if (c_out)
        for (int i = 0; i < v.q; ++i)
            for (int a = 0; a < 3; ++a) c_out[3 * i + a] = v.c[i][a];
    return LB2P_OK;
}

lb2p_status lb2p_default_params(int lattice, int nx, int ny, int nz, int storage, lb2p_params* out)
{
    if (!out) return LB2P_EINVAL;
    lb2p_params p;
    std::memset(&p, 0, sizeof(p));
    p.lattice = lattice;
    p.nx = nx; p.ny = ny; p.nz = nz;
    p.storage = storage;
    p.gamma = 0.0;
    p.kappa = 0.0;
    p.eos.rho1 = 0.3; p.eos.rho2 = 1.0; p.eos.A = 0.0; p.eos.cs2_rho1 = 0.45;
    p.rho0 = 0.3;
    p.tol = storage == LB2P_STORE_F64 ? 1e-13 : 1e-6;
    p.max_iter = 200;
    p.fixed_iter = 0;
    p.warm_start = 1;
    p.check_every = 0;
    p.store_rho_ref = 0.0;
    *out = p;
    return LB2P_OK;
}

lb2p_status lb2p_create(const lb2p_params* params, void* hip_stream, lb2p_ctx** out)
{
    if (!params || !out) return LB2P_EINVAL;
    *out = nullptr;
    const lb2p_params& p = *params;
    if (p.lattice != LB2P_D2Q21 && p.lattice != LB2P_D3Q59) return LB2P_EINVAL;
    if (p.nx < 8 || p.ny < 8) return LB2P_EINVAL;
    if (p.lattice == LB2P_D2Q21 && p.nz != 1) return LB2P_EINVAL;
    if (p.lattice == LB2P_D3Q59 && p.nz < 8) return LB2P_EINVAL;
    if (p.storage < LB2P_STORE_F64 || p.storage > LB2P_STORE_F16) return LB2P_EINVAL;
    if (!(p.gamma > -1.0 && p.gamma < 1.0)) return LB2P_EINVAL;
    if (!(p.kappa >= 0.0) || !(p.tol >= 0.0) || p.max_iter <= 0 || p.fixed_iter < 0)
        return LB2P_EINVAL;
    if (!(p.rho0 > 0.0)) return LB2P_EINVAL;
    if ((long long)p.nx * p.ny * p.nz > (1LL << 31)) return LB2P_EINVAL;
    lb2p_status st = p.lattice == LB2P_D3Q59 ? check_eos<59>(p) : check_eos<21>(p);
    if (st != LB2P_OK) return st;

    lb2p_ctx* c = new (std::nothrow) lb2p_ctx;
    if (!c) return LB2P_ENOMEM;
    c->prm = p;
    c->Q = p.lattice;
    c->D = p.lattice == LB2P_D3Q59 ? 3 : 2;
    c->g.nx = p.nx; c->g.ny = p.ny; c->g.nz = p.nz;
    c->g.N = (long long)p.nx * p.ny * p.nz;
    c->stream = (hipStream_t)hip_stream;
    c->cf.gamma = p.gamma;
    c->cf.kappa = p.kappa;
    c->cf.eos = make_eos(p.eos);
    c->cf.c0sq = eos_cs2<double>(c->cf.eos, p.rho0);
    {
        double w[8] = {0};
        if (c->Q == 59) shell_weights<59, double>(c->cf.c0sq, w);
        else shell_weights<21, double>(c->cf.c0sq, w);
        const int ns = c->Q == 59 ? 8 : 6;
        for (int k = 0; k < ns; ++k) {
            if (!(w[k] > 0.0)) { delete c; return LB2P_EEOS; }
            c->cf.Wk[k] = w[k];
        }
    }
    c->elem = storage_bytes(p.storage);
    c->rsize = p.storage == LB2P_STORE_F64 ? 8 : 4;
    choose_launch(c);

    const long long N = c->g.N;
    const int D = c->D;
    const int nsig = D == 3 ? 6 : 3, nxi = D == 3 ? 10 : 4;
    // rho | j0 | f | j0p | u | jt0 | jt1 | q (alias T) | X | Y | Xi | Sig
    const int ncomp = 1 + 6 * D + nsig + 1 + D + nxi + nsig;
    hipError_t e = hipMalloc(&c->A, (size_t)c->Q * N * c->elem);
    if (e == hipSuccess) e = hipMalloc(&c->B, (size_t)c->Q * N * c->elem);
    if (e == hipSuccess) e = hipMalloc(&c->fields, (size_t)ncomp * N * c->rsize);
    if (e == hipSuccess) e = hipMalloc((void**)&c->partial, (size_t)4 * c->nblk * sizeof(double));
    const int max_it = (p.fixed_iter > 0 ? p.fixed_iter : p.max_iter) + 1;
    const size_t sbytes = 256 + sizeof(unsigned long long) * (size_t)max_it;
    if (e == hipSuccess) e = hipMalloc(&c->scratch, sbytes);
    if (e == hipSuccess) e = hipHostMalloc(&c->host, sizeof(HostScratch), hipHostMallocDefault);
    if (e != hipSuccess) {
        free_ctx(c);
        (void)hipGetLastError();
        return LB2P_ENOMEM;
    }
    char* fb = (char*)c->fields;
    size_t off = 0;
    auto take = [&](int nc) { void* ptr = fb + off * c->rsize; off += (size_t)nc * N; return ptr; };
    c->rho = take(1); c->j0 = take(D); c->f = take(D); c->j0p = take(D); c->u = take(D);
    c->jt0 = take(D); c->jt1 = take(D); c->q = take(nsig); c->T = c->q;
    c->X = take(1); c->Y = take(D); c->Xi = take(nxi); c->Sig = take(nsig);
    char* sb = (char*)c->scratch;
    c->flags = (int*)(sb + 0);
    c->done_at = (int*)(sb + 8);
    c->info = (SolveInfo*)(sb + 16);
    c->jscale = (unsigned long long*)(sb + 32);
    c->sums = (double*)(sb + 64);
    c->res = (unsigned long long*)(sb + 256);
    std::memset(c->host, 0, sizeof(HostScratch));
    if (hipMemsetAsync(c->scratch, 0, sbytes, c->stream) != hipSuccess ||
        hipMemsetAsync(c->fields, 0, (size_t)ncomp * N * c->rsize, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        free_ctx(c);
        return LB2P_EHIP;
    }
    *out = c;
    return LB2P_OK;
}

void lb2p_destroy(lb2p_ctx* ctx)
{
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    free_ctx(ctx);
}

lb2p_status lb2p_init(lb2p_ctx* c, const void* rho, const void* u, int dtype, int on_device)
{
    if (!c || !rho || !u) return LB2P_EINVAL;
    if (dtype != LB2P_DTYPE_F64 && dtype != LB2P_DTYPE_F32) return LB2P_EINVAL;
    lb2p_status st = copy_in(c, rho, 1, c->rho, dtype, on_device);
    if (st != LB2P_OK) return st;
    st = copy_in(c, u, c->D, c->u, dtype, on_device);
    if (st != LB2P_OK) return st;
    // deviation storage reference
    double rref = c->prm.store_rho_ref;
    if (!(rref > 0.0)) {
        // mean density of the initial field (host sum in FP64)
        void* tmp = nullptr;
        HIPCHK(hipMallocAsync(&tmp, (size_t)c->g.N * sizeof(double), c->stream));
        const int tb = 256;
        const long long nb = (c->g.N + tb - 1) / tb;
        if (c->rsize == 8)
            HIPCHK(hipMemcpyAsync(tmp, c->rho, c->g.N * 8, hipMemcpyDeviceToDevice, c->stream));
        else
            hipLaunchKernelGGL((k_convert<float, double>), dim3((unsigned)nb), dim3(tb), 0,
                               c->stream, (const float*)c->rho, (double*)tmp, c->g.N);
        double* hbuf = (double*)std::malloc((size_t)c->g.N * sizeof(double));
        if (!hbuf) { (void)hipFreeAsync(tmp, c->stream); return LB2P_ENOMEM; }
        HIPCHK(hipMemcpyAsync(hbuf, tmp, c->g.N * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipFreeAsync(tmp, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        double acc = 0.0;
        for (long long k = 0; k < c->g.N; ++k) acc += hbuf[k];
        std::free(hbuf);
        rref = acc / (double)c->g.N;
    }
    {
        const double cs2 = eos_cs2<double>(c->cf.eos, rref);
        double w[8] = {0};
        if (c->Q == 59) shell_weights<59, double>(cs2, w);
        else shell_weights<21, double>(cs2, w);
        for (int k = 0; k < 8; ++k) {
            const double wk = w[k] > 0 ? w[k] : 1.0;
            c->ds.off[k] = (float)(wk * rref);
            c->ds.scl[k] = (float)wk;
            c->ds.inv[k] = (float)(1.0 / wk);
        }
    }
    dispatch(c, [&](auto impl) { decltype(impl)::launch_init(c); });
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemsetAsync(c->flags, 0, sizeof(int), c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->initialized = true;
    c->have_prev = false;
    c->sigma_valid = false;
    c->sticky = LB2P_OK;
    return LB2P_OK;
}

lb2p_status lb2p_step(lb2p_ctx* c, int nsteps)
{
    if (!c || nsteps < 0) return LB2P_EINVAL;
    if (!c->initialized) return LB2P_ESTATE;
    for (int s = 0; s < nsteps; ++s) {
        lb2p_status st = dispatch(c, [&](auto impl) { return decltype(impl)::step(c); });
        if (st != LB2P_OK) return st;
    }
    if (c->prm.fixed_iter > 0) HIPCHK(hipGetLastError());
    return c->sticky;
}

lb2p_status lb2p_moments(lb2p_ctx* c, void* rho_out, void* u_out, int dtype, int on_device,
                         lb2p_stats* st)
{
    if (!c) return LB2P_EINVAL;
    if (!c->initialized) return LB2P_ESTATE;
    if (dtype != LB2P_DTYPE_F64 && dtype != LB2P_DTYPE_F32) return LB2P_EINVAL;
    lb2p_status s = dispatch(c, [&](auto impl) { return decltype(impl)::solve(c); });
    if (s != LB2P_OK) return s;
    c->sigma_valid = false;
    if (rho_out) {
        s = copy_out(c, c->rho, 1, rho_out, dtype, on_device);
        if (s != LB2P_OK) return s;
    }
    if (u_out) {
        s = copy_out(c, c->u, c->D, u_out, dtype, on_device);
        if (s != LB2P_OK) return s;
    }
    if (st) {
        s = lb2p_stats_get(c, st);
        if (s != LB2P_OK) return s;
    }
    return c->sticky;
}

lb2p_status lb2p_stats_get(lb2p_ctx* c, lb2p_stats* st)
{
    if (!c || !st) return LB2P_EINVAL;
    if (!c->initialized) return LB2P_ESTATE;
    // totals of the current state (item 1 evaluated into spare field space)
    dispatch(c, [&](auto impl) { decltype(impl)::launch_moments(c, false); });
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, c->stream, c->partial, c->nblk,
                       c->sums);
    HostScratch* hs = (HostScratch*)c->host;
    HIPCHK(hipMemcpyAsync(hs->sums, c->sums, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(&hs->flags, c->flags, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(&hs->info, c->info, sizeof(SolveInfo), hipMemcpyDeviceToHost, c->stream));
    unsigned long long js = 0, rs = 0;
    HIPCHK(hipMemcpyAsync(&js, c->jscale, sizeof(js), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int it = hs->info.iters;
    if (it > 0) {
        HIPCHK(hipMemcpy(&rs, c->res + (it - 1), sizeof(rs), hipMemcpyDeviceToHost));
    }
    st->mass = hs->sums[0];
    st->mom[0] = hs->sums[1];
    st->mom[1] = hs->sums[2];
    st->mom[2] = c->D == 3 ? hs->sums[3] : 0.0;
    st->iters = it;
    double rd, jd;
    std::memcpy(&rd, &rs, sizeof(rd));
    std::memcpy(&jd, &js, sizeof(jd));
    st->resid = rd;
    st->jscale = jd;
    st->nonfinite = hs->flags ? 1 : 0;
    if (hs->flags) c->sticky = LB2P_ENONFINITE;
    return LB2P_OK;
}

lb2p_status lb2p_get_field(lb2p_ctx* c, int field, void* out, int dtype, int on_device)
{
    if (!c || !out) return LB2P_EINVAL;
    if (!c->initialized) return LB2P_ESTATE;
    if (dtype != LB2P_DTYPE_F64 && dtype != LB2P_DTYPE_F32) return LB2P_EINVAL;
    const int D = c->D;
    HostScratch* hs = (HostScratch*)c->host;
    switch (field) {
        case LB2P_FIELD_RHO: return copy_out(c, c->rho, 1, out, dtype, on_device);
        case LB2P_FIELD_J0: return copy_out(c, c->j0, D, out, dtype, on_device);
        case LB2P_FIELD_FORCE: return copy_out(c, c->f, D, out, dtype, on_device);
        case LB2P_FIELD_JTILDE:
            return copy_out(c, hs->info.final_buf ? c->jt1 : c->jt0, D, out, dtype, on_device);
        case LB2P_FIELD_U: return copy_out(c, c->u, D, out, dtype, on_device);
        case LB2P_FIELD_SIGMA:
            if (!c->sigma_valid) return LB2P_ESTATE;
            return copy_out(c, c->Sig, D == 3 ? 6 : 3, out, dtype, on_device);
        case LB2P_FIELD_XI:
            if (!c->sigma_valid) return LB2P_ESTATE;
            return copy_out(c, c->Xi, D == 3 ? 10 : 4, out, dtype, on_device);
        default: return LB2P_EINVAL;
    }
}

lb2p_status lb2p_get_populations(lb2p_ctx* c, double* n_out, int on_device)
{
    if (!c || !n_out) return LB2P_EINVAL;
    if (!c->initialized) return LB2P_ESTATE;
    const size_t bytes = (size_t)c->Q * c->g.N * sizeof(double);
    double* dst = n_out;
    if (!on_device) HIPCHK(hipMallocAsync((void**)&dst, bytes, c->stream));
    dispatch(c, [&](auto impl) { decltype(impl)::export_pop(c, dst); });
    HIPCHK(hipGetLastError());
    if (!on_device) {
        HIPCHK(hipMemcpyAsync(n_out, dst, bytes, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipFreeAsync(dst, c->stream));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return LB2P_OK;
}

lb2p_status lb2p_set_populations(lb2p_ctx* c, const double* n_in, int on_device)
{
    if (!c || !n_in) return LB2P_EINVAL;
    const size_t bytes = (size_t)c->Q * c->g.N * sizeof(double);
    const double* src = n_in;
    double* tmp = nullptr;
    if (!on_device) {
        HIPCHK(hipMallocAsync((void**)&tmp, bytes, c->stream));
        HIPCHK(hipMemcpyAsync(tmp, n_in, bytes, hipMemcpyHostToDevice, c->stream));
        src = tmp;
    }
    if (!c->initialized) {
        // deviation storage needs a reference; use rho1-free default: rho0
        double rref = c->prm.store_rho_ref > 0.0 ? c->prm.store_rho_ref : c->prm.rho0;
        const double cs2 = eos_cs2<double>(c->cf.eos, rref);
        double w[8] = {0};
        if (c->Q == 59) shell_weights<59, double>(cs2, w);
        else shell_weights<21, double>(cs2, w);
        for (int k = 0; k < 8; ++k) {
            const double wk = w[k] > 0 ? w[k] : 1.0;
            c->ds.off[k] = (float)(wk * rref);
            c->ds.scl[k] = (float)wk;
            c->ds.inv[k] = (float)(1.0 / wk);
        }
    }
    dispatch(c, [&](auto impl) { decltype(impl)::import_pop(c, src); });
    HIPCHK(hipGetLastError());
    if (tmp) HIPCHK(hipFreeAsync(tmp, c->stream));
    HIPCHK(hipMemsetAsync(c->flags, 0, sizeof(int), c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->initialized = true;
    c->have_prev = false;
    c->sigma_valid = false;
    c->sticky = LB2P_OK;
    return LB2P_OK;
}

lb2p_status lb2p_profile_enable(lb2p_ctx* c, int on)
{
    if (!c) return LB2P_EINVAL;
    prof_collect(c);
    for (int k = 0; k < LB2P_NKERNEL; ++k) {
        c->prof_ms[k] = 0.0;
        c->prof_n[k] = 0;
    }
    c->prof = on != 0;
    return LB2P_OK;
}

lb2p_status lb2p_profile_read(lb2p_ctx* c, double* ms_out, long long* count_out)
{
    if (!c || !ms_out || !count_out) return LB2P_EINVAL;
    prof_collect(c);
    for (int k = 0; k < LB2P_NKERNEL; ++k) {
        ms_out[k] = c->prof_ms[k];
        count_out[k] = c->prof_n[k];
    }
    return LB2P_OK;
}

}  // extern "C"
