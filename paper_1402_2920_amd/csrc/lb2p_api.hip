// lb2p_api.hip -- host side of the C ABI declared in include/lb2p.h.
//
// A context advances one or more independent periodic lattices ("domains")
// packed into shared buffers: two population buffers (A: read by the next
// step, B: written by it), the per-site fields of items 1-11, a device table
// of per-domain constants and two tile lists (per-site kernels and the fused
// D3Q59 solve pass).  Tiles are dealt to hardware workgroup ids so that each
// of the 8 XCDs receives a contiguous run of tiles (stencil neighbours then
// share that XCD's L2).  Kernels are instantiated per lattice (D2Q21, D3Q59)
// and storage form (F64, F32, BF16, F16); F64 computes in FP64, the others in
// FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/lb2p.h"
#include "kernels.hpp"
#include "kernels_fused.hpp"
#include "kernels_closure.hpp"

using namespace lb2p;

namespace {

constexpr double kPi = 3.14159265358979323846;
// Tile of the fused D3Q59 solve pass: 64 x 8 points for FP32 fields (one
// thread per q point, 68 x 12 threads), 32 x 8 for FP64 fields, whose
// registers would not fit four wavefronts per SIMD in the wider block.
template <class R>
constexpr int fused_tx() { return sizeof(R) == 4 ? 64 : 32; }
constexpr int kFusedTY = 8;
constexpr int kClosTZ = 32;     // longest z chunk of the 3D closure kernels (clos_tz picks it per context)
constexpr int kFused2TX = 32, kFused2TY = 8;    // 2D solve pass: 32-wide strips, 8-row chunks (36 x 8 threads)
constexpr int kClos2TX = 32, kClos2TY = 8;      // 2D closure kernels: LDS tiles (256 threads)
int fused_tx_of(size_t rsize) { return rsize == 4 ? fused_tx<float>() : fused_tx<double>(); }

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

// App. B admissibility: weights positive for every c_s^2 the EOS takes, a
// two-phase region (psi < -1/rho somewhere) and positive bulk viscosity
// (psi < (2/d)/rho everywhere, Sec. VII).
template <int Q>
lb2p_status check_eos(const lb2p_params& p)
{
    const lb2p_eos& e = p.eos;
    if (!(e.rho2 > e.rho1) || !(e.rho1 > 0.0) || !(e.A >= 0.0) || !(e.cs2_rho1 > 0.0))
        return LB2P_EINVAL;
    const int d = Lattice<Q>::D;
    const double lo = e.cs2_rho1, hi = e.cs2_rho1 * std::exp(2.0 * e.A * (e.rho2 - e.rho1) / kPi);
    const int n = 2000;
    for (int k = 0; k <= n; ++k) {
        const double s = lo + (hi - lo) * k / n;
        if (!(min_weight<Q>(s) > 0.0)) return LB2P_EEOS;
    }
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

lb2p_status check_params(const lb2p_params& p)
{
    if (p.lattice != LB2P_D2Q21 && p.lattice != LB2P_D3Q59) return LB2P_EINVAL;
    if (p.nx < 8 || p.ny < 8) return LB2P_EINVAL;
    if (p.lattice == LB2P_D2Q21 && p.nz != 1) return LB2P_EINVAL;
    if (p.lattice == LB2P_D3Q59 && p.nz < 8) return LB2P_EINVAL;
    if (p.storage < LB2P_STORE_F64 || p.storage > LB2P_STORE_F16) return LB2P_EINVAL;
    if (!(p.gamma > -1.0 && p.gamma < 1.0)) return LB2P_EINVAL;
    if (!(p.kappa >= 0.0) || !(p.tol >= 0.0) || p.max_iter <= 0 || p.fixed_iter < 0)
        return LB2P_EINVAL;
    if (p.graph_steps < 0) return LB2P_EINVAL;
    if (p.solver != LB2P_SOLVER_FIXED_POINT && p.solver != LB2P_SOLVER_CHEBYSHEV) return LB2P_EINVAL;
    if (p.warm_start < 0 || p.warm_start > 3) return LB2P_EINVAL;
    if (p.iter_prec != LB2P_ITER_AUTO && p.iter_prec != LB2P_ITER_F32 && p.iter_prec != LB2P_ITER_F64)
        return LB2P_EINVAL;
    if (p.storage == LB2P_STORE_F64 && p.iter_prec == LB2P_ITER_F32) return LB2P_EINVAL;
    if (!(p.spectral_bound >= 0.0 && p.spectral_bound < 1.0)) return LB2P_EINVAL;
    if (!(p.rho0 > 0.0)) return LB2P_EINVAL;
    if ((long long)p.nx * p.ny * p.nz > (1LL << 31)) return LB2P_EINVAL;
    return p.lattice == LB2P_D3Q59 ? check_eos<59>(p) : check_eos<21>(p);
}

// Reduced-storage scales of a domain: W_k at rho_ref, and the cubics P_k
// fitted (least squares, 201 points) to w_k(c_s^2(rho)) rho over [lo, hi].
void set_devscale(DevScale& ds, int Q, const EosParams& eos, double rref, double lo, double hi)
{
    const double cs2 = eos_cs2<double>(eos, rref);
    ds.rref = (float)rref;
    double w[8] = {0};
    if (Q == 59) shell_weights<59, double>(cs2, w);
    else shell_weights<21, double>(cs2, w);
    for (int k = 0; k < 8; ++k) {
        const double wk = w[k] > 0 ? w[k] : 1.0;
        ds.off[k] = (float)(wk * rref);
        ds.scl[k] = (float)wk;
        ds.inv[k] = (float)(1.0 / wk);
        for (int j = 0; j < 4; ++j) ds.pc[k][j] = 0.f;
    }
    const int nshell = Q == 59 ? 8 : 6;
    const double h = std::fmax(std::fmax(rref - lo, hi - rref), 1e-3);   // fit in t = d / h
    for (int k = 1; k < nshell; ++k) {
        double ata[4][5] = {};
        for (int m = 0; m <= 200; ++m) {
            const double t = -1.0 + m / 100.0, r = rref + h * t;
            double wr[8] = {0};
            if (Q == 59) shell_weights<59, double>(eos_cs2<double>(eos, r), wr);
            else shell_weights<21, double>(eos_cs2<double>(eos, r), wr);
            const double f = wr[k] * r;
            const double pw[4] = {1.0, t, t * t, t * t * t};
            for (int a = 0; a < 4; ++a) {
                for (int b = 0; b < 4; ++b) ata[a][b] += pw[a] * pw[b];
                ata[a][4] += pw[a] * f;
            }
        }
        // Gaussian elimination with partial pivoting on the 4x4 normal equations
        for (int col = 0; col < 4; ++col) {
            int piv = col;
            for (int r = col + 1; r < 4; ++r)
                if (std::fabs(ata[r][col]) > std::fabs(ata[piv][col])) piv = r;
            for (int c2 = 0; c2 < 5; ++c2) std::swap(ata[col][c2], ata[piv][c2]);
            for (int r = 0; r < 4; ++r) {
                if (r == col) continue;
                const double fct = ata[r][col] / ata[col][col];
                for (int c2 = col; c2 < 5; ++c2) ata[r][c2] -= fct * ata[col][c2];
            }
        }
        double hj = 1.0;
        for (int j = 0; j < 4; ++j) {
            ds.pc[k][j] = (float)(ata[j][4] / ata[j][j] / hj);
            hj *= h;
        }
    }
}

// c_s^2 and p at the domain's reference density (the per-step planes hold
// deviations from them).
void set_refs(Domain& dm)
{
    const double r = (double)dm.ds.rref;
    dm.cf.cref = eos_cs2<double>(dm.cf.eos, r);
    dm.cf.pref = r * dm.cf.cref;
}

// Upper bound of the spectrum of the j~ map's linear part,
// M = (1/12) Grad^T C Grad diag(1/rho) with C: G -> P1 tr(G) I + p (G + G^T).
// For a plane wave its largest eigenvalue is |s|^2 (2p + P1) / (12 rho) =
// |s|^2 c_s^2 (2 - rho psi) / 12 (longitudinal) or |s|^2 c_s^2 / 12
// (transverse), |s|^2 <= d * max_k s(k)^2 with s(k) the symbol of the
// first-derivative stencil (Sec. IV B); 5% margin for non-uniform rho.
double spectral_bound_from_eos(int D, const EosParams& e, const lb2p_eos& in)
{
    double smax = 0.0;
    for (int k = 0; k <= 4000; ++k) {
        const double t = kPi * k / 4000.0;
        const double sv = (4.0 / 3.0) * std::sin(t) - (1.0 / 6.0) * std::sin(2.0 * t);
        smax = std::fmax(smax, sv * sv);
    }
    double m = 0.0;
    for (int k = 0; k <= 4000; ++k) {
        const double r = e.rho1 + (e.rho3 - e.rho1) * k / 4000.0;
        const double psi = (r > e.rho1 && r < e.rho3) ? in.A * std::sin((r - e.rho1) * e.inv_delta_pi) : 0.0;
        const double cs2 = eos_cs2<double>(e, r);
        m = std::fmax(m, cs2 * std::fmax(2.0 - r * psi, 1.0));
    }
    return 1.05 * D * smax * m / 12.0;
}

// Tile-shape choices remembered per (lattice, storage, domain sizes), shared
// by every context of the process; tune_mutex() guards it (contexts may be
// created and tuned from different threads).
struct TuneChoice {
    int bx, by, tz;
};
std::map<std::string, TuneChoice>& tune_cache()
{
    static std::map<std::string, TuneChoice> m;
    return m;
}
std::mutex& tune_mutex()
{
    static std::mutex mu;
    return mu;
}

// Staging of lb2p_moments_noalloc: a static device array instead of a
// per-call allocation.  Every GPU that runs the library holds its own copy
// (allocated when the code object loads, kept until the process ends).  Its
// name is a host-side stand-in: host code uses only the device address that
// hipGetSymbolAddress returns for the current device, resolved once per
// device by the first lb2p_create there (scratch_address).
constexpr size_t kNoAllocStageBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocStageBytes];

constexpr int kMaxDevices = 64;
std::mutex& scratch_mutex()
{
    static std::mutex mu;
    return mu;
}

// Device address of `scratch` on device dev (the current device).
lb2p_status scratch_address(int dev, void** out)
{
    static void* addr[kMaxDevices] = {};
    if (dev < 0 || dev >= kMaxDevices) return LB2P_EHIP;
    std::lock_guard<std::mutex> lock(scratch_mutex());
    if (!addr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return LB2P_EHIP;
        }
        addr[dev] = ptr;
    }
    *out = addr[dev];
    return LB2P_OK;
}

}  // namespace

struct lb2p_ctx {
    lb2p_params prm;             // shared settings (domain 0's record)
    std::vector<lb2p_params> dprm;
    int Q = 0, D = 0, ndom = 0;
    long long S = 0;             // total sites
    std::vector<Domain> dom;     // host copy of the domain table
    Domain* dtab = nullptr;      // device domain table
    hipStream_t stream = nullptr;
    size_t elem = 0;             // bytes per stored moving population
    size_t pbytes = 0;           // bytes of one population buffer (rest plane + moving planes)
    size_t rsize = 0;            // bytes per field element
    void* A = nullptr;
    void* B = nullptr;
    void* A0 = nullptr;          // buffer that was A at creation (graph parity)
    void* fields = nullptr;
    void* rho = nullptr; void* j0 = nullptr; void* f = nullptr; void* j0p = nullptr;
    void* u = nullptr; void* jt0 = nullptr; void* jt1 = nullptr; void* q = nullptr;
    void* X = nullptr; void* T = nullptr; void* Y = nullptr; void* Xi = nullptr; void* Sig = nullptr;
    void* pf = nullptr;          // p, P1, 1/rho planes (fixed during the j~ solve)
    double* mass = nullptr;      // exact pulled mass per site (item 1, FP64)
    bool any_pull = false;       // some domain has gamma != 0 (collision pulls n_i)
    void* u1 = nullptr;          // second u buffer of the fused solve passes
    double* omega = nullptr;     // Chebyshev weights [ndom][stride], or null
    // tiles
    int bx = 64, by = 4, tz = 32;
    std::vector<Tile> site_host, fused_host;   // launch order
    std::vector<Tile> clos_host;               // closure kernels: 3D z-march chunks, 2D LDS tiles
    Tile* site_tiles = nullptr;
    Tile* fused_tiles = nullptr;
    Tile* clos_tiles = nullptr;
    size_t site_cap = 0, fused_cap = 0, clos_cap = 0;
    double* partial = nullptr;
    size_t partial_cap = 0;
    double* pmax = nullptr;                    // per-block maxima
    size_t pmax_cap = 0;
    int* site_range = nullptr;                 // [ndom+1] tile ranges per domain (domain order)
    int* fused_range = nullptr;
    int* clos_range = nullptr;
    // stop-rule state
    int stride = 0;                            // passes per domain in res
    void* ctl = nullptr;                       // control block (stop rule, flags, sums)
    unsigned long long* res = nullptr;
    unsigned long long* jscale = nullptr;
    int* done_at = nullptr;
    SolveInfo* info = nullptr;
    int* flags = nullptr;
    int* nconv = nullptr;
    int* ndone = nullptr;
    int* go = nullptr;           // 1: the last solve is finished (the kernels after it run)
    double* sums = nullptr;
    struct HostReadback {
        int ndone;       // domains whose stop rule has held
        int ndone_last;  // the largest pass count at which it held
        int nconv;
        int flags;
        double sums[4];
    };
    HostReadback* host = nullptr;               // pinned readback area
    hipEvent_t spec_ev = nullptr;               // marks the arrival of a stop-rule read in pinned host memory
    bool status_pending = false;               // tolerance-mode status not yet read
    bool initialized = false;
    bool solved = false;         // a j~ solve ran since lb2p_init (lb2p_domain_solve)
    bool have_prev = false;      // a time step's j~ exists to start the next solve
    int nprev = 0;               // solves since init whose j~ can start the next one
    // lb2p_moments re-solves the current state into the j~ buffers; the last
    // time step's final j~, which starts the next step's solve, is moved
    // first to the Y field (idle between steps) with its SolveInfo in
    // info_keep, and prev_keep says the next solve reads it from there
    bool prev_keep = false;
    SolveInfo* info_keep = nullptr;
    void* jhist = nullptr;       // final j~ of the steps before the previous one (extrapolated
                                 // warm start: j~(t-2), then j~(t-3) for the quadratic form)
    bool sigma_valid = false;
    lb2p_status sticky = LB2P_OK;
    int last_iters = 0;
    std::vector<SolveInfo> info_host;
    std::vector<unsigned long long> js_host;   // max|j0'| bits per domain (stats readback)
    int device = 0;                            // the HIP device current at create
    void* stage = nullptr;                     // this device's static staging array (device address)
    // graphs of graph_steps fixed-iteration steps, one per buffer parity
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    hipStream_t cap_stream = nullptr;          // capture only (the NULL stream cannot be captured)
    bool capturing = false;
    // optional per-kernel-class event timing (lb2p_profile_*)
    bool prof = false;
    struct Pending { hipEvent_t a, b; int kid; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    unsigned prof_mask = ~0u;    // classes bracketed by events (the others are counted)
    long long prof_passes = 0;   // solve passes that did work while profiling
    double prof_ms[LB2P_NKERNEL] = {0};
    long long prof_n[LB2P_NKERNEL] = {0};
};

namespace {

#define HIPCHK(expr)                                   \
    do {                                               \
        hipError_t _e = (expr);                        \
        if (_e != hipSuccess) return LB2P_EHIP;        \
    } while (0)

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

// Bracket one launch of kernel class `kid` with events on the context stream
// (classes outside prof_mask are only counted: a record without events).
struct ProfScope {
    lb2p_ctx* c;
    int kid;
    bool on = false;
    hipEvent_t a = nullptr;
    ProfScope(lb2p_ctx* cc, int k) : c(cc), kid(k)
    {
        if (c->prof && !c->capturing) {
            on = true;
            if ((c->prof_mask >> k) & 1u) {
                a = prof_event(c);
                if (a) (void)hipEventRecord(a, c->stream);
            }
        }
    }
    ~ProfScope()
    {
        if (!on) return;
        if (a) {
            hipEvent_t b = prof_event(c);
            if (b) {
                (void)hipEventRecord(b, c->stream);
                c->pending.push_back({a, b, kid});
            } else {
                c->pool.push_back(a);
            }
        } else {
            c->pending.push_back({nullptr, nullptr, kid});
        }
    }
};

// Return the events of records [from, end) to the pool and drop the records.
void prof_drop(lb2p_ctx* c, size_t from)
{
    for (size_t k = from; k < c->pending.size(); ++k) {
        if (c->pending[k].a) c->pool.push_back(c->pending[k].a);
        if (c->pending[k].b) c->pool.push_back(c->pending[k].b);
    }
    c->pending.resize(std::min(from, c->pending.size()));
}

// Resolve recorded events into per-class totals (synchronises the stream).
void prof_collect(lb2p_ctx* c)
{
    if (c->pending.empty()) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto& p : c->pending) {
        if (!p.a) {   // counted, not timed
            c->prof_n[p.kid] += 1;
            continue;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->prof_ms[p.kid] += ms;
            c->prof_n[p.kid] += 1;
        }
    }
    prof_drop(c, 0);
}

// Deal a domain-ordered tile list to workgroup ids: id b runs on XCD b % 8,
// so XCD k gets the k-th eighth of the list, in order.  Padding tiles
// (dom = -1) fill the list to a multiple of 8.
std::vector<Tile> deal_xcd(const std::vector<Tile>& in)
{
    const size_t n = (in.size() + 7) / 8 * 8;
    const size_t per = n / 8;
    std::vector<Tile> out(n);
    for (size_t b = 0; b < n; ++b) {
        const size_t src = (b % 8) * per + b / 8;
        if (src < in.size()) {
            out[b] = in[src];
        } else {
            Tile t{};
            t.dom = -1;
            out[b] = t;
        }
    }
    return out;
}

void free_graphs(lb2p_ctx* c)
{
    for (auto& g : c->graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

// (Re)build both tile lists for the current block shapes.
lb2p_status build_tiles(lb2p_ctx* c)
{
    // z chunk of the 3D force and closure kernels: 32 planes, halved (to 8
    // at least) while a launch would have fewer than 1024 blocks, i.e. two
    // rounds of two blocks per CU (a 128^3 grid has 32 tiles per plane:
    // 8-plane chunks take its step from 0.89 to 0.77 ms; at 256^3, 128
    // tiles per plane, 32-plane chunks are the fastest)
    int ctz = kClosTZ;
    if (c->D == 3) {
        auto blocks = [&](int tz) {
            long long n = 0;
            for (const auto& dd : c->dom)
                n += (long long)((dd.g.nx + fused_tx_of(c->rsize) - 1) / fused_tx_of(c->rsize)) *
                     ((dd.g.ny + kFusedTY - 1) / kFusedTY) * ((dd.g.nz + tz - 1) / tz);
            return n;
        };
        while (ctz > 8 && blocks(ctz) < 1024) ctz /= 2;
    }
    std::vector<Tile> site, fused, clos;
    std::vector<int> srange(c->ndom + 1, 0), frange(c->ndom + 1, 0), crange(c->ndom + 1, 0);
    for (int d = 0; d < c->ndom; ++d) {
        srange[d] = (int)site.size();
        frange[d] = (int)fused.size();
        crange[d] = (int)clos.size();
        const Geom& g = c->dom[d].g;
        // A large 3D domain is cut into 8 slabs of rows, each swept through
        // every z: after the XCD deal each XCD owns one slab, so the planes a
        // z-stencil revisits (z +- 2) are a slab's share of a plane and stay
        // in that XCD's L2.  Small domains stay whole (one XCD each).
        // by == 0 selects linear site tiles: 256 consecutive sites each.
        const int by = std::max(c->by, 1);
        const int rows = (g.ny + by - 1) / by;
        const int frows = (g.ny + kFusedTY - 1) / kFusedTY;
        const bool slabs = c->D == 3 && (long long)rows * g.nz * ((g.nx + c->bx - 1) / c->bx) >= 4096;
        const int nslab = slabs ? 8 : 1;
        if (c->by == 0) {
            for (long long i = 0; i < g.N; i += 256) {
                Tile t{};
                t.dom = d; t.x0 = (int)i; t.len = (int)std::min<long long>(256, g.N - i); t.lin = 1;
                site.push_back(t);
            }
        } else {
            for (int sl = 0; sl < nslab; ++sl) {
                const int r0 = (int)((long long)rows * sl / nslab), r1 = (int)((long long)rows * (sl + 1) / nslab);
                for (int z = 0; z < g.nz; ++z)
                    for (int r = r0; r < r1; ++r)
                        for (int x = 0; x < g.nx; x += c->bx) {
                            Tile t{};
                            t.dom = d; t.x0 = x; t.y0 = r * c->by; t.z0 = z; t.len = 1;
                            site.push_back(t);
                        }
            }
        }
        if (c->D == 2) {
            // the 2D fused solve pass: kFused2TX-wide strips over the whole
            // height (each marches along y)
            for (int x = 0; x < g.nx; x += kFused2TX) {
                Tile t{};
                t.dom = d; t.x0 = x; t.y0 = 0; t.z0 = 0; t.len = g.ny;
                fused.push_back(t);
            }
            // the 2D closure kernels: fixed kClos2TX x kClos2TY LDS tiles
            for (int y = 0; y < g.ny; y += kClos2TY)
                for (int x = 0; x < g.nx; x += kClos2TX) {
                    Tile t{};
                    t.dom = d; t.x0 = x; t.y0 = y; t.z0 = 0; t.len = 1;
                    clos.push_back(t);
                }
        } else {
            // the solve pass marches tz planes; the force and closure
            // kernels, which have registers for two blocks per CU, march
            // ctz planes (more blocks in flight)
            for (int pass = 0; pass < 2; ++pass) {
                const int tz = std::min(pass == 0 ? c->tz : ctz, g.nz);
                std::vector<Tile>& lst = pass == 0 ? fused : clos;
                for (int sl = 0; sl < nslab; ++sl) {
                    const int r0 = (int)((long long)frows * sl / nslab),
                              r1 = (int)((long long)frows * (sl + 1) / nslab);
                    for (int z = 0; z < g.nz; z += tz)
                        for (int r = r0; r < r1; ++r)
                            for (int x = 0; x < g.nx; x += fused_tx_of(c->rsize)) {
                                Tile t{};
                                t.dom = d; t.x0 = x; t.y0 = r * kFusedTY; t.z0 = z;
                                t.len = std::min(tz, g.nz - z);
                                lst.push_back(t);
                            }
                }
            }
        }
    }
    srange[c->ndom] = (int)site.size();
    frange[c->ndom] = (int)fused.size();
    crange[c->ndom] = (int)clos.size();
    c->site_host = deal_xcd(site);
    if (c->D == 2 && !fused.empty()) {
        // The 2D solve strips differ in length (their domain's height), by
        // up to 8x in a batch.  Longest first, and neighbours together: the
        // domains, tallest first, are cut into runs of adjacent strips (at
        // most 1/32 of the pass's strip rows each, so a large domain still
        // spreads over the XCDs), and each run goes to the XCD with the
        // fewest strip rows so far.  An XCD then runs its strips in that
        // order, with a strip's x-neighbours (whose columns its stencil
        // reads) on the same XCD and in the same L2.  Each strip keeps its
        // slot in the domain-ordered list for its residual partial; XCDs
        // with fewer strips are padded with empty tiles.
        for (size_t k = 0; k < fused.size(); ++k) fused[k].slot = (int)k;
        long long rows_total = 0;
        for (const Tile& t : fused) rows_total += t.len;
        const long long cap = std::max(1LL, rows_total / 32);
        std::vector<int> order(c->ndom);
        for (int d = 0; d < c->ndom; ++d) order[d] = d;
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return c->dom[a].g.ny > c->dom[b].g.ny; });
        std::vector<std::vector<Tile>> per_xcd(8);
        long long load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int d : order) {
            const int h = std::max(1, c->dom[d].g.ny);
            const int run = (int)std::max(1LL, cap / h);
            for (int t0 = frange[d]; t0 < frange[d + 1]; t0 += run) {
                const int t1 = std::min(frange[d + 1], t0 + run);
                int k = 0;
                for (int q = 1; q < 8; ++q)
                    if (load[q] < load[k]) k = q;
                for (int t = t0; t < t1; ++t) per_xcd[k].push_back(fused[t]);
                load[k] += (long long)(t1 - t0) * h;
            }
        }
        size_t per = 0;
        for (const auto& v : per_xcd) per = std::max(per, v.size());
        std::vector<Tile> pre(8 * per);
        for (auto& t : pre) t.dom = -1;
        for (int k = 0; k < 8; ++k)
            for (size_t i = 0; i < per_xcd[k].size(); ++i) pre[k * per + i] = per_xcd[k][i];
        c->fused_host = deal_xcd(pre);
    } else {
        c->fused_host = fused.empty() ? fused : deal_xcd(fused);
    }
    c->clos_host = clos.empty() ? clos : deal_xcd(clos);
    auto upload = [&](const std::vector<Tile>& h, Tile*& dptr, size_t& cap) -> lb2p_status {
        if (h.empty()) return LB2P_OK;
        if (h.size() > cap) {
            if (dptr) (void)hipFree(dptr);
            dptr = nullptr;
            if (hipMalloc((void**)&dptr, h.size() * sizeof(Tile)) != hipSuccess) return LB2P_ENOMEM;
            cap = h.size();
        }
        HIPCHK(hipMemcpyAsync(dptr, h.data(), h.size() * sizeof(Tile), hipMemcpyHostToDevice, c->stream));
        return LB2P_OK;
    };
    lb2p_status st = upload(c->site_host, c->site_tiles, c->site_cap);
    if (st != LB2P_OK) return st;
    st = upload(c->fused_host, c->fused_tiles, c->fused_cap);
    if (st != LB2P_OK) return st;
    st = upload(c->clos_host, c->clos_tiles, c->clos_cap);
    if (st != LB2P_OK) return st;
    const size_t np = 4 * c->site_host.size();
    if (np > c->partial_cap) {
        if (c->partial) (void)hipFree(c->partial);
        c->partial = nullptr;
        if (hipMalloc((void**)&c->partial, np * sizeof(double)) != hipSuccess) return LB2P_ENOMEM;
        c->partial_cap = np;
    }
    const size_t nm = std::max({c->site_host.size(), c->fused_host.size(), c->clos_host.size()});
    if (nm > c->pmax_cap) {
        if (c->pmax) (void)hipFree(c->pmax);
        c->pmax = nullptr;
        if (hipMalloc((void**)&c->pmax, nm * sizeof(double)) != hipSuccess) return LB2P_ENOMEM;
        c->pmax_cap = nm;
    }
    if (!c->site_range) {
        if (hipMalloc((void**)&c->site_range, (c->ndom + 1) * sizeof(int)) != hipSuccess ||
            hipMalloc((void**)&c->fused_range, (c->ndom + 1) * sizeof(int)) != hipSuccess ||
            hipMalloc((void**)&c->clos_range, (c->ndom + 1) * sizeof(int)) != hipSuccess)
            return LB2P_ENOMEM;
    }
    HIPCHK(hipMemcpyAsync(c->site_range, srange.data(), (c->ndom + 1) * sizeof(int), hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(hipMemcpyAsync(c->fused_range, frange.data(), (c->ndom + 1) * sizeof(int), hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(hipMemcpyAsync(c->clos_range, crange.data(), (c->ndom + 1) * sizeof(int), hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    free_graphs(c);
    return LB2P_OK;
}

// ---- typed dispatch -------------------------------------------------------

template <int Q, class R, class S>
struct Impl {
    static dim3 sgrid(lb2p_ctx* c) { return dim3((unsigned)c->site_host.size()); }
    static dim3 sblock(lb2p_ctx* c) { return c->by == 0 ? dim3(256, 1, 1) : dim3(c->bx, c->by, 1); }

    static void launch_init(lb2p_ctx* c)
    {
        hipLaunchKernelGGL((k_init<Q, R, S>), sgrid(c), sblock(c), 0, c->stream, c->dtab,
                           c->site_tiles, (const double*)c->mass, (const R*)c->u, (S*)c->A);
    }

    static void launch_moments(lb2p_ctx* c, bool write_fields)
    {
        ProfScope _ps(c, LB2P_K_MOMENTS);
        hipLaunchKernelGGL((k_moments<Q, R, S>), sgrid(c), sblock(c), 0, c->stream, c->dtab,
                           c->site_tiles, (const S*)c->A, write_fields ? (R*)c->rho : (R*)c->X,
                           write_fields ? (R*)c->j0 : (R*)c->T, c->partial, c->flags, c->mass,
                           write_fields ? (R*)c->pf : (R*)nullptr);
    }

    static IterCtl iter_ctl(lb2p_ctx* c)
    {
        const lb2p_params& p = c->prm;
        return IterCtl{c->res, c->jscale, c->done_at, c->stride, p.fixed_iter > 0 ? -1.0 : p.tol, c->omega, c->pmax};
    }

    // State of one solve's pass loop: passes launched, the pass count at
    // which the last domain met the stop rule (-1 while unknown), the pass
    // count of the host's next read of the rule, and whether a read is in
    // flight (its copy lands in c->host when c->spec_ev completes).
    struct SolveRun {
        int launched = 0;
        int last_done = -1;
        int next_check = 1;
        bool pending = false;
    };

    // Items 1-8.  In the default (tolerance) mode the host reads how many
    // domains have met the stop rule: first one pass after the previous
    // solve's pass count, then every check_every passes (default 1).  Passes
    // launched after a domain met the rule exit at once (the stop rule is
    // evaluated on the device), so a generous first check costs a few
    // microseconds where an early one costs a host round trip.  The count of
    // domains that hit max_iter and the non-finite flag are read once per
    // lb2p_step / lb2p_moments call (read_status).
    // advance: the solve belongs to a time step (lb2p_step), not to a
    // re-evaluation of the same state (lb2p_moments)
    // form_final: store j~ = rho u - j0' (and u) after a velocity-form
    // solve; a time step leaves that to the first closure kernel
    // (k_closure1_zm, k_closure1_t2), which reads the same words anyway.
    // spec: return at the first read of the stop rule without waiting for
    // it (spec->pending); the caller launches the rest of the step, gated on
    // the device by the rule's outcome, and then finishes the solve.
    static lb2p_status solve(lb2p_ctx* c, bool advance = true, bool form_final = true, SolveRun* spec = nullptr)
    {
        const lb2p_params& p = c->prm;
        const int max_it = p.fixed_iter > 0 ? p.fixed_iter : p.max_iter;
        if (max_it >= c->stride) return LB2P_ESTATE;   // passes index res[] and omega[] below stride
        const long long nres = (long long)c->ndom * c->stride;
        hipLaunchKernelGGL(k_reset_ctl, dim3((unsigned)((std::max<long long>(nres, c->ndom) + 255) / 256)),
                           dim3(256), 0, c->stream, c->res, nres, c->jscale, c->done_at, c->ndom,
                           (int*)nullptr, c->go);
        launch_moments(c, true);
        const IterCtl ic = iter_ctl(c);
        {
            ProfScope _ps(c, LB2P_K_FORCE);
            const SolveInfo* prev =
                (p.warm_start && c->have_prev) ? (c->prev_keep ? c->info_keep : c->info) : nullptr;
            const R* prevA = c->prev_keep ? (const R*)c->Y : (const R*)c->jt0;
            const R* prevB = c->prev_keep ? (const R*)c->Y : (const R*)c->jt1;
            // warm_start 2/3: keep the history only for solves that advance
            // time; extrapolate linearly once two previous steps exist and
            // quadratically (warm_start 3) once three do
            R* hist = (p.warm_start >= 2 && advance && prev) ? (R*)c->jhist : nullptr;
            R* hist2 = (hist && p.warm_start == 3) ? (R*)c->jhist + (size_t)c->D * c->S : nullptr;
            const int order = !hist ? 0 : std::min(c->nprev, p.warm_start) - 1;
            // the fused (velocity-form) solve starts from u alone and forms
            // j~ after its last pass, so x_0 is not stored for it
            const bool fused_solve = !(p.flags & LB2P_FLAG_UNFUSED_SOLVE);
            R* const jstart = fused_solve ? (R*)nullptr : (R*)c->jt0;
            if constexpr (Lattice<Q>::D == 3) {
                constexpr int TX = fused_tx<R>();
                hipLaunchKernelGGL((k_force_zm<R, TX, kFusedTY>), dim3((unsigned)c->clos_host.size()),
                                   dim3(TX, kFusedTY, 1), 0, c->stream, c->dtab, c->clos_tiles, ic,
                                   (const double*)c->mass, (const R*)c->j0, (R*)c->f, (R*)c->j0p, (R*)c->u,
                                   prevA, prevB, prev, jstart, hist, hist2, order);
            } else {
                hipLaunchKernelGGL((k_force_t2<R, kClos2TX, kClos2TY>), dim3((unsigned)c->clos_host.size()),
                                   dim3(kClos2TX, kClos2TY, 1), 0, c->stream, c->dtab, c->clos_tiles, ic,
                                   (const double*)c->mass, (const R*)c->j0, (R*)c->f, (R*)c->j0p, (R*)c->u,
                                   prevA, prevB, prev, jstart, hist, hist2, order);
            }
            hipLaunchKernelGGL(k_reduce_max, dim3(c->ndom), dim3(256), 0, c->stream, (const double*)c->pmax,
                               (const int*)c->clos_range, c->jscale, 1LL, (const int*)nullptr);
        }
        SolveRun run;
        run.next_check = std::max(1, c->last_iters + 1);
        lb2p_status st = iterate(c, run, spec != nullptr);
        if (st != LB2P_OK) return st;
        if (run.pending) {
            *spec = run;
            return LB2P_OK;
        }
        st = launch_finish(c, run, form_final, false);
        if (st != LB2P_OK) return st;
        book(c, run, advance);
        return LB2P_OK;
    }

    // Passes run.launched, run.launched + 1, ... until the stop rule holds
    // in every domain (read by the host at run.next_check, then every
    // check_every passes) or max_iter.  speculate: at the first read, record
    // c->spec_ev after the copy and return with run.pending set.
    static lb2p_status iterate(lb2p_ctx* c, SolveRun& run, bool speculate)
    {
        const lb2p_params& p = c->prm;
        const int max_it = p.fixed_iter > 0 ? p.fixed_iter : p.max_iter;
        const IterCtl ic = iter_ctl(c);
        const bool fused = !(p.flags & LB2P_FLAG_UNFUSED_SOLVE);
        constexpr int kFusedTX = Lattice<Q>::D == 3 ? fused_tx<R>() : kFused2TX;
        constexpr int kTY = Lattice<Q>::D == 3 ? kFusedTY : kFused2TY;
        // 3D: one thread per q point of a (TX+4) x (TY+4) plane tile; 2D: one
        // per q point of a (TX+4)-wide strip row, kFused2TY rows per chunk
        const dim3 fblock(kFusedTX + 4, Lattice<Q>::D == 3 ? kTY + 4 : kTY, 1);
        const dim3 fgrid((unsigned)c->fused_host.size());
        const int every = p.check_every > 0 ? p.check_every : 1;
        for (int it = run.launched; it < max_it; ++it) {
            R* jold = (R*)((it & 1) ? c->jt1 : c->jt0);
            R* jnew = (R*)((it & 1) ? c->jt0 : c->jt1);
            R* uold = (R*)((it & 1) ? c->u1 : c->u);
            R* unew = (R*)((it & 1) ? c->u : c->u1);
            if (fused) {
                if constexpr (Lattice<Q>::D == 2) {
                    ProfScope _ps(c, LB2P_K_ITER_FUSED);
                    if (c->omega)
                        hipLaunchKernelGGL((k_iter_fused2<R, kFusedTX, kTY, true>), fgrid, fblock, 0,
                                           c->stream, c->dtab, c->fused_tiles, ic, it, (const R*)c->pf,
                                           (const R*)c->rho, (const R*)c->j0p, (const R*)uold, unew);
                    else
                        hipLaunchKernelGGL((k_iter_fused2<R, kFusedTX, kTY, false>), fgrid, fblock, 0,
                                           c->stream, c->dtab, c->fused_tiles, ic, it, (const R*)c->pf,
                                           (const R*)c->rho, (const R*)c->j0p, (const R*)uold, unew);
                } else {
                    ProfScope _ps(c, LB2P_K_ITER_FUSED);
                    if (c->omega)
                        hipLaunchKernelGGL((k_iter_fused3<R, kFusedTX, kFusedTY, true>), fgrid, fblock, 0,
                                           c->stream, c->dtab, c->fused_tiles, ic, it, (const R*)c->pf,
                                           (const R*)c->rho, (const R*)c->j0p, (const R*)uold, unew);
                    else
                        hipLaunchKernelGGL((k_iter_fused3<R, kFusedTX, kFusedTY, false>), fgrid, fblock, 0,
                                           c->stream, c->dtab, c->fused_tiles, ic, it, (const R*)c->pf,
                                           (const R*)c->rho, (const R*)c->j0p, (const R*)uold, unew);
                }
            } else {
                {
                    ProfScope _ps(c, LB2P_K_ITER_Q);
                    hipLaunchKernelGGL((k_iter_q<Q, R>), sgrid(c), sblock(c), 0, c->stream, c->dtab,
                                       c->site_tiles, ic, it, (const R*)c->pf, (const R*)c->u,
                                       (R*)c->q);
                }
                {
                    ProfScope _ps(c, LB2P_K_ITER_JT);
                    hipLaunchKernelGGL((k_iter_jt<Q, R>), sgrid(c), sblock(c), 0, c->stream, c->dtab,
                                       c->site_tiles, ic, it, (const R*)c->pf, (const R*)c->q,
                                       (const R*)c->j0p, (const R*)jold, jnew, (R*)c->u);
                }
            }
            // the pass's residual per domain: read by the next pass's stop
            // rule (tolerance mode); with a fixed pass count only the last
            // one is read (lb2p_domain_solve, lb2p_stats_get)
            if (p.fixed_iter <= 0 || it == max_it - 1)
                hipLaunchKernelGGL(k_reduce_max, dim3(c->ndom), dim3(256), 0, c->stream, (const double*)c->pmax,
                                   (const int*)(fused ? c->fused_range : c->site_range), c->res + it,
                                   (long long)c->stride, (const int*)c->done_at);
            run.launched = it + 1;
            if (p.fixed_iter <= 0 && run.launched >= run.next_check && run.launched < max_it) {
                run.next_check = run.launched + every;
                hipLaunchKernelGGL(k_check_done, dim3(1), dim3(256), 0, c->stream, ic, run.launched, c->ndom,
                                   c->ndone, c->go);
                HIPCHK(hipMemcpyAsync(&c->host->ndone, c->ndone, 2 * sizeof(int), hipMemcpyDeviceToHost,
                                      c->stream));
                if (speculate) {
                    HIPCHK(hipEventRecord(c->spec_ev, c->stream));
                    run.pending = true;
                    return LB2P_OK;
                }
                HIPCHK(hipStreamSynchronize(c->stream));
                if (c->host->ndone >= c->ndom) {
                    run.last_done = c->host->ndone_last;
                    break;
                }
            }
        }
        return LB2P_OK;
    }

    // The solve's final record (SolveInfo per domain; the count of domains
    // that reached max_iter) and, unless a time step leaves it to the first
    // closure kernel, the final j~ and u.  gated: launched before the
    // host's read of the stop rule (k_iter_finish then does nothing unless
    // the rule held in every domain); ungated it also sets go = 1.
    static lb2p_status launch_finish(lb2p_ctx* c, const SolveRun& run, bool form_final, bool gated)
    {
        const IterCtl ic = iter_ctl(c);
        const bool fused = !(c->prm.flags & LB2P_FLAG_UNFUSED_SOLVE);
        hipLaunchKernelGGL(k_iter_finish, dim3((c->ndom + 255) / 256), dim3(256), 0, c->stream, ic,
                           run.launched, c->ndom, c->info, c->nconv, c->go, gated ? 1 : 0);
        if (fused && form_final)
            hipLaunchKernelGGL((k_jt_final<Q, R>), sgrid(c), sblock(c), 0, c->stream, c->dtab,
                               c->site_tiles, (const SolveInfo*)c->info, (const R*)c->rho,
                               (const R*)c->j0p, (R*)c->u, (const R*)c->u1, (R*)c->jt0, (R*)c->jt1);
        else if (!fused)
            hipLaunchKernelGGL((k_u_final<Q, R>), sgrid(c), sblock(c), 0, c->stream, c->dtab,
                               c->site_tiles, (const SolveInfo*)c->info, (const R*)c->rho,
                               (const R*)c->j0p, (const R*)c->jt0, (const R*)c->jt1, (R*)c->u);
        HIPCHK(hipGetLastError());
        return LB2P_OK;
    }

    // Host bookkeeping once the solve's pass count is known.
    static void book(lb2p_ctx* c, const SolveRun& run, bool advance)
    {
        if (c->prm.fixed_iter <= 0) {
            c->last_iters = run.last_done >= 0 ? run.last_done : run.launched;
            c->status_pending = true;
        } else {
            c->last_iters = c->prm.fixed_iter;
        }
        if (c->prof && !c->capturing) c->prof_passes += c->last_iters;
        if (advance) {
            c->have_prev = true;
            c->prev_keep = false;
            c->nprev = std::min(c->nprev + 1, 3);
        }
        c->solved = true;
    }

    // Before lb2p_moments re-solves the current state: move the last step's
    // final j~ (the next step's warm start) out of the j~ buffers.
    static void keep_prev(lb2p_ctx* c)
    {
        if (!c->have_prev || c->prev_keep || !c->prm.warm_start) return;
        hipLaunchKernelGGL((k_keep_jt<Q, R>), sgrid(c), sblock(c), 0, c->stream, c->dtab, c->site_tiles,
                           (const SolveInfo*)c->info, (const R*)c->jt0, (const R*)c->jt1, (R*)c->Y);
        hipLaunchKernelGGL(k_info_keep, dim3((c->ndom + 255) / 256), dim3(256), 0, c->stream,
                           (const SolveInfo*)c->info, c->info_keep, c->ndom);
        c->prev_keep = true;
    }

    static lb2p_status step(lb2p_ctx* c)
    {
        // after the fused solve the first closure kernel forms the final j~
        // and u (k_closure1_zm in 3D, k_closure1_t2 in 2D)
        const bool closure_forms = !(c->prm.flags & LB2P_FLAG_UNFUSED_SOLVE);
        // Tolerance mode: the rest of the step is launched behind the
        // host's first read of the stop rule, without waiting for it, so the
        // GPU does not idle while the read travels.  Those kernels run only
        // if the rule then held in every domain (go = 1, set on the device by
        // that check); otherwise they do nothing, the passes go on and the
        // rest of the step is launched again after them.
        const bool speculate = closure_forms && c->prm.fixed_iter <= 0 && !c->capturing;
        SolveRun run;
        lb2p_status st = solve(c, true, !closure_forms, speculate ? &run : nullptr);
        if (st != LB2P_OK) return st;
        if (!run.pending) return post_solve(c, closure_forms);
        st = launch_finish(c, run, false, true);
        if (st != LB2P_OK) return st;
        const size_t mark = c->pending.size();
        st = post_kernels(c, closure_forms);
        if (st != LB2P_OK) return st;
        HIPCHK(hipEventSynchronize(c->spec_ev));
        if (c->host->ndone >= c->ndom) {
            run.last_done = c->host->ndone_last;
        } else {
            // the launches behind the read did nothing: drop their timing
            // records, run the remaining passes and launch them again
            prof_drop(c, mark);
            run.pending = false;
            st = iterate(c, run, false);
            if (st != LB2P_OK) return st;
            st = launch_finish(c, run, false, false);
            if (st != LB2P_OK) return st;
            st = post_kernels(c, closure_forms);
            if (st != LB2P_OK) return st;
        }
        book(c, run, true);
        return end_step(c);
    }

    static lb2p_status post_solve(lb2p_ctx* c, bool closure_forms)
    {
        lb2p_status st = post_kernels(c, closure_forms);
        if (st != LB2P_OK) return st;
        return end_step(c);
    }

    static lb2p_status end_step(lb2p_ctx* c)
    {
        std::swap(c->A, c->B);
        c->sigma_valid = true;
        return LB2P_OK;
    }

    // Items 9-12 after the solve: the closure fields, Sigma and the
    // collision into the other population buffer.  Each kernel runs only if
    // go = 1 (the solve is finished).
    static lb2p_status post_kernels(lb2p_ctx* c, bool closure_forms)
    {
        {
            ProfScope _ps(c, LB2P_K_CLOSURE1);
            if constexpr (Lattice<Q>::D == 3) {
                constexpr int TX = fused_tx<R>();
                hipLaunchKernelGGL((k_closure1_zm<R, TX, kFusedTY>), dim3((unsigned)c->clos_host.size()),
                                   dim3(TX, kFusedTY, 1), 0, c->stream, c->dtab, c->clos_tiles,
                                   (const SolveInfo*)c->info, (const R*)c->pf, (const R*)c->rho,
                                   (const R*)c->j0p, (R*)c->u, (const R*)c->u1, (R*)c->jt0, (R*)c->jt1,
                                   (R*)c->X, (R*)c->T, (R*)c->Y, (R*)c->Xi, closure_forms ? 1 : 0,
                                   (const int*)c->go);
            } else {
                hipLaunchKernelGGL((k_closure1_t2<R, kClos2TX, kClos2TY>), dim3((unsigned)c->clos_host.size()),
                                   dim3(kClos2TX, kClos2TY, 1), 0, c->stream, c->dtab, c->clos_tiles,
                                   (const SolveInfo*)c->info, (const R*)c->pf, (const R*)c->rho,
                                   (const R*)c->j0p, (R*)c->u, (const R*)c->u1, (R*)c->jt0, (R*)c->jt1,
                                   (R*)c->X, (R*)c->T, (R*)c->Y, (R*)c->Xi, closure_forms ? 1 : 0,
                                   (const int*)c->go);
            }
        }
        if (c->prm.flags & LB2P_FLAG_STENCIL_CLOSURE) {
            ProfScope _ps(c, LB2P_K_CLOSURE2);
            hipLaunchKernelGGL((k_sigma_stencil<Q, R>), sgrid(c), sblock(c), 0, c->stream, c->dtab, c->site_tiles,
                               (const R*)c->pf, (const double*)c->mass, (const R*)c->u, (R*)c->Sig,
                               (const int*)c->go);
        } else {
            ProfScope _ps(c, LB2P_K_CLOSURE2);
            if constexpr (Lattice<Q>::D == 3) {
                constexpr int TX = fused_tx<R>();
                hipLaunchKernelGGL((k_closure2_zm<R, TX, kFusedTY>), dim3((unsigned)c->clos_host.size()),
                                   dim3(TX, kFusedTY, 1), 0, c->stream, c->dtab, c->clos_tiles,
                                   (const R*)c->rho, (const R*)c->u, (const R*)c->X, (const R*)c->T,
                                   (const R*)c->Y, (R*)c->Sig, (const int*)c->go);
            } else {
                hipLaunchKernelGGL((k_closure2_t2<R, kClos2TX, kClos2TY>), dim3((unsigned)c->clos_host.size()),
                                   dim3(kClos2TX, kClos2TY, 1), 0, c->stream, c->dtab, c->clos_tiles,
                                   (const R*)c->rho, (const R*)c->u, (const R*)c->X, (const R*)c->T,
                                   (const R*)c->Y, (R*)c->Sig, (const int*)c->go);
            }
        }
        {
            ProfScope _ps(c, LB2P_K_COLLIDE);
            auto kc = c->any_pull ? k_collide<Q, R, S, true> : k_collide<Q, R, S, false>;
            hipLaunchKernelGGL(kc, sgrid(c), sblock(c), 0, c->stream, c->dtab,
                               c->site_tiles, (const SolveInfo*)c->info, (const S*)c->A, (S*)c->B,
                               (const R*)c->u, (const R*)c->f, (const R*)c->jt0,
                               (const R*)c->jt1, (const R*)c->Sig, (const R*)c->Xi, (const double*)c->mass,
                               (const int*)c->go);
        }
        HIPCHK(hipGetLastError());
        return LB2P_OK;
    }

    static void export_pop(lb2p_ctx* c, double* out)
    {
        hipLaunchKernelGGL((k_export<Q, S>), sgrid(c), sblock(c), 0, c->stream, c->dtab, c->site_tiles,
                           (const S*)c->A, out);
    }
    static void import_pop(lb2p_ctx* c, const double* in)
    {
        hipLaunchKernelGGL((k_import<Q, S>), sgrid(c), sblock(c), 0, c->stream, c->dtab, c->site_tiles,
                           in, (S*)c->A);
    }
};

template <int Q, class F>
auto by_storage(lb2p_ctx* c, F&& fn)
{
    switch (c->prm.storage) {
        case LB2P_STORE_F64: return fn(Impl<Q, double, double>{});
        case LB2P_STORE_F32:
            if (c->rsize == 8) return fn(Impl<Q, double, float>{});
            return fn(Impl<Q, float, float>{});
        case LB2P_STORE_BF16:
            if (c->rsize == 8) return fn(Impl<Q, double, __bf16>{});
            return fn(Impl<Q, float, __bf16>{});
        default:
            if (c->rsize == 8) return fn(Impl<Q, double, _Float16>{});
            return fn(Impl<Q, float, _Float16>{});
    }
}

template <class F>
auto dispatch(lb2p_ctx* c, F&& fn)
{
    if (c->Q == 59) return by_storage<59>(c, fn);
    return by_storage<21>(c, fn);
}

// Precision of the per-site fields, and with them of the j~ iteration:
// FP64 with FP64 storage; otherwise FP32 unless iter_prec asks for FP64, or
// leaves it to the library (AUTO) and the stop rule's tolerance is below
// what the FP32 iteration can meet.  In the FP32 velocity-form iteration the
// iterate u is an FP32 number, so |G(x_k) - x_k| = |G + j0' - rho u_k|
// cannot fall much below the rounding of rho u next to max|j0'|
// (measured: it stalls at tol 1e-7 on the slab workload, and tolerances
// down to 2e-7 converge).
size_t field_bytes(const lb2p_params& p)
{
    if (p.storage == LB2P_STORE_F64 || p.iter_prec == LB2P_ITER_F64) return 8;
    if (p.iter_prec == LB2P_ITER_AUTO && p.fixed_iter <= 0 && p.tol < LB2P_F32_TOL_FLOOR) return 8;
    return 4;
}

// Default stop-rule tolerance per storage form.  FP64: 1e-13.  FP32: 4e-7,
// twice the floor of the FP32 iteration.  BF16 and FP16: half the format's
// unit roundoff (2^-9, 2^-12, the roundoffs being 2^-8 and 2^-11): j0' comes
// from populations that carry relative rounding of that size, so the fixed
// point is not known better than that,
// and a tighter rule spends passes on the storage noise (measured on the
// slab workload: the velocity error is the same from 1e-3 to 4e-7).
double default_tol(int storage)
{
    switch (storage) {
        case LB2P_STORE_F64: return 1e-13;
        case LB2P_STORE_F32: return 4e-7;
        case LB2P_STORE_BF16: return 1.0 / 512.0;
        default: return 1.0 / 4096.0;
    }
}

size_t storage_bytes(int storage)
{
    switch (storage) {
        case LB2P_STORE_F64: return 8;
        case LB2P_STORE_F32: return 4;
        default: return 2;
    }
}

// Copy a field [ncomp][S] of type R to a caller buffer of dtype.  A device
// buffer of the other precision is converted into directly; a host one goes
// through a device staging area: `stage` (at least ncomp * S elements of
// dtype) when given, else a stream-ordered allocation.
lb2p_status copy_out(lb2p_ctx* c, const void* src, int ncomp, void* dst, int dtype, int on_device,
                     void* stage = nullptr)
{
    const long long n = (long long)ncomp * c->S;
    const bool same = (dtype == LB2P_DTYPE_F64) == (c->rsize == 8);
    const size_t out_elem = dtype == LB2P_DTYPE_F64 ? 8 : 4;
    const void* from = src;
    void* tmp = nullptr;
    if (!same) {
        if (on_device)
            tmp = dst;
        else if (stage)
            tmp = stage;
        else
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
    if (from != dst)
        HIPCHK(hipMemcpyAsync(dst, from, n * out_elem,
                              on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    if (tmp && tmp != dst && tmp != stage) HIPCHK(hipFreeAsync(tmp, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return LB2P_OK;
}

// Copy a caller buffer [ncomp][S] of dtype into a field of type R.
lb2p_status copy_in(lb2p_ctx* c, const void* src, int ncomp, void* dst, int dtype, int on_device)
{
    const long long n = (long long)ncomp * c->S;
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

// Copy a caller buffer of n elements of dtype into an FP64 device array.
lb2p_status copy_in_f64(lb2p_ctx* c, const void* src, long long n, double* dst, int dtype, int on_device)
{
    if (dtype == LB2P_DTYPE_F64) {
        HIPCHK(hipMemcpyAsync(dst, src, n * 8, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                              c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        return LB2P_OK;
    }
    void* tmp = nullptr;
    HIPCHK(hipMallocAsync(&tmp, n * 4, c->stream));
    HIPCHK(hipMemcpyAsync(tmp, src, n * 4, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          c->stream));
    hipLaunchKernelGGL((k_convert<float, double>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                       (const float*)tmp, dst, n);
    HIPCHK(hipFreeAsync(tmp, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return LB2P_OK;
}

void free_ctx(lb2p_ctx* c)
{
    if (!c) return;
    free_graphs(c);
    if (c->A) (void)hipFree(c->A);
    if (c->B) (void)hipFree(c->B);
    if (c->fields) (void)hipFree(c->fields);
    if (c->partial) (void)hipFree(c->partial);
    if (c->pmax) (void)hipFree(c->pmax);
    if (c->site_range) (void)hipFree(c->site_range);
    if (c->fused_range) (void)hipFree(c->fused_range);
    if (c->clos_range) (void)hipFree(c->clos_range);
    if (c->ctl) (void)hipFree(c->ctl);
    if (c->dtab) (void)hipFree(c->dtab);
    if (c->omega) (void)hipFree(c->omega);
    if (c->jhist) (void)hipFree(c->jhist);
    if (c->mass) (void)hipFree(c->mass);
    if (c->site_tiles) (void)hipFree(c->site_tiles);
    if (c->fused_tiles) (void)hipFree(c->fused_tiles);
    if (c->clos_tiles) (void)hipFree(c->clos_tiles);
    if (c->host) (void)hipHostFree(c->host);
    if (c->spec_ev) (void)hipEventDestroy(c->spec_ev);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    prof_drop(c, 0);   // records of counted-only launches hold no events
    for (auto e : c->pool) (void)hipEventDestroy(e);
    delete c;
}

std::string tune_key(const lb2p_ctx* c)
{
    std::vector<long long> sz;
    for (const auto& d : c->dom) sz.push_back(((long long)d.g.nx << 40) | ((long long)d.g.ny << 20) | d.g.nz);
    std::sort(sz.begin(), sz.end());
    unsigned long long h = 1469598103934665603ull;
    for (long long v : sz) {
        h ^= (unsigned long long)v;
        h *= 1099511628211ull;
    }
    char buf[96];
    std::snprintf(buf, sizeof(buf), "Q%d-s%d-n%d-%016llx", c->Q, c->prm.storage, c->ndom, h);
    return buf;
}

void default_shape(lb2p_ctx* c)
{
    int maxnx = 0;
    for (const auto& d : c->dom) maxnx = std::max(maxnx, d.g.nx);
    c->bx = maxnx >= 256 ? 256 : (maxnx >= 128 ? 128 : 64);
    c->by = 256 / c->bx;
    c->tz = 128;
    std::lock_guard<std::mutex> lock(tune_mutex());
    auto it = tune_cache().find(tune_key(c));
    if (it != tune_cache().end()) {
        c->bx = it->second.bx;
        c->by = it->second.by;
        c->tz = it->second.tz;
    }
}

void load_tune_file()
{
    std::lock_guard<std::mutex> lock(tune_mutex());
    static bool loaded = false;
    if (loaded) return;
    loaded = true;
    const char* path = std::getenv("LB2P_TUNE_CACHE");
    if (!path) return;
    FILE* fh = std::fopen(path, "r");
    if (!fh) return;
    char key[128];
    int bx, by, tz;
    while (std::fscanf(fh, "%127s %d %d %d", key, &bx, &by, &tz) == 4)
        if (((bx > 0 && by > 0 && bx * by == 256) || (bx == 256 && by == 0)) && tz > 0)
            tune_cache()[key] = TuneChoice{bx, by, tz};
    std::fclose(fh);
}

lb2p_status create_impl(int ndom, const lb2p_params* pp, void* hip_stream, lb2p_ctx** out)
{
    if (!pp || !out || ndom <= 0) return LB2P_EINVAL;
    *out = nullptr;
    const lb2p_params& p0 = pp[0];
    for (int d = 0; d < ndom; ++d) {
        const lb2p_params& p = pp[d];
        lb2p_status st = check_params(p);
        if (st != LB2P_OK) return st;
        if (p.lattice != p0.lattice || p.storage != p0.storage || p.tol != p0.tol ||
            p.max_iter != p0.max_iter || p.fixed_iter != p0.fixed_iter ||
            p.warm_start != p0.warm_start || p.flags != p0.flags || p.graph_steps != p0.graph_steps ||
            p.solver != p0.solver || p.iter_prec != p0.iter_prec)
            return LB2P_EINVAL;
    }
    load_tune_file();
    lb2p_ctx* c = new (std::nothrow) lb2p_ctx;
    if (!c) return LB2P_ENOMEM;
    c->prm = p0;
    c->dprm.assign(pp, pp + ndom);
    c->Q = p0.lattice;
    c->D = p0.lattice == LB2P_D3Q59 ? 3 : 2;
    c->ndom = ndom;
    c->stream = (hipStream_t)hip_stream;
    c->elem = storage_bytes(p0.storage);
    c->rsize = field_bytes(p0);
    long long off = 0;
    std::vector<double> cheb_rho;
    for (int d = 0; d < ndom; ++d) {
        const lb2p_params& p = pp[d];
        Domain dm{};
        dm.g.nx = p.nx; dm.g.ny = p.ny; dm.g.nz = p.nz;
        dm.g.N = (long long)p.nx * p.ny * p.nz;
        // kernels address one component plane of a domain with 32-bit byte
        // offsets; the widest plane is the FP64 mass
        if ((unsigned long long)dm.g.N * 8ull >= (1ull << 32)) {
            delete c;
            return LB2P_EINVAL;
        }
        dm.off = off;
        off += dm.g.N;
        dm.cf.gamma = p.gamma;
        if (p.gamma != 0.0) c->any_pull = true;
        dm.cf.kappa = p.kappa;
        dm.cf.eos = make_eos(p.eos);
        dm.cf.c0sq = eos_cs2<double>(dm.cf.eos, p.rho0);
        double w[8] = {0};
        if (c->Q == 59) shell_weights<59, double>(dm.cf.c0sq, w);
        else shell_weights<21, double>(dm.cf.c0sq, w);
        const int ns = c->Q == 59 ? 8 : 6;
        for (int k = 0; k < ns; ++k) {
            if (!(w[k] > 0.0)) { delete c; return LB2P_EEOS; }
            dm.cf.Wk[k] = w[k];
        }
        {
            const double r0 = p.store_rho_ref > 0.0 ? p.store_rho_ref : p.rho0;
            set_devscale(dm.ds, c->Q, dm.cf.eos, r0, 0.75 * r0, 1.25 * r0);
            set_refs(dm);
        }
        {
            const double b = p.spectral_bound > 0.0 ? p.spectral_bound
                                                    : spectral_bound_from_eos(c->D, dm.cf.eos, p.eos);
            if (p.solver == LB2P_SOLVER_CHEBYSHEV && !(b < 1.0)) { delete c; return LB2P_EINVAL; }
            dm.cf.cheb_gamma = 2.0 / (2.0 - b);
            cheb_rho.push_back(b / (2.0 - b));
        }
        c->dom.push_back(dm);
    }
    c->S = off;
    if (c->S > (1LL << 31)) { delete c; return LB2P_EINVAL; }
    for (auto& dm : c->dom) dm.g.S = c->S;
    c->stride = (p0.fixed_iter > 0 ? p0.fixed_iter : p0.max_iter) + 1;

    const long long S = c->S;
    const int D = c->D;
    const int nsig = D == 3 ? 6 : 3, nxi = D == 3 ? 10 : 4;
    // rho | j0 | f | j0p | u | jt0 | jt1 | q (alias T) | X | Y | Xi | Sig | pf (4) | u1
    const int ncomp = 1 + 6 * D + nsig + 1 + D + nxi + nsig + 4 + D;
    {
        long long mo = 0;
        switch (p0.storage) {
            case LB2P_STORE_F64: mo = moving_offset_bytes<double>(S); break;
            case LB2P_STORE_F32: mo = moving_offset_bytes<float>(S); break;
            case LB2P_STORE_BF16: mo = moving_offset_bytes<__bf16>(S); break;
            default: mo = moving_offset_bytes<_Float16>(S); break;
        }
        c->pbytes = (size_t)mo + (size_t)(c->Q - 1) * S * c->elem;
    }
    hipError_t e = hipMalloc(&c->A, c->pbytes);
    if (e == hipSuccess) e = hipMalloc(&c->B, c->pbytes);
    if (e == hipSuccess) e = hipMalloc(&c->fields, (size_t)ncomp * S * c->rsize);
    if (e == hipSuccess) e = hipMalloc((void**)&c->dtab, ndom * sizeof(Domain));
    const size_t nres = (size_t)ndom * c->stride;
    const size_t sbytes = 256 + sizeof(unsigned long long) * nres + (sizeof(unsigned long long) +
                          sizeof(int) + 2 * sizeof(SolveInfo)) * (size_t)ndom + 64;
    if (e == hipSuccess) e = hipMalloc(&c->ctl, sbytes);
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->host, sizeof(lb2p_ctx::HostReadback), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->spec_ev, hipEventDisableTiming);
    if (e == hipSuccess && p0.solver == LB2P_SOLVER_CHEBYSHEV)
        e = hipMalloc((void**)&c->omega, sizeof(double) * nres);
    if (e == hipSuccess) e = hipMalloc((void**)&c->mass, sizeof(double) * (size_t)S);
    if (e == hipSuccess && p0.warm_start >= 2) {
        const size_t hb = (size_t)(p0.warm_start - 1) * D * S * c->rsize;
        e = hipMalloc(&c->jhist, hb);
        if (e == hipSuccess) e = hipMemsetAsync(c->jhist, 0, hb, c->stream);
    }
    if (e != hipSuccess) {
        free_ctx(c);
        (void)hipGetLastError();
        return LB2P_ENOMEM;
    }
    c->A0 = c->A;
    char* fb = (char*)c->fields;
    size_t foff = 0;
    auto take = [&](int nc) { void* ptr = fb + foff * c->rsize; foff += (size_t)nc * S; return ptr; };
    c->rho = take(1); c->j0 = take(D); c->f = take(D); c->j0p = take(D); c->u = take(D);
    c->jt0 = take(D); c->jt1 = take(D); c->q = take(nsig); c->T = c->q;
    c->X = take(1); c->Y = take(D); c->Xi = take(nxi); c->Sig = take(nsig); c->pf = take(4); c->u1 = take(D);
    char* sb = (char*)c->ctl;
    c->flags = (int*)(sb + 0);
    c->nconv = (int*)(sb + 4);
    c->ndone = (int*)(sb + 8);   // two ints
    c->go = (int*)(sb + 16);
    c->sums = (double*)(sb + 64);
    c->res = (unsigned long long*)(sb + 256);
    c->jscale = c->res + nres;
    c->info = (SolveInfo*)(c->jscale + ndom);
    c->info_keep = c->info + ndom;
    c->done_at = (int*)(c->info_keep + ndom);
    std::memset(c->host, 0, sizeof(lb2p_ctx::HostReadback));
    c->info_host.assign(ndom, SolveInfo{0, 0, 1, 0});
    c->js_host.assign(ndom, 0ull);
    if (hipGetDevice(&c->device) != hipSuccess || scratch_address(c->device, &c->stage) != LB2P_OK) {
        free_ctx(c);
        return LB2P_EHIP;
    }
    std::vector<double> om;
    if (c->omega) {
        // Chebyshev weights per domain: omega_0 = 1, omega_1 = 1/(1 - r^2/2),
        // omega_m = 1/(1 - r^2 omega_{m-1}/4), r = b/(2-b) (Golub-Varga)
        om.resize(nres);
        for (int d = 0; d < ndom; ++d) {
            const double r2 = cheb_rho[d] * cheb_rho[d];
            double* w = om.data() + (size_t)d * c->stride;
            for (int m = 0; m < c->stride; ++m)
                w[m] = m == 0 ? 1.0 : (m == 1 ? 1.0 / (1.0 - 0.5 * r2) : 1.0 / (1.0 - 0.25 * r2 * w[m - 1]));
        }
    }
    if ((c->omega && hipMemcpyAsync(c->omega, om.data(), sizeof(double) * nres, hipMemcpyHostToDevice,
                                    c->stream) != hipSuccess) ||
        hipMemcpyAsync(c->dtab, c->dom.data(), ndom * sizeof(Domain), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemsetAsync(c->ctl, 0, sbytes, c->stream) != hipSuccess ||
        hipMemsetAsync(c->fields, 0, (size_t)ncomp * S * c->rsize, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        free_ctx(c);
        return LB2P_EHIP;
    }
    default_shape(c);
    lb2p_status st = build_tiles(c);
    if (st != LB2P_OK) {
        free_ctx(c);
        return st;
    }
    *out = c;
    return LB2P_OK;
}

// nsteps steps: eager launches, or replays of the captured graph (fixed
// iteration count, graph_steps > 0).
// Tolerance mode: the domains that hit max_iter (counted on the device over
// the steps since the last read) and the non-finite flag, read with one
// synchronisation per call.
lb2p_status read_status(lb2p_ctx* c)
{
    if (!c->status_pending) return LB2P_OK;
    c->status_pending = false;
    HIPCHK(hipMemcpyAsync(&c->host->nconv, c->nconv, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(&c->host->flags, c->flags, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemsetAsync(c->nconv, 0, sizeof(int), c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->host->nconv > 0 && c->sticky == LB2P_OK) c->sticky = LB2P_ENOCONV;
    if (c->host->flags) c->sticky = LB2P_ENONFINITE;
    return LB2P_OK;
}

lb2p_status run_steps(lb2p_ctx* c, int nsteps)
{
    const int gs = c->prm.graph_steps > 0 && c->prm.fixed_iter > 0 ? (c->prm.graph_steps + 1) / 2 * 2 : 0;
    int s = 0;
    if (gs > 0 && !c->prof) {
        // a captured step warm-starts j~ from the previous step(s); the first
        // steps after lb2p_init have none, so they run eagerly
        // (and so does the first step after lb2p_moments, which reads its start
        // from where that call kept it)
        while (s < nsteps && (!c->have_prev || c->prev_keep ||
                              (c->prm.warm_start >= 2 && c->nprev < c->prm.warm_start))) {
            lb2p_status st = dispatch(c, [&](auto impl) { return decltype(impl)::step(c); });
            if (st != LB2P_OK) return st;
            ++s;
        }
        while (nsteps - s >= gs) {
            const int par = c->A == c->A0 ? 0 : 1;
            if (!c->graph[par]) {
                // capture gs steps (an even count: the buffers end as they
                // began) on a private stream; the graph runs on c->stream
                if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
                HIPCHK(hipStreamSynchronize(c->stream));
                hipStream_t user = c->stream;
                c->stream = c->cap_stream;
                hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
                if (e != hipSuccess) {
                    c->stream = user;
                    return LB2P_EHIP;
                }
                c->capturing = true;
                lb2p_status st = LB2P_OK;
                for (int k = 0; k < gs && st == LB2P_OK; ++k)
                    st = dispatch(c, [&](auto impl) { return decltype(impl)::step(c); });
                c->capturing = false;
                hipGraph_t g = nullptr;
                e = hipStreamEndCapture(c->stream, &g);
                c->stream = user;
                if (st != LB2P_OK) {
                    if (g) (void)hipGraphDestroy(g);
                    return st;
                }
                if (e != hipSuccess) return LB2P_EHIP;
                e = hipGraphInstantiate(&c->graph[par], g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) return LB2P_EHIP;
            }
            HIPCHK(hipGraphLaunch(c->graph[par], c->stream));
            s += gs;
        }
    }
    for (; s < nsteps; ++s) {
        lb2p_status st = dispatch(c, [&](auto impl) { return decltype(impl)::step(c); });
        if (st != LB2P_OK) return st;
    }
    return LB2P_OK;
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
        case LB2P_ESIZE: return "output larger than the static staging area of lb2p_moments_noalloc";
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
    p.tol = default_tol(storage);
    p.max_iter = 200;
    p.fixed_iter = 0;
    p.warm_start = 1;
    p.check_every = 0;
    p.store_rho_ref = 0.0;
    p.flags = 0;
    p.graph_steps = 0;
    p.solver = LB2P_SOLVER_FIXED_POINT;
    p.spectral_bound = 0.0;
    p.iter_prec = LB2P_ITER_AUTO;
    *out = p;
    return LB2P_OK;
}

lb2p_status lb2p_create(const lb2p_params* params, void* hip_stream, lb2p_ctx** out)
{
    return create_impl(1, params, hip_stream, out);
}

lb2p_status lb2p_create_batch(int ndom, const lb2p_params* per_dom, void* hip_stream, lb2p_ctx** out)
{
    return create_impl(ndom, per_dom, hip_stream, out);
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
    // the density goes to the FP64 mass plane (the initial populations are
    // evaluated from it in FP64) and, rounded, to the rho field
    lb2p_status st = copy_in_f64(c, rho, c->S, c->mass, dtype, on_device);
    if (st != LB2P_OK) return st;
    st = copy_in(c, u, c->D, c->u, dtype, on_device);
    if (st != LB2P_OK) return st;
    // deviation-storage reference per domain: the given value, else the
    // domain's mean initial density (host FP64 sum)
    // the density range of every domain (for the reduced-storage offsets)
    // and, where no reference density is given, its mean
    const bool need_rho = c->prm.storage != LB2P_STORE_F64 ||
                          std::any_of(c->dprm.begin(), c->dprm.end(),
                                      [](const lb2p_params& p) { return !(p.store_rho_ref > 0.0); });
    {
        const long long n = c->S;
        const long long nb = (n + 255) / 256;
        if (c->rsize == 8)
            HIPCHK(hipMemcpyAsync(c->rho, c->mass, n * 8, hipMemcpyDeviceToDevice, c->stream));
        else
            hipLaunchKernelGGL((k_convert<double, float>), dim3((unsigned)nb), dim3(256), 0, c->stream,
                               (const double*)c->mass, (float*)c->rho, n);
    }
    std::vector<double> hrho;
    if (need_rho) {
        hrho.resize(c->S);
        HIPCHK(hipMemcpyAsync(hrho.data(), c->mass, c->S * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    for (int d = 0; d < c->ndom; ++d) {
        double rref = c->dprm[d].store_rho_ref;
        double lo = 0.75 * rref, hi = 1.25 * rref;
        if (need_rho) {
            double acc = 0.0, mn = 1e300, mx = -1e300;
            const Domain& dm = c->dom[d];
            for (long long k = 0; k < dm.g.N; ++k) {
                const double v = hrho[dm.off + k];
                acc += v;
                mn = std::fmin(mn, v);
                mx = std::fmax(mx, v);
            }
            if (!(rref > 0.0)) rref = acc / (double)dm.g.N;
            const double pad = 0.05 + 0.25 * (mx - mn);
            lo = mn - pad;
            hi = mx + pad;
        }
        set_devscale(c->dom[d].ds, c->Q, c->dom[d].cf.eos, rref, lo, hi);
        set_refs(c->dom[d]);
    }
    HIPCHK(hipMemcpyAsync(c->dtab, c->dom.data(), c->ndom * sizeof(Domain), hipMemcpyHostToDevice, c->stream));
    dispatch(c, [&](auto impl) { decltype(impl)::launch_init(c); });
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemsetAsync(c->flags, 0, sizeof(int), c->stream));
    HIPCHK(hipMemsetAsync(c->nconv, 0, sizeof(int), c->stream));
    c->status_pending = false;
    HIPCHK(hipStreamSynchronize(c->stream));
    c->initialized = true;
    c->solved = false;
    c->have_prev = false;
    c->prev_keep = false;
    c->nprev = 0;
    c->sigma_valid = false;
    c->sticky = LB2P_OK;
    return LB2P_OK;
}

lb2p_status lb2p_step(lb2p_ctx* c, int nsteps)
{
    if (!c || nsteps < 0) return LB2P_EINVAL;
    if (!c->initialized) return LB2P_ESTATE;
    lb2p_status st = run_steps(c, nsteps);
    if (st != LB2P_OK) return st;
    if (c->prm.fixed_iter > 0) HIPCHK(hipGetLastError());
    st = read_status(c);
    if (st != LB2P_OK) return st;
    return c->sticky;
}

}  // extern "C"

namespace {

// lb2p_moments; `stage` (device, or null) stages the precision conversion of
// host outputs, one field at a time.
lb2p_status moments_impl(lb2p_ctx* c, void* rho_out, void* u_out, int dtype, int on_device, lb2p_stats* st,
                         void* stage)
{
    if (!c) return LB2P_EINVAL;
    if (!c->initialized) return LB2P_ESTATE;
    if (dtype != LB2P_DTYPE_F64 && dtype != LB2P_DTYPE_F32) return LB2P_EINVAL;
    // the solve below must not change what the next lb2p_step starts from
    lb2p_status s = dispatch(c, [&](auto impl) {
        decltype(impl)::keep_prev(c);
        return decltype(impl)::solve(c, false);
    });
    if (s != LB2P_OK) return s;
    c->status_pending = true;   // the call synchronises anyway: read the flags too
    s = read_status(c);
    if (s != LB2P_OK) return s;
    c->sigma_valid = false;
    if (rho_out) {
        s = copy_out(c, c->rho, 1, rho_out, dtype, on_device, stage);
        if (s != LB2P_OK) return s;
    }
    if (u_out) {
        s = copy_out(c, c->u, c->D, u_out, dtype, on_device, stage);
        if (s != LB2P_OK) return s;
    }
    if (st) {
        s = lb2p_stats_get(c, st);
        if (s != LB2P_OK) return s;
    }
    return c->sticky;
}

}  // namespace

extern "C" {

lb2p_status lb2p_moments(lb2p_ctx* c, void* rho_out, void* u_out, int dtype, int on_device,
                         lb2p_stats* st)
{
    return moments_impl(c, rho_out, u_out, dtype, on_device, st, nullptr);
}

lb2p_status lb2p_moments_noalloc(lb2p_ctx* c, void* rho_out, void* u_out, int dtype, int on_device,
                                 lb2p_stats* st)
{
    if (!c) return LB2P_EINVAL;
    if (dtype != LB2P_DTYPE_F64 && dtype != LB2P_DTYPE_F32) return LB2P_EINVAL;
    // host outputs of the other precision are staged one field at a time,
    // the widest being u: d * N elements of dtype
    const bool convert = (dtype == LB2P_DTYPE_F64) != (c->rsize == 8);
    const size_t need = (size_t)c->D * (size_t)c->S * (dtype == LB2P_DTYPE_F64 ? 8 : 4);
    if (convert && !on_device && need > kNoAllocStageBytes) return LB2P_ESIZE;
    return moments_impl(c, rho_out, u_out, dtype, on_device, st, c->stage);
}

lb2p_status lb2p_stats_get(lb2p_ctx* c, lb2p_stats* st)
{
    if (!c || !st) return LB2P_EINVAL;
    if (!c->initialized) return LB2P_ESTATE;
    // totals of the current state (item 1 evaluated into spare field space)
    dispatch(c, [&](auto impl) { decltype(impl)::launch_moments(c, false); });
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, c->stream, c->partial, 0LL,
                       (long long)c->site_host.size(), c->sums);
    HIPCHK(hipMemcpyAsync(c->host->sums, c->sums, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(&c->host->flags, c->flags, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(c->info_host.data(), c->info, c->ndom * sizeof(SolveInfo),
                          hipMemcpyDeviceToHost, c->stream));
    std::vector<unsigned long long>& js = c->js_host;
    HIPCHK(hipMemcpyAsync(js.data(), c->jscale, c->ndom * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    // iteration count and residual: the largest over domains
    int it = 0;
    for (const auto& si : c->info_host) it = std::max(it, si.iters);
    double rmax = 0.0, jmax = 0.0;
    for (int d = 0; d < c->ndom; ++d) {
        const int k = c->info_host[d].iters;
        if (k > 0) {
            unsigned long long rs = 0;
            HIPCHK(hipMemcpy(&rs, c->res + (size_t)d * c->stride + (k - 1), sizeof(rs), hipMemcpyDeviceToHost));
            double rd;
            std::memcpy(&rd, &rs, sizeof(rd));
            rmax = std::max(rmax, rd);
        }
        double jd;
        std::memcpy(&jd, &js[d], sizeof(jd));
        jmax = std::max(jmax, jd);
    }
    st->mass = c->host->sums[0];
    st->mom[0] = c->host->sums[1];
    st->mom[1] = c->host->sums[2];
    st->mom[2] = c->D == 3 ? c->host->sums[3] : 0.0;
    st->iters = it;
    st->resid = rmax;
    st->jscale = jmax;
    st->nonfinite = c->host->flags ? 1 : 0;
    if (c->host->flags) c->sticky = LB2P_ENONFINITE;
    return LB2P_OK;
}

lb2p_status lb2p_domain_totals(lb2p_ctx* c, double* out)
{
    if (!c || !out) return LB2P_EINVAL;
    if (!c->initialized) return LB2P_ESTATE;
    dispatch(c, [&](auto impl) { decltype(impl)::launch_moments(c, false); });
    const size_t nb = c->site_host.size();
    std::vector<double> part(4 * nb);
    HIPCHK(hipMemcpyAsync(part.data(), c->partial, 4 * nb * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    std::fill(out, out + 4 * c->ndom, 0.0);
    // deterministic: tiles of a domain in launch order
    for (size_t b = 0; b < nb; ++b) {
        const int d = c->site_host[b].dom;
        if (d < 0) continue;
        for (int k = 0; k < 4; ++k) out[4 * d + k] += part[4 * b + k];
    }
    if (c->D == 2)
        for (int d = 0; d < c->ndom; ++d) out[4 * d + 3] = 0.0;
    return LB2P_OK;
}

lb2p_status lb2p_domain_solve(lb2p_ctx* c, int* iters, double* resid, double* jscale, int* converged)
{
    if (!c) return LB2P_EINVAL;
    if (!c->initialized || !c->solved) return LB2P_ESTATE;
    std::vector<SolveInfo> info(c->ndom);
    std::vector<unsigned long long> res((size_t)c->ndom * c->stride), js(c->ndom);
    HIPCHK(hipMemcpyAsync(info.data(), c->info, c->ndom * sizeof(SolveInfo), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(res.data(), c->res, res.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipMemcpyAsync(js.data(), c->jscale, c->ndom * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int d = 0; d < c->ndom; ++d) {
        const int k = info[d].iters;
        if (iters) iters[d] = k;
        if (converged) converged[d] = info[d].converged;
        if (resid) {
            double r = 0.0;
            if (k > 0) std::memcpy(&r, &res[(size_t)d * c->stride + (k - 1)], sizeof(r));
            resid[d] = r;
        }
        if (jscale) std::memcpy(&jscale[d], &js[d], sizeof(double));
    }
    return LB2P_OK;
}

lb2p_status lb2p_get_field(lb2p_ctx* c, int field, void* out, int dtype, int on_device)
{
    if (!c || !out) return LB2P_EINVAL;
    if (!c->initialized) return LB2P_ESTATE;
    if (dtype != LB2P_DTYPE_F64 && dtype != LB2P_DTYPE_F32) return LB2P_EINVAL;
    const int D = c->D;
    switch (field) {
        case LB2P_FIELD_RHO: return copy_out(c, c->rho, 1, out, dtype, on_device);
        case LB2P_FIELD_J0: return copy_out(c, c->j0, D, out, dtype, on_device);
        case LB2P_FIELD_FORCE: return copy_out(c, c->f, D, out, dtype, on_device);
        case LB2P_FIELD_JTILDE: {
            // the final iterate of each domain may sit in either buffer
            HIPCHK(hipMemcpyAsync(c->info_host.data(), c->info, c->ndom * sizeof(SolveInfo),
                                  hipMemcpyDeviceToHost, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            bool all0 = true, all1 = true;
            for (const auto& si : c->info_host) {
                all0 &= si.final_buf == 0;
                all1 &= si.final_buf == 1;
            }
            if (all0 || all1) return copy_out(c, all1 ? c->jt1 : c->jt0, D, out, dtype, on_device);
            // mixed: gather per domain into the (free) q space
            const size_t rs = c->rsize;
            for (int d = 0; d < c->ndom; ++d) {
                const Domain& dm = c->dom[d];
                const char* src = (const char*)(c->info_host[d].final_buf ? c->jt1 : c->jt0);
                for (int a = 0; a < D; ++a)
                    HIPCHK(hipMemcpyAsync((char*)c->q + (a * c->S + dm.off) * rs, src + (a * c->S + dm.off) * rs,
                                          dm.g.N * rs, hipMemcpyDeviceToDevice, c->stream));
            }
            return copy_out(c, c->q, D, out, dtype, on_device);
        }
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
    const size_t bytes = (size_t)c->Q * c->S * sizeof(double);
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
    const size_t bytes = (size_t)c->Q * c->S * sizeof(double);
    const double* src = n_in;
    double* tmp = nullptr;
    if (!on_device) {
        HIPCHK(hipMallocAsync((void**)&tmp, bytes, c->stream));
        HIPCHK(hipMemcpyAsync(tmp, n_in, bytes, hipMemcpyHostToDevice, c->stream));
        src = tmp;
    }
    dispatch(c, [&](auto impl) { decltype(impl)::import_pop(c, src); });
    HIPCHK(hipGetLastError());
    if (tmp) HIPCHK(hipFreeAsync(tmp, c->stream));
    HIPCHK(hipMemsetAsync(c->flags, 0, sizeof(int), c->stream));
    HIPCHK(hipMemsetAsync(c->nconv, 0, sizeof(int), c->stream));
    c->status_pending = false;
    HIPCHK(hipStreamSynchronize(c->stream));
    c->initialized = true;
    c->solved = false;
    c->have_prev = false;
    c->prev_keep = false;
    c->nprev = 0;
    c->sigma_valid = false;
    c->sticky = LB2P_OK;
    return LB2P_OK;
}

lb2p_status lb2p_autotune(lb2p_ctx* c, int steps)
{
    if (!c) return LB2P_EINVAL;
    if (!c->initialized) return LB2P_ESTATE;
    if (steps <= 0) steps = 2;
    const size_t pbytes = c->pbytes;
    void* save = nullptr;
    if (hipMalloc(&save, pbytes) != hipSuccess) {
        (void)hipGetLastError();
        return LB2P_ENOMEM;
    }
    HIPCHK(hipMemcpyAsync(save, c->A, pbytes, hipMemcpyDeviceToDevice, c->stream));
    void* const A_orig = c->A;
    void* const B_orig = c->B;
    const lb2p_params keep = c->prm;
    // the same work for every candidate; the residual record of each domain
    // has max_iter + 1 slots (fixed_iter + 1 when fixed), so at most that
    if (c->prm.fixed_iter <= 0) c->prm.fixed_iter = std::min(4, c->prm.max_iter);
    c->prm.graph_steps = 0;
    const bool prof_keep = c->prof;
    c->prof = false;
    // site-tile shapes (bx, by); (256, 0): linear tiles of 256 consecutive sites
    const int shapes[5][2] = {{64, 4}, {128, 2}, {256, 1}, {32, 8}, {256, 0}};
    const int tzs[5] = {8, 16, 32, 64, 128};   // solve-pass chunks (8 pays on grids of 64^3 and below)
    hipEvent_t e0 = nullptr, e1 = nullptr;
    lb2p_status st = LB2P_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = LB2P_EHIP;
    TuneChoice best{c->bx, c->by, c->tz};
    float best_ms = 1e30f;
    for (int si = 0; si < 5 && st == LB2P_OK; ++si)
        for (int ti = 0; ti < (c->D == 3 ? 5 : 1) && st == LB2P_OK; ++ti) {
            c->bx = shapes[si][0];
            c->by = shapes[si][1];
            c->tz = tzs[ti];
            st = build_tiles(c);
            if (st != LB2P_OK) break;
            // every candidate starts from the same populations
            c->A = A_orig;
            c->B = B_orig;
            if (hipMemcpyAsync(c->A, save, pbytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess) {
                st = LB2P_EHIP;
                break;
            }
            c->have_prev = false;
            c->prev_keep = false;
            c->nprev = 0;
            st = run_steps(c, 1);   // warm-up
            if (st != LB2P_OK) break;
            float ms = 0.f;
            if (hipEventRecord(e0, c->stream) != hipSuccess) { st = LB2P_EHIP; break; }
            st = run_steps(c, steps);
            if (st != LB2P_OK) break;
            if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                st = LB2P_EHIP;
                break;
            }
            if (ms < best_ms) {
                best_ms = ms;
                best = TuneChoice{c->bx, c->by, c->tz};
            }
        }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    c->prm = keep;
    c->prof = prof_keep;
    c->bx = best.bx;
    c->by = best.by;
    c->tz = best.tz;
    c->A = A_orig;
    c->B = B_orig;
    if (st == LB2P_OK) st = build_tiles(c);
    (void)hipMemcpyAsync(c->A, save, pbytes, hipMemcpyDeviceToDevice, c->stream);
    (void)hipMemsetAsync(c->flags, 0, sizeof(int), c->stream);
    (void)hipMemsetAsync(c->nconv, 0, sizeof(int), c->stream);
    c->status_pending = false;
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(save);
    c->have_prev = false;
    c->prev_keep = false;
    c->nprev = 0;
    c->sticky = LB2P_OK;
    if (st != LB2P_OK) return st;
    const std::string key = tune_key(c);
    {
        std::lock_guard<std::mutex> lock(tune_mutex());
        tune_cache()[key] = best;
    }
    if (const char* path = std::getenv("LB2P_TUNE_CACHE")) {
        if (FILE* fh = std::fopen(path, "a")) {
            std::fprintf(fh, "%s %d %d %d\n", key.c_str(), best.bx, best.by, best.tz);
            std::fclose(fh);
        }
    }
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
    c->prof_passes = 0;
    return LB2P_OK;
}

lb2p_status lb2p_profile_passes(lb2p_ctx* c, long long* passes_out)
{
    if (!c || !passes_out) return LB2P_EINVAL;
    *passes_out = c->prof_passes;
    return LB2P_OK;
}

lb2p_status lb2p_set_tiling(lb2p_ctx* c, int bx, int by, int tz)
{
    if (!c || tz < 1) return LB2P_EINVAL;
    if (!((bx > 0 && by > 0 && bx * by == 256) || (bx == 256 && by == 0))) return LB2P_EINVAL;
    c->bx = bx;
    c->by = by;
    c->tz = tz;
    return build_tiles(c);
}

lb2p_status lb2p_profile_classes(lb2p_ctx* c, unsigned mask)
{
    if (!c || (mask >> LB2P_NKERNEL) != 0u) return LB2P_EINVAL;
    c->prof_mask = mask;
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
