// kernels.hpp -- gfx950 kernels of one consistent two-phase LB step.
//
// Populations live in two structure-of-arrays buffers A/B (a rest plane and
// Q-1 moving planes, layout at RestOf below).  The
// buffer read by a step holds post-collision values at their source sites,
// so the pre-collision population of the step is the pull
// n_i(r) = A_i(r - c_i); the collision writes n*_i(r) at r into the other
// buffer.  (The paper pushes n*_i to r + c_i; on a periodic lattice the two
// forms are the same map.)
//
// Every buffer may hold several independent lattices ("domains") packed one
// after the other: component k of a field at local site s of domain d is
// F[k*S + off_d + s], S the total number of sites.  A kernel block works on
// one tile of one domain, read from a tile list; the domain table carries the
// geometry, the collision constants and the storage scales of each domain.
// Threads map one-to-one onto sites with x fastest.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <type_traits>

#include "lattice.hpp"

namespace lb2p {

struct Geom {
    int nx, ny, nz;
    long long N;   // sites of the domain
    long long S;   // component stride of the packed arrays
};

// Constants of the collision (one domain).
struct Coef {
    double gamma, kappa;
    double c0sq;          // c_s^2(rho0)
    double Wk[8];         // W_k = w_k(c0^2), reference shell weights
    EosParams eos;
    double cheb_gamma;    // extrapolation 2/(2 - b) of the Chebyshev solver
    // c_s^2 and p at the domain's reference density rho_ref (DevScale): the
    // per-step planes hold p and c_s^2 = p/rho as deviations from these
    double cref, pref;
};

// Population storage codecs.  FP64 storage holds n_i itself.  The FP32,
// BF16 and FP16 forms hold d_i = n_i - o_i, the deviation from the rest
// equilibrium of the site that wrote the value (BF16/FP16 scaled per shell
// by the reference weight, d_i / W_k).  That site keeps a record of its
// density, rec = fp16(rho - rho_ref), beside the populations, and
// o_i = P_k(rec) with P_k a cubic fitted on the host to w_k(c_s^2(rho)) rho
// (Sec. III weights) over the domain's density range, evaluated in FP32.
// Writer and reader evaluate the same P_k on the same record, so the offsets
// agree exactly and n_i = o_i + d_i holds as a sum of two exact numbers; the
// fit only decides how small the stored deviation is.  What remains is the
// velocity and non-equilibrium part, small next to o_i.  Readers never form
// n_i in the storage precision: sums over velocities (item 1, the mass
// balance of the collision) add o_i and d_i in FP64, and the collision
// computes the deviation it stores in FP64.
struct DevScale {
    float off[8];       // w_k(c_s^2(rho_ref)) rho_ref
    float scl[8];       // W_k
    float inv[8];       // 1 / W_k
    float rref;         // rho_ref
    float pc[8][4];     // P_k(d) = pc[k][0] + d (pc[k][1] + d (pc[k][2] + d pc[k][3]))
};

struct Domain {
    Geom g;
    long long off;   // first site of the domain in the packed arrays
    Coef cf;
    DevScale ds;
};

// One block's work: a tile of a domain (dom < 0: padding, the block exits).
struct Tile {
    int dom, x0, y0, z0;
    int len;    // planes (3D) or rows (2D) marched by the solve kernel; sites of a linear tile
    int slot;   // 2D solve strips: the block's residual slot (see block_max_part)
    int lin;    // site kernels: 1 = the block covers sites x0 .. x0+len-1 of the domain in index order
    int pad2;
};

template <class S>
struct Codec;

// dev(v, ...): the value's deviation from its offset (the value itself for
// FP64); put(d, ...): the stored form of deviation d.
template <>
struct Codec<double> {
    static constexpr bool kLocal = false;
    __device__ static inline double dev(double v, const DevScale&, int) { return v; }
    __device__ static inline double put(double d, const DevScale&, int) { return d; }
};
// BF16/FP16 store the deviation scaled by 1/W_k (formed in FP32: the FP32
// rounding is far below the format's, and FP32 -> BF16/FP16 is one
// conversion instruction where FP64 -> FP16 is a long sequence); FP32
// stores it unscaled (its exponent range needs no scale).
template <class S>
struct DevCodec {
    static constexpr bool kLocal = true;
    __device__ static inline float dev(S v, const DevScale& s, int k) { return static_cast<float>(v) * s.scl[k]; }
    __device__ static inline S put(double d, const DevScale& s, int k)
    {
        return static_cast<S>(static_cast<float>(d) * s.inv[k]);
    }
};
template <>
struct Codec<float> {
    static constexpr bool kLocal = true;
    __device__ static inline float dev(float v, const DevScale&, int) { return v; }
    __device__ static inline float put(double d, const DevScale&, int) { return static_cast<float>(d); }
};
template <>
struct Codec<_Float16> : DevCodec<_Float16> {};
template <>
struct Codec<__bf16> : DevCodec<__bf16> {};

// The rest population (c = 0) is kept apart from the moving ones, at higher
// precision: FP64 beside FP64/FP32 moving populations, FP32 beside BF16/FP16.
// The collision sets it from the site's mass balance (the collision invariant
// sum_i Delta_i = 0 of Sec. VI), so it absorbs the rounding of the stored
// moving populations and the lattice mass stays conserved to the rounding of
// that plane alone.  Buffer layout: rest plane [S] of RestOf<S>::T, padded
// to 256 bytes, then the moving planes i = 1..Q-1 as [Q-1][S] of S.
template <class S>
struct RestOf {
    using T = double;
};
template <>
struct RestOf<__bf16> {
    using T = float;
};
template <>
struct RestOf<_Float16> {
    using T = float;
};

template <class S>
__host__ __device__ inline long long eq_offset_bytes(long long St)
{
    return (St * (long long)sizeof(typename RestOf<S>::T) + 255) / 256 * 256;
}
// After the rest plane: for the deviation forms (FP32, BF16, FP16) the
// density record of the site that wrote each value (fp16 [S]), then the
// moving planes.
template <class S>
__host__ __device__ inline long long moving_offset_bytes(long long St)
{
    return eq_offset_bytes<S>(St) + (Codec<S>::kLocal ? (St * 2 + 255) / 256 * 256 : 0);
}
template <class S>
__device__ inline _Float16* eq_plane(S* A, long long St)
{
    return reinterpret_cast<_Float16*>(reinterpret_cast<char*>(A) + eq_offset_bytes<S>(St));
}
template <class S>
__device__ inline const _Float16* eq_plane(const S* A, long long St)
{
    return reinterpret_cast<const _Float16*>(reinterpret_cast<const char*>(A) + eq_offset_bytes<S>(St));
}

template <class S>
__device__ inline typename RestOf<S>::T* rest_plane(S* A)
{
    return reinterpret_cast<typename RestOf<S>::T*>(A);
}
template <class S>
__device__ inline const typename RestOf<S>::T* rest_plane(const S* A)
{
    return reinterpret_cast<const typename RestOf<S>::T*>(A);
}
// Moving population i (1..Q-1) of site s: moving_planes(A, St)[(i-1)*St + s].
template <class S>
__device__ inline S* moving_planes(S* A, long long St)
{
    return reinterpret_cast<S*>(reinterpret_cast<char*>(A) + moving_offset_bytes<S>(St));
}
template <class S>
__device__ inline const S* moving_planes(const S* A, long long St)
{
    return reinterpret_cast<const S*>(reinterpret_cast<const char*>(A) + moving_offset_bytes<S>(St));
}

// Number of velocities in shell k.
template <int Q>
__host__ __device__ constexpr int kShellSize(int k)
{
    return Q == 59 ? kD3Q59.shell_size[k] : kD2Q21.shell_size[k];
}

// Density record of a site and the offset of a value of shell k it wrote.
__device__ __forceinline__ _Float16 density_record(const DevScale& ds, float rho)
{
    return static_cast<_Float16>(rho - ds.rref);
}
__device__ __forceinline__ float rest_offset(const DevScale& ds, int k, _Float16 rec)
{
    const float d = static_cast<float>(rec);
    return fmaf(d, fmaf(d, fmaf(d, ds.pc[k][3], ds.pc[k][2]), ds.pc[k][1]), ds.pc[k][0]);
}

__device__ __forceinline__ int wrap(int v, int n)
{
    v += (v < 0) ? n : 0;
    v -= (v >= n) ? n : 0;
    return v;
}

__device__ __forceinline__ long long sidx(const Geom& g, int x, int y, int z)
{
    return (long long)x + (long long)g.nx * ((long long)y + (long long)g.ny * z);
}

__device__ __forceinline__ long long nbr(const Geom& g, int x, int y, int z, int dx, int dy, int dz)
{
    return sidx(g, wrap(x + dx, g.nx), wrap(y + dy, g.ny), wrap(z + dz, g.nz));
}

// Where this thread works: its domain and site.  `ok` is false for threads
// past the edge of a ragged tile; `dom` < 0 marks a padding block.
struct Where {
    int dom;
    int x, y, z;
    bool ok;
};

// The site of this thread: a bx x by patch of a plane at (x0, y0, z0), or,
// for a linear tile, site x0 + (thread index) in the domain's index order
// x + nx (y + ny z), so that no lane of a narrow domain's tile idles.
__device__ __forceinline__ Where locate(const Domain* __restrict__ tab, const Tile* __restrict__ tiles)
{
    const Tile t = tiles[blockIdx.x];
    Where w;
    w.dom = t.dom;
    w.ok = false;
    if (t.lin) {
        const int lid = (int)(threadIdx.x + blockDim.x * threadIdx.y);
        w.x = 0; w.y = 0; w.z = 0;
        if (t.dom >= 0 && lid < t.len) {
            const Geom& g = tab[t.dom].g;
            const int i = t.x0 + lid;
            const int row = i / g.nx;
            w.x = i - row * g.nx;
            w.z = row / g.ny;
            w.y = row - w.z * g.ny;
            w.ok = true;
        }
        return w;
    }
    w.x = t.x0 + threadIdx.x;
    w.y = t.y0 + threadIdx.y;
    w.z = t.z0;
    if (t.dom >= 0) {
        const Geom& g = tab[t.dom].g;
        w.ok = w.x < g.nx && w.y < g.ny;
    }
    return w;
}

// Neighbours at -2, -1, +1, +2 along each axis of one site, as offsets from
// its index inside the domain (periodic wrap taken once per thread).  Site
// indices inside a domain fit 32 bits, and so do the byte offsets of one
// component plane of a domain (the host limits the domain size), so every
// access below is a uniform component base plus a 32-bit byte offset.
struct Nb2 {
    unsigned i0;
    int o[3][4];
};

__device__ __forceinline__ Nb2 make_nb2(const Geom& g, int x, int y, int z)
{
    Nb2 nb;
    nb.i0 = (unsigned)x + (unsigned)g.nx * ((unsigned)y + (unsigned)g.ny * (unsigned)z);
    const int sx = 1, sy = g.nx, sz = g.nx * g.ny;
    const int d[4] = {-2, -1, 1, 2};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        nb.o[0][k] = (wrap(x + d[k], g.nx) - x) * sx;
        nb.o[1][k] = (wrap(y + d[k], g.ny) - y) * sy;
        nb.o[2][k] = g.nz > 1 ? (wrap(z + d[k], g.nz) - z) * sz : 0;
    }
    return nb;
}

template <class R>
__device__ __forceinline__ R ldo(const R* base, unsigned i)
{
    return *reinterpret_cast<const R*>(reinterpret_cast<const char*>(base) + i * (unsigned)sizeof(R));
}
template <class R>
__device__ __forceinline__ void sto(R* base, unsigned i, R v)
{
    *reinterpret_cast<R*>(reinterpret_cast<char*>(base) + i * (unsigned)sizeof(R)) = v;
}

// Offsets of the pull sources r - c_i (|c_i| components up to 4) from a
// site's index inside the domain, periodic wrap taken once per axis.
struct NbP {
    unsigned i0;
    int ox[9], oy[9], oz[9];   // index d + 4
    __device__ __forceinline__ unsigned at(int dx, int dy, int dz) const
    {
        return i0 + (unsigned)(ox[dx + 4] + oy[dy + 4] + oz[dz + 4]);
    }
};

__device__ __forceinline__ NbP make_nbp(const Geom& g, int x, int y, int z)
{
    NbP nb;
    nb.i0 = (unsigned)x + (unsigned)g.nx * ((unsigned)y + (unsigned)g.ny * (unsigned)z);
    const int sy = g.nx, sz = g.nx * g.ny;
#pragma unroll
    for (int d = -4; d <= 4; ++d) {
        nb.ox[d + 4] = wrap(x + d, g.nx) - x;
        nb.oy[d + 4] = (wrap(y + d, g.ny) - y) * sy;
        nb.oz[d + 4] = g.nz > 1 ? (wrap(z + d, g.nz) - z) * sz : 0;
    }
    return nb;
}

// D1 (Sec. IV B) of one component plane F (domain base) along axis a.
template <class R>
__device__ __forceinline__ R d1_nb(const R* F, const Nb2& nb, int a)
{
    return d1<R>(ldo(F, nb.i0 + nb.o[a][0]), ldo(F, nb.i0 + nb.o[a][1]), ldo(F, nb.i0 + nb.o[a][2]),
                 ldo(F, nb.i0 + nb.o[a][3]));
}

// Symmetric rank-2 component index (xx yy zz xy xz yz / xx yy xy).
template <int D>
__host__ __device__ constexpr int sym2(int a, int b)
{
    if (a == b) return a;
    int lo = a < b ? a : b, hi = a < b ? b : a;
    if (D == 2) return 2;
    return lo == 0 ? (hi == 1 ? 3 : 4) : 5;
}

// Symmetric rank-3 component index.
// 3D: xxx yyy zzz xxy xxz xyy xzz yyz yzz xyz ; 2D: xxx yyy xxy xyy.
template <int D>
__host__ __device__ constexpr int sym3(int a, int b, int c)
{
    int n[3] = {0, 0, 0};
    n[a]++; n[b]++; n[c]++;
    if (D == 2) {
        if (n[0] == 3) return 0;
        if (n[1] == 3) return 1;
        if (n[0] == 2) return 2;
        return 3;
    }
    if (n[0] == 3) return 0;
    if (n[1] == 3) return 1;
    if (n[2] == 3) return 2;
    if (n[0] == 2 && n[1] == 1) return 3;
    if (n[0] == 2 && n[2] == 1) return 4;
    if (n[1] == 2 && n[0] == 1) return 5;
    if (n[2] == 2 && n[0] == 1) return 6;
    if (n[1] == 2 && n[2] == 1) return 7;
    if (n[2] == 2 && n[1] == 1) return 8;
    return 9;
}

// Wavefront (64-lane) reductions.
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block maxima (stop rule of Sec. IX: max|j0'| and the residual of a pass).
// Each block stores its maximum to a slot of its own; k_reduce_max then
// reduces each domain's slots.  No two blocks touch one address: tens of
// thousands of atomics (or coherent loads) on one address serialise across
// the XCDs.  Slots are in domain order: a launch grid of n blocks (a multiple
// of 8) runs tile (b % 8) * (n / 8) + b / 8 of the domain-ordered list at
// workgroup b (the XCD deal), so that is the block's slot, unless the tile
// list was reordered and the tile names its slot (slot >= 0).
// NaN is stored as +inf so that it is never lost.  Every thread of the block
// must call it.
__device__ inline void block_max_part(double* part, double v, int slot = -1)
{
    __shared__ double red[16];
    if (v != v) v = __longlong_as_double(0x7ff0000000000000LL);
    v = wave_max(v);
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int lane = tid & 63, wid = tid >> 6;
    const int nw = (blockDim.x * blockDim.y + 63) >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    if (tid == 0) {
        double m = red[0];
        for (int k = 1; k < nw; ++k) m = fmax(m, red[k]);
        const unsigned n = gridDim.x, b = blockIdx.x;
        part[slot >= 0 ? (unsigned)slot : (b % 8u) * (n / 8u) + b / 8u] = m;
    }
}

// One block per domain: out[d * stride] = bits of max over part[range[d] ..
// range[d+1]).  Domains already done (done_at >= 0) are left alone: their
// blocks skipped the pass and wrote nothing.
__global__ void __launch_bounds__(256) k_reduce_max(const double* __restrict__ part,
                                                    const int* __restrict__ range,
                                                    unsigned long long* __restrict__ out, long long stride,
                                                    const int* __restrict__ done_at)
{
    const int d = blockIdx.x;
    if (done_at && *((volatile const int*)(done_at + d)) >= 0) return;
    double m = 0.0;
    for (int i = range[d] + threadIdx.x; i < range[d + 1]; i += blockDim.x) m = fmax(m, part[i]);
    m = wave_max(m);
    __shared__ double red[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = red[0];
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) t = fmax(t, red[k]);
        out[(long long)d * stride] = (unsigned long long)__double_as_longlong(t);
    }
}

// The per-step planes of one site (item 1's EOS, fixed during the solve):
// [0] p - p_ref, [1] P1 = p - rho p', [2] 1/rho, [3] c_s^2 - c_s^2(rho_ref).
// p and c_s^2 are evaluated in FP64 from the FP64 density and kept as
// deviations from their reference values: the closure differentiates them,
// and their deviations carry the field precision of their own size.  P1 and
// 1/rho only scale other terms.
template <class R>
__device__ __forceinline__ void store_step_planes(const Coef& cf, R* at, long long St, double r64, R r, R inv)
{
    const double cs2 = eos_cs2<double>(cf.eos, r64);
    const R psi = eos_psi<R>(cf.eos, r);
    at[0] = R(r64 * cs2 - cf.pref);
    at[St] = -r * r * R(cs2) * psi;
    at[2 * St] = inv;
    at[3 * St] = R(cs2 - cf.cref);
}

// ---------------------------------------------------------------------------
// Initial populations: n_i(r) = n_eq(rho(r), u(r)) with local weights,
// written pre-shifted so that the first pull returns them.  Evaluated in FP64
// from the caller's FP64 density (u in the field precision): only the
// storage rounds.
// ---------------------------------------------------------------------------
template <int Q, class R, class S>
__global__ void __launch_bounds__(256) k_init(const Domain* __restrict__ tab, const Tile* __restrict__ tiles,
                                              const double* __restrict__ rho, const R* __restrict__ u,
                                              S* __restrict__ A)
{
    using L = Lattice<Q>;
    const Where w = locate(tab, tiles);
    if (!w.ok) return;
    const Domain& dm = tab[w.dom];
    const Geom g = dm.g;
    const long long o = dm.off, St = g.S;
    const NbP nb = make_nbp(g, w.x, w.y, w.z);
    const unsigned i0 = nb.i0;
    const double r = ldo(rho + o, i0);
    double uu[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < L::D; ++a) uu[a] = (double)ldo(u + o + a * St, i0);
    const double cs2 = eos_cs2<double>(dm.cf.eos, r);
    double wl[8];
    shell_weights<Q, double>(cs2, wl);
    const double inv = 1.0 / cs2;
    const double a0 = 1.0 - (uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2]) * 0.5 * inv;
    using T0 = typename RestOf<S>::T;
    S* const mv = moving_planes(A, St) + o;
    if constexpr (Codec<S>::kLocal) sto(eq_plane(A, St) + o, i0, density_record(dm.ds, float(r)));
    double moved = 0.0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const double uc = uu[0] * L::cx(i) + uu[1] * L::cy(i) + uu[2] * L::cz(i);
        const double neq = wl[L::shell(i)] * r * (a0 + uc * inv + 0.5 * uc * uc * inv * inv);
        const unsigned slot = nb.at(-L::cx(i), -L::cy(i), -L::cz(i));
        if constexpr (Codec<S>::kLocal) {
            // the record the slot's own thread writes
            const float off =
                rest_offset(dm.ds, L::shell(i), density_record(dm.ds, float(ldo(rho + o, slot))));
            const S e = Codec<S>::put(neq - (double)off, dm.ds, L::shell(i));
            sto(mv + (size_t)(i - 1) * St, slot, e);
            moved += (double)off + (double)Codec<S>::dev(e, dm.ds, L::shell(i));
        } else {
            const S e = Codec<S>::put(S(neq), dm.ds, L::shell(i));
            sto(mv + (size_t)(i - 1) * St, slot, e);
            moved += (double)e;
        }
    }
    // rest population: the site's density minus the stored moving ones
    sto(rest_plane(A) + o, i0, T0(r - moved));
}

// Pulled population i of a site as an FP64 number: o_i + d_i for the
// deviation forms (both terms exact in FP64), n_i for FP64 storage.
template <class S>
__device__ __forceinline__ double pulled(const S* mv, const _Float16* eqa, const DevScale& ds, int k,
                                         unsigned src)
{
    const S b = ldo(mv, src);
    if constexpr (Codec<S>::kLocal)
        return (double)rest_offset(ds, k, ldo(eqa, src)) + (double)Codec<S>::dev(b, ds, k);
    else
        return (double)b;
}

// ---------------------------------------------------------------------------
// Item 1: rho = sum_i n_i, j0 = sum_i n_i c_i of the pulled populations, and
// FP64 block partial sums of mass and momentum plus a non-finite flag.  Both
// sums run in FP64, so rho and j0 carry only the rounding of their own
// precision (the FP32 rounding of j0 next to its own size, not next to the
// populations').
// ---------------------------------------------------------------------------
template <int Q, class R, class S>
__global__ void __launch_bounds__(256) k_moments(const Domain* __restrict__ tab,
                                                 const Tile* __restrict__ tiles,
                                                 const S* __restrict__ A, R* __restrict__ rho,
                                                 R* __restrict__ j0, double* __restrict__ partial,
                                                 int* __restrict__ flags, double* __restrict__ mass,
                                                 R* __restrict__ pf)
{
    using L = Lattice<Q>;
    const Where w = locate(tab, tiles);
    if (w.dom < 0) {   // padding block: empty partial sums
        const int tid = threadIdx.x + blockDim.x * threadIdx.y;
        if (tid < 4) partial[4 * (long long)blockIdx.x + tid] = 0.0;
        return;
    }
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    if (w.ok) {
        const Domain& dm = tab[w.dom];
        const Geom g = dm.g;
        const long long o = dm.off, St = g.S;
        const NbP nb = make_nbp(g, w.x, w.y, w.z);
        const unsigned i0 = nb.i0;
        // the density is the exact sum of the stored values (the conserved
        // mass), kept for the collision's mass balance
        double racc = (double)ldo(rest_plane(A) + o, i0);
        double jx = 0.0, jy = 0.0, jz = 0.0;
        const S* const mv = moving_planes(A, St) + o;
        const _Float16* const eqa = eq_plane(A, St) + o;
#pragma unroll
        for (int p = 0; p < L::NPAIR; ++p) {
            const int ip = 2 * p + 1, im = 2 * p + 2, k = L::shell(ip);
            // the antipodal pair (c, -c): its sum enters rho, its difference j0
            const double vp = pulled(mv + (size_t)(ip - 1) * St, eqa, dm.ds, k,
                                     nb.at(-L::cx(ip), -L::cy(ip), -L::cz(ip)));
            const double vm = pulled(mv + (size_t)(im - 1) * St, eqa, dm.ds, k,
                                     nb.at(-L::cx(im), -L::cy(im), -L::cz(im)));
            racc += vp + vm;
            const double dv = vp - vm;
            if (L::cx(ip)) jx += L::cx(ip) * dv;
            if (L::cy(ip)) jy += L::cy(ip) * dv;
            if (L::cz(ip)) jz += L::cz(ip) * dv;
        }
        const R r = R(racc);
        sto(mass + o, i0, racc);
        sto(rho + o, i0, r);
        // item 1's EOS, fixed for the rest of the step (the per-step planes)
        if (pf) store_step_planes<R>(dm.cf, pf + o + i0, St, racc, r, R(1) / r);
        sto(j0 + o, i0, R(jx));
        sto(j0 + o + St, i0, R(jy));
        if (L::D == 3) sto(j0 + o + 2 * St, i0, R(jz));
        if (!(r > R(0) && r < R(1e30))) atomicOr(flags, 1);
        m[0] = racc; m[1] = jx; m[2] = jy; m[3] = jz;
    }
    __shared__ double red[4][16];
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int lane = tid & 63, wid = tid >> 6;
    const int nw = (blockDim.x * blockDim.y + 63) >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double v = wave_sum(m[k]);
        if (lane == 0) red[k][wid] = v;
    }
    __syncthreads();
    if (tid < 4) {
        double acc = 0.0;
        for (int q = 0; q < nw; ++q) acc += red[tid][q];
        partial[4 * (long long)blockIdx.x + tid] = acc;
    }
}

// Which j~ buffer holds each domain's final iterate, and its pass count.
struct SolveInfo {
    int final_buf;
    int iters;
    int converged;
    int pad;
};

// Stop-rule bookkeeping of the j~ iteration, one set per domain:
// res[dom*stride + k] = bits of max|j~new - j~| of pass k, jscale[dom] =
// bits of max|j0'|, done_at[dom] = pass at which the rule held (or -1).
struct IterCtl {
    unsigned long long* res;
    unsigned long long* jscale;
    int* done_at;
    int stride;
    double tol;                  // < 0: never stop early (fixed count)
    const double* omega;         // Chebyshev weights [dom*stride + pass], or null (plain)
    double* part;                // per-block maxima (block_max_part)
};

__device__ __forceinline__ bool iter_skip(const IterCtl& c, int dom, int it)
{
    if (*((volatile int*)(c.done_at + dom)) >= 0) return true;
    if (it > 0 && c.tol >= 0.0) {
        const double r = __longlong_as_double((long long)c.res[(long long)dom * c.stride + it - 1]);
        const double thr = c.tol * __longlong_as_double((long long)c.jscale[dom]);
        if (r <= thr) {
            *((volatile int*)(c.done_at + dom)) = it;
            return true;
        }
    }
    return false;
}

// ---------------------------------------------------------------------------
// Item 4: q_ab = (p - rho dp/drho) d_ab d_g u_g + p (d_b u_a + d_a u_b),
// derivatives with the stencil of Sec. IV B.  q is symmetric.
// ---------------------------------------------------------------------------
template <int Q, class R>
__global__ void __launch_bounds__(256) k_iter_q(const Domain* __restrict__ tab,
                                                const Tile* __restrict__ tiles, IterCtl ic, int it,
                                                const R* __restrict__ pf, const R* __restrict__ u,
                                                R* __restrict__ q)
{
    using L = Lattice<Q>;
    constexpr int D = L::D;
    const Where w = locate(tab, tiles);
    if (w.dom < 0 || iter_skip(ic, w.dom, it) || !w.ok) return;
    const Domain& dm = tab[w.dom];
    const long long o = dm.off, St = dm.g.S;
    const Nb2 nb = make_nb2(dm.g, w.x, w.y, w.z);
    R G[3][3];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) G[a][b] = d1_nb<R>(u + o + b * St, nb, a);
    R trG = R(0);
#pragma unroll
    for (int a = 0; a < D; ++a) trG += G[a][a];
    const R p = R(dm.cf.pref) + ldo(pf + o, nb.i0), P1 = ldo(pf + o + St, nb.i0);
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a; b < D; ++b) {
            R v = p * (G[a][b] + G[b][a]);
            if (a == b) v += P1 * trG;
            sto(q + o + sym2<D>(a, b) * St, nb.i0, v);
        }
}

// Next iterate from the map's value g = G(x_k) at one site.  Plain fixed
// point (Sec. IX): x_{k+1} = g.  Chebyshev semi-iteration on the same map
// (its linear part is similar to a symmetric positive semi-definite operator,
// so the spectrum is real in [0, b]): with gamma = 2/(2-b),
// x_{k+1} = x_{k-1} + omega_k (gamma g + (1-gamma) x_k - x_{k-1}), omega_0 = 1.
// The stop rule tests |g - x_k| in both cases.
template <class R>
__device__ __forceinline__ R next_iterate(R g, R xk, R xkm1, R omega, R gam, bool first)
{
    const R y = gam * g + (R(1) - gam) * xk;
    return first ? y : xkm1 + omega * (y - xkm1);
}

// ---------------------------------------------------------------------------
// Item 5: j~new_a = -(1/12) d_b q_ab; item 6 residual; item 3 of the next
// pass: u = (j0' + j~new)/rho.  With the Chebyshev solver jt_prev holds
// x_{k-1} and is overwritten in place by x_{k+1} (jt_prev == jt_new).
// ---------------------------------------------------------------------------
template <int Q, class R>
__global__ void __launch_bounds__(256) k_iter_jt(const Domain* __restrict__ tab,
                                                 const Tile* __restrict__ tiles, IterCtl ic, int it,
                                                 const R* __restrict__ pf, const R* __restrict__ q,
                                                 const R* __restrict__ j0p,
                                                 const R* __restrict__ jt_old,
                                                 R* jt_new, R* __restrict__ u)
{
    using L = Lattice<Q>;
    constexpr int D = L::D;
    const Where w = locate(tab, tiles);
    if (w.dom < 0) return;
    if (*((volatile int*)(ic.done_at + w.dom)) >= 0) return;   // uniform per block
    double dmax = 0.0, dsum = 0.0;   // dsum only carries a NaN (fmax drops it)
    if (w.ok) {
        const Domain& dm = tab[w.dom];
        const long long o = dm.off, St = dm.g.S;
        const Nb2 nb = make_nb2(dm.g, w.x, w.y, w.z);
        const unsigned i0 = nb.i0;
        const R inv = ldo(pf + o + 2 * St, i0);
        const bool cheb = ic.omega != nullptr;
        const R omega = cheb ? R(ic.omega[(long long)w.dom * ic.stride + it]) : R(1);
        const R gam = cheb ? R(dm.cf.cheb_gamma) : R(1);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            R acc = R(0);
#pragma unroll
            for (int b = 0; b < D; ++b) acc += d1_nb<R>(q + o + sym2<D>(a, b) * St, nb, b);
            const R gv = -acc * R(1.0 / 12.0);
            const R xk = ldo(jt_old + o + a * St, i0);
            const double d = fabs((double)(gv - xk));
            dmax = fmax(dmax, d);
            dsum += d;
            R xn = gv;
            if (cheb) xn = next_iterate<R>(gv, xk, it > 0 ? ldo<R>(jt_new + o + a * St, i0) : R(0), omega, gam, it == 0);
            sto(jt_new + o + a * St, i0, xn);
            sto(u + o + a * St, i0, (ldo(j0p + o + a * St, i0) + xn) * inv);
        }
    }
    block_max_part(ic.part, dsum == dsum ? dmax : dsum);
}

// One thread per domain.
// gated = 1: launched ahead of the host's check of the stop rule, it does
// nothing unless that check found every domain done (go = 1).  gated = 0: it
// runs and sets go = 1 for the kernels after it.
__global__ void k_iter_finish(IterCtl ic, int launched, int ndom, SolveInfo* info, int* nconv, int* go,
                              int gated)
{
    if (gated) {
        if (*go == 0) return;
    } else if (blockIdx.x == 0 && threadIdx.x == 0) {
        *go = 1;
    }
    const int dom = blockIdx.x * blockDim.x + threadIdx.x;
    if (dom >= ndom) return;
    int d = *((volatile int*)(ic.done_at + dom));
    if (d < 0 && ic.tol >= 0.0 && launched > 0) {
        // stop rule on the last launched pass (no later pass tested it)
        const double r = __longlong_as_double((long long)ic.res[(long long)dom * ic.stride + launched - 1]);
        const double thr = ic.tol * __longlong_as_double((long long)ic.jscale[dom]);
        if (r <= thr) d = launched;
    }
    const int iters = d >= 0 ? d : launched;
    info[dom].iters = iters;
    info[dom].final_buf = iters & 1;
    info[dom].converged = d >= 0 || ic.tol < 0.0;
    if (!(d >= 0 || ic.tol < 0.0)) atomicAdd(nconv, 1);
}

// After `launched` passes: apply the stop rule to the last pass of every
// domain still iterating (as the next pass would), and report for the host's
// early exit the number of domains whose rule has held (out[0]) and the
// largest pass count at which it held (out[1]); go = 1 when that is every
// domain, else 0 (the kernels that follow a solve run only when go = 1).
__global__ void k_check_done(IterCtl ic, int launched, int ndom, int* out, int* go)
{
    __shared__ int cnt, last;
    if (threadIdx.x == 0) { cnt = 0; last = 0; }
    __syncthreads();
    for (int d = threadIdx.x; d < ndom; d += blockDim.x) {
        int da = ic.done_at[d];
        if (da < 0 && launched > 0) {
            const double r = __longlong_as_double((long long)ic.res[(long long)d * ic.stride + launched - 1]);
            const double thr = ic.tol * __longlong_as_double((long long)ic.jscale[d]);
            if (r <= thr) {
                da = launched;
                ic.done_at[d] = da;
            }
        }
        if (da >= 0) {
            atomicAdd(&cnt, 1);
            atomicMax(&last, da);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = cnt;
        out[1] = last;
        *go = cnt >= ndom ? 1 : 0;
    }
}

// ---------------------------------------------------------------------------
// Item 11 per velocity and item 12: pull n_i(r), collide with
// Delta^bulk + Delta^int + Delta^corr and store n*_i(r) in the other buffer.
// Velocities come in antipodal pairs; each pair shares its even part.
// The deviation forms store n*_i - o_i: with n*_i = g n_i + (1-g) n_eq_i +
// Delta_i, that is g (n_i - o_i) + (1-g) (w_k rho - o_i) + (1-g) w_k rho
// (u.c/c_s^2 + ...) + Delta_i, whose O(1) part (1-g)(w_k rho - o_i) is formed
// in FP64 once per shell, so the stored deviation carries no rounding of
// the O(1) equilibrium.
// ---------------------------------------------------------------------------
template <int Q, class R, class S, bool ANY_PULL>
__global__ void __launch_bounds__(256) k_collide(const Domain* __restrict__ tab,
                                                 const Tile* __restrict__ tiles,
                                                 const SolveInfo* __restrict__ info,
                                                 const S* __restrict__ A, S* __restrict__ B,
                                                 const R* __restrict__ u,
                                                 const R* __restrict__ f, const R* __restrict__ jtA,
                                                 const R* __restrict__ jtB, const R* __restrict__ Sig,
                                                 const R* __restrict__ Xi, const double* __restrict__ mass,
                                                 const int* __restrict__ go)
{
    // multiply-adds fused only as written in each expression, so that both
    // instantiations round a gamma = 0 site identically
#pragma clang fp contract(on)
    if (*go == 0) return;   // the solve is not finished (launched ahead of the host's check)
    // Precision.  The O(1) parts -- c_s^2, the local weights and the
    // per-shell rest part (1-g)(w_k rho - o_k) -- are FP64 in every form.
    // The per-velocity Hermite terms (E) are FP64 beside FP64 and FP32
    // storage: at an interface Xi' and Sigma are large next to the flow (Xi'
    // holds p d(c_s^2), of order 1e-2 where u is 1e-4), their terms leave no
    // first moment only in exact arithmetic, and FP32 rounding of them would
    // feed the momentum of every step (the arithmetic is then a few percent
    // of this memory-bound kernel's time).  Beside BF16/FP16 storage with
    // FP32 fields they are FP32: the stored deviation rounds each of those
    // terms at 2^-9 (BF16) or 2^-12 (FP16) of its size, 2^15 and 2^12 times
    // the FP32 rounding, and in FP64 this kernel would be bound by FP64
    // issue rather than by its 230 bytes per site.
    using E = typename std::conditional<sizeof(S) == 2 && sizeof(R) == 4, float, double>::type;
    using L = Lattice<Q>;
    constexpr int D = L::D;
    const Where w = locate(tab, tiles);
    if (!w.ok) return;
    const Domain& dm = tab[w.dom];
    const Geom g = dm.g;
    const long long o = dm.off, St = g.S;
    const NbP nb = make_nbp(g, w.x, w.y, w.z);
    const unsigned i0 = nb.i0;
    const R* jt = (info[w.dom].final_buf ? jtB : jtA) + o;

    const double r64 = ldo(mass + o, i0);   // the exact pulled mass of item 1
    E us[3] = {E(0), E(0), E(0)}, fs[3] = {E(0), E(0), E(0)}, js[3] = {E(0), E(0), E(0)};
#pragma unroll
    for (int a = 0; a < D; ++a) {
        us[a] = ldo(u + o + a * St, i0);
        fs[a] = ldo(f + o + a * St, i0);
        js[a] = ldo(jt + a * St, i0);
    }
    E Sg[6], Xp[10];
#pragma unroll
    for (int k = 0; k < L::NSIG; ++k) Sg[k] = ldo(Sig + o + k * St, i0);
#pragma unroll
    for (int k = 0; k < L::NXI; ++k) Xp[k] = ldo(Xi + o + k * St, i0);

    const E gm = E(dm.cf.gamma);
    const E c0 = E(dm.cf.c0sq);
    const E ic0 = E(1) / c0;
    // n_eq pieces (local weights), (1-g) w_k rho in FP64
    const double cs2 = eos_cs2<double>(dm.cf.eos, r64);
    double wl64[8];
    shell_weights<Q, double>(cs2, wl64);
    const double omg64 = 1.0 - dm.cf.gamma;   // weight of n_eq
#pragma unroll
    for (int k = 0; k < L::NSHELL; ++k) wl64[k] *= omg64 * r64;
    E wl[8];
#pragma unroll
    for (int k = 0; k < L::NSHELL; ++k) wl[k] = E(wl64[k]);
    const E ics = E(1.0 / cs2);
    const E uu = us[0] * us[0] + us[1] * us[1] + us[2] * us[2];
    const E a0m = -E(0.5) * uu * ics;   // a0 - 1
    const E a1 = ics;
    const E a2 = E(0.5) * ics * ics;
    // Delta^corr pieces: W_k [ b.c + c.S'.c + s0 + X'(c,c,c) ]
    E trS = E(0);
#pragma unroll
    for (int a = 0; a < D; ++a) trS += Sg[a];
    E v[3] = {E(0), E(0), E(0)};   // v_g = sum_a Xi'_aag
#pragma unroll
    for (int gg = 0; gg < D; ++gg)
#pragma unroll
        for (int a = 0; a < D; ++a) v[gg] += Xp[sym3<D>(a, a, gg)];
    const E kS = E(0.5) * ic0 * ic0;
    const E kX = ic0 * ic0 * ic0 / E(6);
    E bvec[3];
#pragma unroll
    for (int a = 0; a < D; ++a)
        bvec[a] = E(0.5) * (E(1) + gm) * ic0 * fs[a] + (gm - E(1)) * ic0 * js[a] - E(0.5) * ic0 * ic0 * v[a];
    const E s0 = -E(0.5) * ic0 * trS;

    // Moving velocities first; the rest population then takes what the
    // collision invariant sum_i Delta_i = 0 (Sec. VI) leaves for it,
    // n*_0 = n_0 + sum_{i>0} n_i - sum_{i>0} n*_i with the n*_i as stored, so
    // the site's mass is kept to the rounding of the rest plane.  With
    // gamma = 0 the bulk operator relaxes fully: n*_i = n_eq_i + Delta^int_i
    // + Delta^corr_i does not depend on n_i, the pulled populations are not
    // read at all, and the mass balance uses the exact pulled mass of item 1.
    // Otherwise n_i is pulled and n*_0 = n_0 - sum_{i>0} (n*_i - n_i).
    // Uniform per block; instantiated without the pulling path when no
    // domain of the launch has gamma != 0.
    const bool pull = ANY_PULL && dm.cf.gamma != 0.0;
    const S* const amv = moving_planes(A, St) + o;
    S* const bmv = moving_planes(B, St) + o;
    const _Float16* const eqa = eq_plane(A, St) + o;
    // Per shell: the offset of the values this site writes (its own record)
    // and the O(1) part of what it stores, (1-g)(w_k rho - o_k), which is
    // small only as a difference of two O(1) FP64 numbers
    float ownoff[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    E rest[8];
    double moved = 0.0;   // no pull: sum of n*_i (exact in FP64)
    if constexpr (Codec<S>::kLocal) {
        const _Float16 rec = density_record(dm.ds, float(r64));
        sto(eq_plane(B, St) + o, i0, rec);
#pragma unroll
        for (int k = 1; k < L::NSHELL; ++k) {
            ownoff[k] = rest_offset(dm.ds, k, rec);
            rest[k] = E(wl64[k] - omg64 * (double)ownoff[k]);
            moved += (double)kShellSize<Q>(k) * (double)ownoff[k];
        }
    } else {
#pragma unroll
        for (int k = 1; k < L::NSHELL; ++k) rest[k] = E(wl64[k]);
    }
    double dsum = 0.0;   // pull: sum of (n*_i - n_i)
#pragma unroll
    for (int p = 0; p < L::NPAIR; ++p) {
        const int ip = 2 * p + 1, im = 2 * p + 2;
        const int cxv = L::cx(ip), cyv = L::cy(ip), czv = L::cz(ip);
        const int k = L::shell(ip);
        const E cx = E(cxv), cy = E(cyv), cz = E(czv);
        const E uc = us[0] * cx + us[1] * cy + us[2] * cz;
        // c.Sigma.c
        E cSc = Sg[0] * cx * cx + Sg[1] * cy * cy;
        if (D == 3) {
            cSc += Sg[2] * cz * cz + E(2) * (Sg[3] * cx * cy + Sg[4] * cx * cz + Sg[5] * cy * cz);
        } else {
            cSc += E(2) * Sg[2] * cx * cy;
        }
        // Xi'(c,c,c)
        E cXc;
        if (D == 3) {
            cXc = Xp[0] * cx * cx * cx + Xp[1] * cy * cy * cy + Xp[2] * cz * cz * cz +
                  E(3) * (Xp[3] * cx * cx * cy + Xp[4] * cx * cx * cz + Xp[5] * cx * cy * cy +
                          Xp[6] * cx * cz * cz + Xp[7] * cy * cy * cz + Xp[8] * cy * cz * cz) +
                  E(6) * Xp[9] * cx * cy * cz;
        } else {
            cXc = Xp[0] * cx * cx * cx + Xp[1] * cy * cy * cy +
                  E(3) * (Xp[2] * cx * cx * cy + Xp[3] * cx * cy * cy);
        }
        const E bc = bvec[0] * cx + bvec[1] * cy + (D == 3 ? bvec[2] * cz : E(0));
        const E Wk = E(dm.cf.Wk[k]);
        const E even = rest[k] + wl[k] * (a0m + a2 * uc * uc) + Wk * (kS * cSc + s0);
        const E odd = wl[k] * a1 * uc + Wk * (bc + kX * cXc);
        // pulled n_i relative to this site's offset (the value itself for
        // FP64 storage), and its exact FP64 form for the mass balance
        E np = E(0), nm = E(0);
        double npx = 0.0, nmx = 0.0;
        if (pull) {
            const unsigned sp = nb.at(-cxv, -cyv, -czv), sm = nb.at(cxv, cyv, czv);
            const S bp = ldo(amv + (size_t)(ip - 1) * St, sp), bm = ldo(amv + (size_t)(im - 1) * St, sm);
            if constexpr (Codec<S>::kLocal) {
                const double dp0 = (double)rest_offset(dm.ds, k, ldo(eqa, sp)) - (double)ownoff[k];
                const double dm0 = (double)rest_offset(dm.ds, k, ldo(eqa, sm)) - (double)ownoff[k];
                npx = dp0 + (double)Codec<S>::dev(bp, dm.ds, k);
                nmx = dm0 + (double)Codec<S>::dev(bm, dm.ds, k);
            } else {
                npx = (double)bp;
                nmx = (double)bm;
            }
            np = E(npx);
            nm = E(nmx);
        }
        const S ep = Codec<S>::put(gm * np + even + odd, dm.ds, k);
        const S em = Codec<S>::put(gm * nm + even - odd, dm.ds, k);
        sto(bmv + (size_t)(ip - 1) * St, i0, ep);
        sto(bmv + (size_t)(im - 1) * St, i0, em);
        const double dp = (double)Codec<S>::dev(ep, dm.ds, k), dmm = (double)Codec<S>::dev(em, dm.ds, k);
        if (pull)
            dsum += (dp - npx) + (dmm - nmx);
        else
            moved += dp + dmm;
    }
    using T0 = typename RestOf<S>::T;
    if (pull)
        sto(rest_plane(B) + o, i0, T0((double)ldo(rest_plane(A) + o, i0) - dsum));
    else
        sto(rest_plane(B) + o, i0, T0(r64 - moved));
}

// Pre-collision populations of the current state as FP64 [Q][S].
template <int Q, class S>
__global__ void __launch_bounds__(256) k_export(const Domain* __restrict__ tab,
                                                const Tile* __restrict__ tiles,
                                                const S* __restrict__ A, double* __restrict__ out)
{
    using L = Lattice<Q>;
    const Where w = locate(tab, tiles);
    if (!w.ok) return;
    const Domain& dm = tab[w.dom];
    const Geom g = dm.g;
    const long long o = dm.off, St = g.S;
    const NbP nb = make_nbp(g, w.x, w.y, w.z);
    const unsigned i0 = nb.i0;
    const S* const mv = moving_planes(A, St) + o;
    const _Float16* const eqa = eq_plane(A, St) + o;
    sto(out + o, i0, (double)ldo(rest_plane(A) + o, i0));
#pragma unroll
    for (int i = 1; i < Q; ++i)
        sto(out + o + (size_t)i * St, i0,
            pulled(mv + (size_t)(i - 1) * St, eqa, dm.ds, L::shell(i), nb.at(-L::cx(i), -L::cy(i), -L::cz(i))));
}

template <int Q, class S>
__global__ void __launch_bounds__(256) k_import(const Domain* __restrict__ tab,
                                                const Tile* __restrict__ tiles,
                                                const double* __restrict__ in, S* __restrict__ A)
{
    using L = Lattice<Q>;
    const Where w = locate(tab, tiles);
    if (!w.ok) return;
    const Domain& dm = tab[w.dom];
    const Geom g = dm.g;
    const long long o = dm.off, St = g.S;
    const NbP nb = make_nbp(g, w.x, w.y, w.z);
    const unsigned i0 = nb.i0;
    S* const mv = moving_planes(A, St) + o;
    sto(rest_plane(A) + o, i0, (typename RestOf<S>::T)ldo(in + o, i0));
    // no density is at hand for the slots: every record is the reference
    // density's, until the first collision writes local ones
    const _Float16 eref = density_record(dm.ds, dm.ds.rref);
    if constexpr (Codec<S>::kLocal) sto(eq_plane(A, St) + o, i0, eref);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const double v = ldo(in + o + (size_t)i * St, i0);
        S e;
        if constexpr (Codec<S>::kLocal)
            e = Codec<S>::put(v - (double)rest_offset(dm.ds, L::shell(i), eref), dm.ds, L::shell(i));
        else
            e = Codec<S>::put(S(v), dm.ds, L::shell(i));
        sto(mv + (size_t)(i - 1) * St, nb.at(-L::cx(i), -L::cy(i), -L::cz(i)), e);
    }
}

// Small helpers.
__global__ void k_reset_ctl(unsigned long long* res, long long nres, unsigned long long* jscale,
                            int* done_at, int ndom, int* nconv, int* go)
{
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t < nres) res[t] = 0ull;
    if (t < ndom) {
        jscale[t] = 0ull;
        done_at[t] = -1;
    }
    if (t == 0 && nconv) *nconv = 0;
    if (t == 0) *go = 1;
}

// Deterministic sum of block partials [first, last) (one block).
__global__ void k_sum_partials(const double* __restrict__ partial, long long first, long long last,
                               double* out)
{
    __shared__ double red[4][16];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (long long b = first + threadIdx.x; b < last; b += blockDim.x)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] += partial[4 * b + k];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double v = wave_sum(acc[k]);
        if (lane == 0) red[k][wid] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += red[threadIdx.x][q];
        out[threadIdx.x] = t;
    }
}

template <class Rin, class Rout>
__global__ void k_convert(const Rin* __restrict__ in, Rout* __restrict__ out, long long n)
{
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t < n) out[t] = (Rout)in[t];
}

}  // namespace lb2p
