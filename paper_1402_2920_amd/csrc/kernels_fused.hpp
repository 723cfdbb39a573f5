// kernels_fused.hpp -- one kernel per pass of the correction-current
// iteration (Supplemental items 3-6), carried in velocity form: the z-march
// k_iter_fused3 for D3Q59 and the y-march k_iter_fused2 for D2Q21.
//
// The pass maps u_k = (j0' + x_k)/rho to u_{k+1} = (j0' + G(x_k))/rho, where
// G(x) = -(1/12) d_b q_ab depends on x only through u (item 4 builds q from
// u).  This is the iteration of items 3-6 with the iterate stored as u: the
// map x -> u is affine with fixed j0' and rho, and both the plain and the
// Chebyshev update are affine combinations of iterates, so the sequence is
// the same up to rounding.  The stop rule's |G(x_k) - x_k| is evaluated as
// |G + j0' - rho u_k|, and the final x = rho u - j0' is formed once after
// the last pass.  Each pass then reads u (stencil), p and P1 (stencil; both
// evaluated once per step) and, at its own point, j0' and rho, and writes
// the next u (the Chebyshev form also reads u_{k-1}, which it overwrites in
// place).
//
// In 3D a block owns a TX x TY tile of an xy plane and marches through TZ
// planes of z.  Its threads are the (TX+4) x (TY+4) points where q is needed
// (the tile and a 2-wide frame for the outer first derivative).  Each thread keeps, in
// registers, five planes of u at its point (z-derivatives of u, and u_k at
// the output plane) and of q_az (z-derivative in d_b q_ab); LDS holds a u
// plane (tile + 4-wide frame) and a q plane (tile + 2-wide frame) for the x
// and y derivatives, in two buffers each, so that a plane step writes one
// buffer while it reads the other and needs a single barrier.
#pragma once

#include "kernels.hpp"

namespace lb2p {

// Periodic index for v in [-n, 3n) (z planes: the chunk length TZ <= nz).
__device__ __forceinline__ int wrap3(int v, int n)
{
    v += (v < 0) ? n : 0;
    v -= (v >= n) ? n : 0;
    v -= (v >= n) ? n : 0;
    return v;
}

// Periodic index for any v (used once per thread for the tile coordinates,
// where a tile may be wider than the grid).
__device__ __forceinline__ int wrapmod(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// One component plane of a domain as a raw buffer resource (stride 0, the
// plane's byte size as its range).  A load at an offset at or past the range
// returns 0 and a store there is dropped by the hardware's range check, so
// every lane can issue every load and store of a step: a lane with nothing to
// read or write passes the offset `range` itself.  With no load or store
// under a branch, the compiler counts outstanding memory operations exactly
// and can wait for one step's loads while the next step's are still in
// flight.  (Planes stay below 4 GiB: the host limits a domain to fewer than
// 2^29 sites.)
struct PlaneBuf {
    __amdgpu_buffer_rsrc_t rs;
    unsigned range;
};
__device__ __forceinline__ PlaneBuf plane_buf(const void* base, unsigned bytes)
{
    // dword 3 of the resource: 32-bit data format (the gfx9 raw-buffer value)
    return PlaneBuf{__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000),
                    bytes};
}
template <class R>
__device__ __forceinline__ R bload(const PlaneBuf& b, unsigned off)
{
    if constexpr (sizeof(R) == 4) {
        return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b32(b.rs, (int)off, 0, 0));
    } else {
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        return __builtin_bit_cast(R, (u2)__builtin_amdgcn_raw_buffer_load_b64(b.rs, (int)off, 0, 0));
    }
}
template <class R>
__device__ __forceinline__ void bstore(const PlaneBuf& b, unsigned off, R v)
{
    if constexpr (sizeof(R) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), b.rs, (int)off, 0, 0);
    } else {
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), b.rs, (int)off, 0, 0);
    }
}

// Inputs of one z step, loaded two steps ahead.
template <class R>
struct StepIn {
    R u[3];      // u, own point, lead plane
    R p, P1;     // p, P1, own point, centre plane
    R fu[3];     // u, frame point, centre plane
    R j[3];      // j0', own point, output plane
    R rho;       // rho there
    R v[3];      // u_{k-1} there (Chebyshev)
};

template <class R, int TX, int TY, bool CHEB>
__global__ void __launch_bounds__((TX + 4) * (TY + 4)) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 1)))
k_iter_fused3(const Domain* __restrict__ tab, const Tile* __restrict__ tiles, IterCtl ic, int it,
              const R* __restrict__ pf, const R* __restrict__ rho, const R* __restrict__ j0p,
              const R* __restrict__ u_old, R* u_new)
{
    constexpr int QX = TX + 4, QY = TY + 4;   // q points
    constexpr int UX = TX + 8, UY = TY + 8;   // u points
    constexpr int NFRAME = UX * UY - QX * QY;
    static_assert(NFRAME <= QX * QY, "frame larger than the block");
    // two buffers of each plane: a step writes one while it reads the other
    __shared__ R su[2][3][UY][UX];
    __shared__ R sq[2][5][QY][QX];   // q_xx, q_yy, q_xy, q_xz, q_yz (q_zz is only needed along z)

    const Tile tl = tiles[blockIdx.x];
    if (tl.dom < 0 || iter_skip(ic, tl.dom, it)) return;   // uniform per block
    const Domain& dm = tab[tl.dom];
    const int nx = dm.g.nx, ny = dm.g.ny, nz = dm.g.nz;
    const long long N = dm.g.S;   // component stride
    const unsigned plane = (unsigned)nx * (unsigned)ny;
    const unsigned bytes = (unsigned)dm.g.N * (unsigned)sizeof(R);
    const PlaneBuf bP = plane_buf(pf + dm.off, bytes);   // p - p_ref
    const PlaneBuf bP1 = plane_buf(pf + dm.off + N, bytes);
    const R pref = R(dm.cf.pref);
    const PlaneBuf bRho = plane_buf(rho + dm.off, bytes);
    const PlaneBuf bJ[3] = {plane_buf(j0p + dm.off, bytes), plane_buf(j0p + dm.off + N, bytes),
                            plane_buf(j0p + dm.off + 2 * N, bytes)};
    const PlaneBuf bU[3] = {plane_buf(u_old + dm.off, bytes), plane_buf(u_old + dm.off + N, bytes),
                            plane_buf(u_old + dm.off + 2 * N, bytes)};
    const PlaneBuf bV[3] = {plane_buf(u_new + dm.off, bytes), plane_buf(u_new + dm.off + N, bytes),
                            plane_buf(u_new + dm.off + 2 * N, bytes)};
    const unsigned OUT = bytes;   // an offset outside every plane
    R omega = R(1), gam = R(1);
    if (CHEB) {
        omega = R(ic.omega[(long long)tl.dom * ic.stride + it]);
        gam = R(dm.cf.cheb_gamma);
    }
    // q point (qx, qy) of this thread in the QX x QY region: the TX x TY
    // tile points first (whole wavefronts when TX * TY is a multiple of 64,
    // so the output step is uniform per wavefront and a wavefront reads whole
    // rows), then the 2-wide frame around them
    static_assert((TX * TY) % 64 == 0, "tile points must fill whole wavefronts");
    const int tid = threadIdx.x + QX * threadIdx.y;
    int qx, qy;
    // uniform per wavefront (the compiler then branches on it)
    const bool interior = __builtin_amdgcn_readfirstlane(tid >> 6) < (TX * TY) / 64;
    if (interior) {
        qx = 2 + tid % TX; qy = 2 + tid / TX;
    } else {
        const int e = tid - TX * TY;
        if (e < 2 * QX) {                    // two rows at the bottom
            qy = e / QX; qx = e % QX;
        } else if (e < 4 * QX) {             // two rows at the top
            qy = QY - 4 + e / QX; qx = e % QX;
        } else {                             // two columns left, two right
            const int t = e - 4 * QX;
            const int c = t % 4;
            qy = 2 + t / 4;
            qx = c < 2 ? c : QX - 4 + c;
        }
    }
    const int x0 = tl.x0, y0 = tl.y0, z0 = tl.z0, TZ = tl.len;
    const int gx = wrapmod(x0 + qx - 2, nx), gy = wrapmod(y0 + qy - 2, ny);
    const unsigned col = (unsigned)gx + (unsigned)nx * (unsigned)gy;
    const bool owned = interior && (x0 + qx - 2 < nx) && (y0 + qy - 2 < ny);

    // this thread's u-frame point (outer 2-wide ring of the UX x UY region)
    int fx = 0, fy = 0;
    const bool has_frame = tid < NFRAME;
    if (has_frame) {
        if (tid < 2 * UX) {                  // two rows at the bottom
            fy = tid / UX; fx = tid % UX;
        } else if (tid < 4 * UX) {           // two rows at the top
            const int t = tid - 2 * UX;
            fy = UY - 2 + t / UX; fx = t % UX;
        } else {                             // two columns left, two right
            const int t = tid - 4 * UX;
            const int row = t / 4, c = t % 4;
            fy = 2 + row;
            fx = c < 2 ? c : UX - 4 + c;
        }
    }
    const unsigned fcol = has_frame
        ? (unsigned)wrapmod(x0 + fx - 4, nx) + (unsigned)nx * (unsigned)wrapmod(y0 + fy - 4, ny) : 0u;

    // Plane rings, oldest first; each step shifts them by one.  (Rings
    // addressed by a compile-time phase avoid the moves but need the loop
    // unrolled five times, which costs registers and, measured, occupancy
    // and time.)
    R ur[5][3];        // u at five consecutive planes (see the step below)
    R qz[5][3];        // q_xz, q_yz, q_zz at planes c-4 .. c of the last q plane c
    R sd[2][3];        // x,y part of d_b q_ab at the last two planes it was taken
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) { ur[k][a] = R(0); qz[k][a] = R(0); }
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) sd[k][a] = R(0);
    R dmax = R(0), dsum = R(0);   // dsum only carries a NaN (fmax drops it)
    const R c12 = R(1.0 / 12.0);

    // Step k, with c_k = z0-6+k and one barrier, at its end:
    //   1. u plane c_k into LDS buffer k&1 (own point from the ring, frame
    //      point loaded);
    //   2. q at plane c_{k-1} from LDS buffer (k-1)&1 (written last step)
    //      and the ring, into q buffer (k-1)&1;
    //   3. the x,y part of d_b q_ab at plane c_{k-2} from q buffer k&1
    //      (written last step), and the next iterate at the output plane
    //      o = c_{k-3} = z0-9+k (written for 9 <= k < TZ+9);
    //   4. the ring shifts in the lead plane z0-4+k.
    // Before its shift the ring holds planes z0-9+k .. z0-5+k: ur[0] is the
    // output plane, ur[2] = c_{k-1}, ur[3] = c_k.  The three phases touch
    // different buffers, so one barrier per step orders every LDS write
    // before its reads in the next step and every read before the write two
    // steps later.  Steps run in pairs, so one past the end may run with its
    // output dropped; every plane index stays in [z0-7, z0+TZ+7) and is
    // wrapped.
    const int nsteps = TZ + 9;
    auto out_plane = [&](int k) -> bool { return k >= 9 && k < nsteps && z0 + k - 9 < nz; };
    // Loaders of the inputs of step k, one per group of fields.
    auto load_own = [&](int k, StepIn<R>& in) {
        const bool own = owned && out_plane(k);
        const unsigned io = own ? (col + plane * (unsigned)(z0 + k - 9)) * (unsigned)sizeof(R) : OUT;
#pragma unroll
        for (int a = 0; a < 3; ++a) in.j[a] = bload<R>(bJ[a], io);
        in.rho = bload<R>(bRho, io);
        if (CHEB) {
            const unsigned iv = it > 0 ? io : OUT;
#pragma unroll
            for (int a = 0; a < 3; ++a) in.v[a] = bload<R>(bV[a], iv);
        }
    };
    auto load_lead = [&](int k, StepIn<R>& in) {
        const unsigned il = (col + plane * (unsigned)wrap3(z0 - 4 + k, nz)) * (unsigned)sizeof(R);
#pragma unroll
        for (int a = 0; a < 3; ++a) in.u[a] = bload<R>(bU[a], il);
    };
    auto load_frame = [&](int k, StepIn<R>& in) {
        const unsigned zc = plane * (unsigned)wrap3(z0 - 6 + k, nz);
        const unsigned ifr = has_frame ? (fcol + zc) * (unsigned)sizeof(R) : OUT;
#pragma unroll
        for (int a = 0; a < 3; ++a) in.fu[a] = bload<R>(bU[a], ifr);
    };
    auto load_pp = [&](int k, StepIn<R>& in) {
        const unsigned ic_ = (col + plane * (unsigned)wrap3(z0 - 7 + k, nz)) * (unsigned)sizeof(R);
        in.p = pref + bload<R>(bP, ic_);
        in.P1 = bload<R>(bP1, ic_);
    };

    // Step k reads its inputs from `in` and refills each group, right after
    // its last use, with the inputs of step k+2 (the same phase two steps
    // later): every load has two steps to complete, in two register sets.
    auto run_step = [&](int k, StepIn<R>& in) {
        const int b = k & 1;
        // 1. u plane c_k into LDS buffer b: own point and frame point
#pragma unroll
        for (int a = 0; a < 3; ++a) su[b][a][qy + 2][qx + 2] = ur[3][a];
        if (has_frame) {
#pragma unroll
            for (int a = 0; a < 3; ++a) su[b][a][fy][fx] = in.fu[a];
        }
        load_frame(k + 2, in);
        // 2. q at plane c_{k-1}
        if (k >= 5) {
            const int bu = b ^ 1;
            R G[3][3];   // G[a][b] = d_a u_b
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                G[0][c] = d1<R>(su[bu][c][qy + 2][qx], su[bu][c][qy + 2][qx + 1], su[bu][c][qy + 2][qx + 3],
                                su[bu][c][qy + 2][qx + 4]);
                G[1][c] = d1<R>(su[bu][c][qy][qx + 2], su[bu][c][qy + 1][qx + 2], su[bu][c][qy + 3][qx + 2],
                                su[bu][c][qy + 4][qx + 2]);
                G[2][c] = d1<R>(ur[0][c], ur[1][c], ur[3][c], ur[4][c]);
            }
            const R X = in.P1 * (G[0][0] + G[1][1] + G[2][2]);
            const R p2 = R(2) * in.p;
            const R qxz = in.p * (G[0][2] + G[2][0]);
            const R qyz = in.p * (G[1][2] + G[2][1]);
            sq[bu][0][qy][qx] = X + p2 * G[0][0];
            sq[bu][1][qy][qx] = X + p2 * G[1][1];
            sq[bu][2][qy][qx] = in.p * (G[0][1] + G[1][0]);
            sq[bu][3][qy][qx] = qxz;
            sq[bu][4][qy][qx] = qyz;
            if (interior) {   // d_z q_az is only taken at tile points
#pragma unroll
                for (int s_ = 0; s_ < 4; ++s_)
#pragma unroll
                    for (int a = 0; a < 3; ++a) qz[s_][a] = qz[s_ + 1][a];
                qz[4][0] = qxz; qz[4][1] = qyz; qz[4][2] = X + p2 * G[2][2];
            }
        }
        load_pp(k + 2, in);
        // 3. the x,y part of the divergence at c_{k-2}; the next iterate at
        //    the output plane c_{k-3}
        R un[3] = {R(0), R(0), R(0)};
        const bool out = owned && out_plane(k);
        if (k >= 6 && interior) {
            const int px = qx, py = qy;
#pragma unroll
            for (int a = 0; a < 3; ++a) sd[0][a] = sd[1][a];
            // a = x: d_x q_xx + d_y q_xy ; a = y: d_x q_xy + d_y q_yy ; a = z: d_x q_xz + d_y q_yz
            sd[1][0] = d1<R>(sq[b][0][py][px - 2], sq[b][0][py][px - 1], sq[b][0][py][px + 1], sq[b][0][py][px + 2]) +
                       d1<R>(sq[b][2][py - 2][px], sq[b][2][py - 1][px], sq[b][2][py + 1][px], sq[b][2][py + 2][px]);
            sd[1][1] = d1<R>(sq[b][2][py][px - 2], sq[b][2][py][px - 1], sq[b][2][py][px + 1], sq[b][2][py][px + 2]) +
                       d1<R>(sq[b][1][py - 2][px], sq[b][1][py - 1][px], sq[b][1][py + 1][px], sq[b][1][py + 2][px]);
            sd[1][2] = d1<R>(sq[b][3][py][px - 2], sq[b][3][py][px - 1], sq[b][3][py][px + 1], sq[b][3][py][px + 2]) +
                       d1<R>(sq[b][4][py - 2][px], sq[b][4][py - 1][px], sq[b][4][py + 1][px], sq[b][4][py + 2][px]);
            if (out) {
                const R ri = R(1) / in.rho;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const R dz = d1<R>(qz[0][a], qz[1][a], qz[3][a], qz[4][a]);
                    const R gv = -(sd[0][a] + dz) * c12;          // G(x_k)_a
                    // item 6: |G(x_k) - x_k| with x_k = rho u_k - j0'
                    const R d = fabs(gv + in.j[a] - in.rho * ur[0][a]);
                    dmax = fmax(dmax, d);
                    dsum += d;
                    // item 3 of the next pass: u = (j0' + G)/rho
                    const R gu = (in.j[a] + gv) * ri;
                    un[a] = CHEB ? next_iterate<R>(gu, ur[0][a], in.v[a], omega, gam, it == 0) : gu;
                }
            }
        }
        // every lane stores; lanes without an output point write nowhere
        const unsigned io = out ? (col + plane * (unsigned)(z0 + k - 9)) * (unsigned)sizeof(R) : OUT;
#pragma unroll
        for (int a = 0; a < 3; ++a) bstore<R>(bV[a], io, un[a]);
        load_own(k + 2, in);
        // 4. the ring takes the lead plane
#pragma unroll
        for (int s_ = 0; s_ < 4; ++s_)
#pragma unroll
            for (int a = 0; a < 3; ++a) ur[s_][a] = ur[s_ + 1][a];
#pragma unroll
        for (int a = 0; a < 3; ++a) ur[4][a] = in.u[a];
        load_lead(k + 2, in);
        __syncthreads();
    };

    StepIn<R> A, B;
    load_lead(0, A); load_frame(0, A); load_pp(0, A); load_own(0, A);
    load_lead(1, B); load_frame(1, B); load_pp(1, B); load_own(1, B);
    for (int k = 0; k < nsteps; k += 2) {
        run_step(k, A);
        run_step(k + 1, B);
    }
    block_max_part(ic.part, dsum == dsum ? (double)dmax : (double)dsum);
}

// One pass of the correction-current iteration for D2Q21 (items 3-6), in the
// velocity form of the 3D pass: u_{k+1} = (j0' + G)/rho with G = -(1/12)
// d_b q_ab and q built from u_k.  A block owns a TX-wide column strip of
// tl.len rows and marches along y in chunks of CH rows.  Rows of u (strip +
// 4-wide frame) and of q (strip + 2-wide frame) pass through LDS rings
// indexed by the row number, so each u and q row is loaded or computed once
// per strip: per chunk the threads load the next CH rows of u, compute the
// next CH rows of q, then the strip's wavefronts take the divergence for the
// chunk's CH output rows.  Threads: one per q point of a chunk, (TX+4) x CH,
// the strip's TX x CH points first (whole wavefronts).
template <class R, int TX, int CH, bool CHEB>
__global__ void __launch_bounds__((TX + 4) * CH)
k_iter_fused2(const Domain* __restrict__ tab, const Tile* __restrict__ tiles, IterCtl ic, int it,
              const R* __restrict__ pf, const R* __restrict__ rho, const R* __restrict__ j0p,
              const R* __restrict__ u_old, R* u_new)
{
    constexpr int QX = TX + 4, UX = TX + 8;
    constexpr int RU = 2 * CH + 8;   // u ring: rows a chunk's q and output phases read, and the next chunk's
    constexpr int RQ = CH + 4;       // q ring
    static_assert((TX * CH) % 64 == 0, "strip points must fill whole wavefronts");
    __shared__ R su[2][RU][UX];
    __shared__ R sq[3][RQ][QX];   // q_xx, q_yy, q_xy

    const Tile tl = tiles[blockIdx.x];
    if (tl.dom < 0 || iter_skip(ic, tl.dom, it)) return;   // uniform per block
    const Domain& dm = tab[tl.dom];
    const int nx = dm.g.nx, ny = dm.g.ny;
    const long long N = dm.g.S;
    const unsigned bytes = (unsigned)dm.g.N * (unsigned)sizeof(R);
    const unsigned OUT = bytes;
    const long long o = dm.off;
    const PlaneBuf bP = plane_buf(pf + o, bytes);   // p - p_ref
    const PlaneBuf bP1 = plane_buf(pf + o + N, bytes);
    const R pref = R(dm.cf.pref);
    const PlaneBuf bRho = plane_buf(rho + o, bytes);
    const PlaneBuf bJ[2] = {plane_buf(j0p + o, bytes), plane_buf(j0p + o + N, bytes)};
    const PlaneBuf bU[2] = {plane_buf(u_old + o, bytes), plane_buf(u_old + o + N, bytes)};
    const PlaneBuf bV[2] = {plane_buf(u_new + o, bytes), plane_buf(u_new + o + N, bytes)};
    R omega = R(1), gam = R(1);
    if (CHEB) {
        omega = R(ic.omega[(long long)tl.dom * ic.stride + it]);
        gam = R(dm.cf.cheb_gamma);
    }

    const int tid = threadIdx.x + QX * threadIdx.y;
    int qx, r;   // q column (LDS column qx + 2) and row within the chunk
    const bool interior = __builtin_amdgcn_readfirstlane(tid >> 6) < (TX * CH) / 64;
    if (interior) {
        qx = 2 + tid % TX; r = tid / TX;
    } else {
        const int e = tid - TX * CH;   // 0 .. 4 CH - 1
        const int c = e % 4;
        r = e / 4;
        qx = c < 2 ? c : TX + c;
    }
    // the extra u columns (LDS 0, 1, TX+6, TX+7) of a chunk row, loaded by
    // the frame threads
    const bool has_extra = !interior;
    const int ux_extra = has_extra ? ((tid - TX * CH) % 4 < 2 ? (tid - TX * CH) % 4 : TX + 4 + (tid - TX * CH) % 4) : 0;
    const int x0 = tl.x0, y0 = tl.y0, H = tl.len;
    const unsigned gx = (unsigned)wrapmod(x0 + qx - 2, nx);
    const unsigned gxe = (unsigned)wrapmod(x0 + ux_extra - 4, nx);
    const bool col_owned = interior && (x0 + qx - 2 < nx);
    auto row_off = [&](int y) { return (unsigned)nx * (unsigned)wrapmod(y, ny); };
    auto slotU = [&](int y) { return (y - y0 + 4 + RU) % RU; };   // y >= y0 - 4
    auto slotQ = [&](int y) { return (y - y0 + 2 + RQ) % RQ; };   // y >= y0 - 2

    // u row y of the strip (+ frame) into the ring
    auto load_u_row = [&](int y, bool live) {
        const unsigned ro = row_off(y);
        const unsigned iu = live ? (gx + ro) * (unsigned)sizeof(R) : OUT;
        const unsigned ie = live && has_extra ? (gxe + ro) * (unsigned)sizeof(R) : OUT;
        R v[2], w[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            v[a] = bload<R>(bU[a], iu);
            w[a] = bload<R>(bU[a], ie);
        }
        if (live) {
            const int sl = slotU(y);
#pragma unroll
            for (int a = 0; a < 2; ++a) su[a][sl][qx + 2] = v[a];
            if (has_extra) {
#pragma unroll
                for (int a = 0; a < 2; ++a) su[a][sl][ux_extra] = w[a];
            }
        }
    };
    // q row y (needs u rows y-2 .. y+2 in the ring)
    auto q_row = [&](int y, R p, R P1) {
        const int s0 = slotU(y), sm1 = slotU(y - 1), sm2 = slotU(y - 2), sp1 = slotU(y + 1), sp2 = slotU(y + 2);
        R G[2][2];   // G[a][b] = d_a u_b
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            G[0][b] = d1<R>(su[b][s0][qx], su[b][s0][qx + 1], su[b][s0][qx + 3], su[b][s0][qx + 4]);
            G[1][b] = d1<R>(su[b][sm2][qx + 2], su[b][sm1][qx + 2], su[b][sp1][qx + 2], su[b][sp2][qx + 2]);
        }
        const R X = P1 * (G[0][0] + G[1][1]);
        const R p2 = R(2) * p;
        const int sl = slotQ(y);
        sq[0][sl][qx] = X + p2 * G[0][0];
        sq[1][sl][qx] = X + p2 * G[1][1];
        sq[2][sl][qx] = p * (G[0][1] + G[1][0]);
    };

    // prologue: u rows y0-4 .. y0+3, then q rows y0-2 .. y0+1
    if (r < 8) load_u_row(y0 - 4 + r, true);
    R pp = R(0), pP1 = R(0);
    {
        const unsigned ip = r < 4 ? (gx + row_off(y0 - 2 + r)) * (unsigned)sizeof(R) : OUT;
        pp = pref + bload<R>(bP, ip);
        pP1 = bload<R>(bP1, ip);
    }
    __syncthreads();
    if (r < 4) q_row(y0 - 2 + r, pp, pP1);

    R dmax = R(0), dsum = R(0);   // dsum only carries a NaN (fmax drops it)
    const R c12 = R(1.0 / 12.0);
    // Inputs of one chunk, loaded a chunk ahead (they arrive while the
    // previous chunk computes q and its outputs).
    struct ChunkIn {
        R u[2], ue[2];   // u row Y+4+r at the q column and the extra column
        R p, P1;         // row Y+2+r
        R j[2], v[2], rho;   // output row Y+r
    };
    auto load_chunk = [&](int Y, ChunkIn& c) {
        const unsigned ro = row_off(Y + 4 + r);
        const unsigned iu = (gx + ro) * (unsigned)sizeof(R);
        const unsigned ie = has_extra ? (gxe + ro) * (unsigned)sizeof(R) : OUT;
        const unsigned ip = (gx + row_off(Y + 2 + r)) * (unsigned)sizeof(R);
        const bool out = col_owned && Y + r < y0 + H;
        const unsigned io = out ? (gx + row_off(Y + r)) * (unsigned)sizeof(R) : OUT;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            c.u[a] = bload<R>(bU[a], iu);
            c.ue[a] = bload<R>(bU[a], ie);
            c.j[a] = bload<R>(bJ[a], io);
            c.v[a] = CHEB ? bload<R>(bV[a], it > 0 ? io : OUT) : R(0);
        }
        c.p = pref + bload<R>(bP, ip);
        c.P1 = bload<R>(bP1, ip);
        c.rho = bload<R>(bRho, io);
    };
    ChunkIn nx_in;
    load_chunk(y0, nx_in);
    for (int Y = y0; Y < y0 + H; Y += CH) {
        const ChunkIn cur = nx_in;
        // L: the chunk's u rows into the ring
        {
            const int sl = slotU(Y + 4 + r);
#pragma unroll
            for (int a = 0; a < 2; ++a) su[a][sl][qx + 2] = cur.u[a];
            if (has_extra) {
#pragma unroll
                for (int a = 0; a < 2; ++a) su[a][sl][ux_extra] = cur.ue[a];
            }
        }
        load_chunk(Y + CH, nx_in);   // rows wrap, so the loads past the strip stay in range
        const int yo = Y + r;
        const bool out = col_owned && yo < y0 + H;
        const unsigned io = out ? (gx + row_off(yo)) * (unsigned)sizeof(R) : OUT;
        __syncthreads();
        // Q: q rows Y+2 .. Y+CH+1
        q_row(Y + 2 + r, cur.p, cur.P1);
        __syncthreads();
        // O: output rows Y .. Y+CH-1 on the strip's wavefronts
        R un[2] = {R(0), R(0)};
        if (interior) {
            const int s0 = slotQ(yo), sm1 = slotQ(yo - 1), sm2 = slotQ(yo - 2), sp1 = slotQ(yo + 1),
                      sp2 = slotQ(yo + 2);
            const int px = qx;
            const R sd[2] = {
                d1<R>(sq[0][s0][px - 2], sq[0][s0][px - 1], sq[0][s0][px + 1], sq[0][s0][px + 2]) +
                    d1<R>(sq[2][sm2][px], sq[2][sm1][px], sq[2][sp1][px], sq[2][sp2][px]),
                d1<R>(sq[2][s0][px - 2], sq[2][s0][px - 1], sq[2][s0][px + 1], sq[2][s0][px + 2]) +
                    d1<R>(sq[1][sm2][px], sq[1][sm1][px], sq[1][sp1][px], sq[1][sp2][px])};
            const int su0 = slotU(yo);
            if (out) {
                const R rr = cur.rho;
                const R ri = R(1) / rr;
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const R uk = su[a][su0][qx + 2];
                    const R gv = -sd[a] * c12;                     // G(x_k)_a
                    const R d = fabs(gv + cur.j[a] - rr * uk);     // |G(x_k) - x_k|, x_k = rho u_k - j0'
                    dmax = fmax(dmax, d);
                    dsum += d;
                    const R gu = (cur.j[a] + gv) * ri;
                    un[a] = CHEB ? next_iterate<R>(gu, uk, cur.v[a], omega, gam, it == 0) : gu;
                }
            }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a) bstore<R>(bV[a], io, un[a]);
    }
    block_max_part(ic.part, dsum == dsum ? (double)dmax : (double)dsum, tl.slot);
}

// u = (j0' + j~)/rho for the final iterate (item 8).
template <int Q, class R>
__global__ void __launch_bounds__(256) k_u_final(const Domain* __restrict__ tab,
                                                 const Tile* __restrict__ tiles,
                                                 const SolveInfo* __restrict__ info,
                                                 const R* __restrict__ rho, const R* __restrict__ j0p,
                                                 const R* __restrict__ jtA, const R* __restrict__ jtB,
                                                 R* __restrict__ u)
{
    using L = Lattice<Q>;
    const Where w = locate(tab, tiles);
    if (!w.ok) return;
    const Domain& dm = tab[w.dom];
    const long long St = dm.g.S;
    const long long i0 = dm.off + sidx(dm.g, w.x, w.y, w.z);
    const R* jt = info[w.dom].final_buf ? jtB : jtA;
    const R inv = R(1) / rho[i0];
#pragma unroll
    for (int a = 0; a < L::D; ++a) u[a * St + i0] = (j0p[a * St + i0] + jt[a * St + i0]) * inv;
}

// The velocity-form solve ends with u_final in u (even pass count) or u1
// (odd): x = rho u - j0' (the correction current of items 7-12) goes to the
// j~ buffer the pass count selects, as in the current form, and u_final to u.
template <int Q, class R>
__global__ void __launch_bounds__(256) k_jt_final(const Domain* __restrict__ tab,
                                                  const Tile* __restrict__ tiles,
                                                  const SolveInfo* __restrict__ info,
                                                  const R* __restrict__ rho, const R* __restrict__ j0p,
                                                  R* __restrict__ u0, const R* __restrict__ u1,
                                                  R* __restrict__ jtA, R* __restrict__ jtB)
{
    using L = Lattice<Q>;
    const Where w = locate(tab, tiles);
    if (!w.ok) return;
    const Domain& dm = tab[w.dom];
    const long long St = dm.g.S;
    const long long i0 = dm.off + sidx(dm.g, w.x, w.y, w.z);
    const bool odd = info[w.dom].final_buf != 0;   // uniform per block
    const R* uf = odd ? u1 : u0;
    R* jt = odd ? jtB : jtA;
    const R r = rho[i0];
#pragma unroll
    for (int a = 0; a < L::D; ++a) {
        const R v = uf[a * St + i0];
        jt[a * St + i0] = r * v - j0p[a * St + i0];
        if (odd) u0[a * St + i0] = v;
    }
}

// Copy each domain's final j~ (the buffer its SolveInfo selects) into a
// plain [d][S] field.
template <int Q, class R>
__global__ void __launch_bounds__(256) k_keep_jt(const Domain* __restrict__ tab,
                                                 const Tile* __restrict__ tiles,
                                                 const SolveInfo* __restrict__ info,
                                                 const R* __restrict__ jtA, const R* __restrict__ jtB,
                                                 R* __restrict__ out)
{
    using L = Lattice<Q>;
    const Where w = locate(tab, tiles);
    if (!w.ok) return;
    const Domain& dm = tab[w.dom];
    const long long St = dm.g.S;
    const long long i0 = dm.off + sidx(dm.g, w.x, w.y, w.z);
    const R* jt = info[w.dom].final_buf ? jtB : jtA;
#pragma unroll
    for (int a = 0; a < L::D; ++a) out[a * St + i0] = jt[a * St + i0];
}

// The SolveInfo of a kept j~: its pass count, in buffer 0 of the kept field.
__global__ void k_info_keep(const SolveInfo* __restrict__ info, SolveInfo* __restrict__ keep, int ndom)
{
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= ndom) return;
    SolveInfo k = info[d];
    k.final_buf = 0;
    keep[d] = k;
}

}  // namespace lb2p
