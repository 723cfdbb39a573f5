// kernels_fused.hpp -- one kernel per pass of the correction-current
// iteration (Supplemental items 3-6) for D3Q59, carried in velocity form.
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
// A block owns a TX x TY tile of an xy plane and marches through TZ planes of
// z.  Its threads are the (TX+4) x (TY+4) points where q is needed (the tile
// and a 2-wide frame for the outer first derivative).  Each thread keeps, in
// registers, the last five planes of u at its point (z-derivatives of u, and
// u_k at the output plane) and of q_az (z-derivative in d_b q_ab); LDS holds
// one u plane (tile + 4-wide frame) and one q plane (tile + 2-wide frame)
// for the x and y derivatives.
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

// Element i of a component plane: a uniform base plus a 32-bit byte offset
// (the host keeps one plane of a domain under 4 GiB for this kernel), which
// lets loads use the scalar-base addressing form instead of 64-bit VALU math.
template <class R>
__device__ __forceinline__ R ld(const R* base, unsigned i)
{
    return *reinterpret_cast<const R*>(reinterpret_cast<const char*>(base) + i * (unsigned)sizeof(R));
}
template <class R>
__device__ __forceinline__ void st(R* base, unsigned i, R v)
{
    *reinterpret_cast<R*>(reinterpret_cast<char*>(base) + i * (unsigned)sizeof(R)) = v;
}

template <class R, int TX, int TY, bool CHEB>
__global__ void __launch_bounds__((TX + 4) * (TY + 4))
k_iter_fused3(const Domain* __restrict__ tab, const Tile* __restrict__ tiles, IterCtl ic, int it,
              const R* __restrict__ pf, const R* __restrict__ rho, const R* __restrict__ j0p,
              const R* __restrict__ u_old, R* u_new)
{
    constexpr int QX = TX + 4, QY = TY + 4;   // q points
    constexpr int UX = TX + 8, UY = TY + 8;   // u points
    constexpr int NFRAME = UX * UY - QX * QY;
    static_assert(NFRAME <= QX * QY, "frame larger than the block");
    __shared__ R su[3][UY][UX];
    __shared__ R sq[5][QY][QX];   // q_xx, q_yy, q_xy, q_xz, q_yz (q_zz is only needed along z)

    const Tile tl = tiles[blockIdx.x];
    if (tl.dom < 0 || iter_skip(ic, tl.dom, it)) return;   // uniform per block
    const Domain& dm = tab[tl.dom];
    const int nx = dm.g.nx, ny = dm.g.ny, nz = dm.g.nz;
    const long long N = dm.g.S;   // component stride
    const unsigned plane = (unsigned)nx * (unsigned)ny;
    const R* const pP = pf + dm.off;
    const R* const pP1 = pP + N;
    const R* const pRho = rho + dm.off;
    const R* const j0x = j0p + dm.off;
    const R* const j0y = j0x + N;
    const R* const j0z = j0y + N;
    const R* const ux = u_old + dm.off;
    const R* const uy = ux + N;
    const R* const uz = uy + N;
    R* const vx = u_new + dm.off;
    R* const vy = vx + N;
    R* const vz = vy + N;
    R omega = R(1), gam = R(1);
    if (CHEB) {
        omega = R(ic.omega[(long long)tl.dom * ic.stride + it]);
        gam = R(dm.cf.cheb_gamma);
    }
    const int lx = threadIdx.x, ly = threadIdx.y;
    const int tid = lx + QX * ly;
    const int x0 = tl.x0, y0 = tl.y0, z0 = tl.z0, TZ = tl.len;
    const int gx = wrapmod(x0 + lx - 2, nx), gy = wrapmod(y0 + ly - 2, ny);
    const unsigned col = (unsigned)gx + (unsigned)nx * (unsigned)gy;
    const bool interior = lx >= 2 && lx < TX + 2 && ly >= 2 && ly < TY + 2;
    const bool owned = interior && (x0 + lx - 2 < nx) && (y0 + ly - 2 < ny);

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
    R ur[5][3];        // u at planes lead-4 .. lead (lead-4 is the output plane)
    R qz[5][3];        // q_xz, q_yz, q_zz at planes c-4 .. c
    R sd[3][3];        // x,y part of d_b q_ab at planes c-2 .. c
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) { ur[k][a] = R(0); qz[k][a] = R(0); }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) sd[k][a] = R(0);
    R dmax = R(0), dsum = R(0);   // dsum only carries a NaN (fmax drops it)
    const R c12 = R(1.0 / 12.0);

    // one-plane lookahead: the inputs of step k+1 are loaded while step k
    // computes
    R nu[3] = {R(0), R(0), R(0)};                 // u, own point, lead plane
    R np = R(0), nP1 = R(0);                      // p, P1, own point, centre plane
    R fu[3] = {R(0), R(0), R(0)};                 // u, frame point, centre plane
    R nv[3] = {R(0), R(0), R(0)};                 // u_{k-1}, own point, output plane (Chebyshev)
    R nj[3] = {R(0), R(0), R(0)}, nrho = R(1);    // j0' and rho there
    auto load_step = [&](int k) {
        if (k >= 8 && owned && z0 + k - 8 < nz) {
            const unsigned io = col + plane * (unsigned)(z0 + k - 8);
            nj[0] = ld(j0x, io); nj[1] = ld(j0y, io); nj[2] = ld(j0z, io);
            nrho = ld(pRho, io);
            if (CHEB && it > 0) { nv[0] = ld<R>(vx, io); nv[1] = ld<R>(vy, io); nv[2] = ld<R>(vz, io); }
        }
        const unsigned i = col + plane * (unsigned)wrap3(z0 - 4 + k, nz);
        nu[0] = ld(ux, i); nu[1] = ld(uy, i); nu[2] = ld(uz, i);
        const unsigned zc = plane * (unsigned)wrap3(z0 - 6 + k, nz);
        np = ld(pP, col + zc);
        nP1 = ld(pP1, col + zc);
        if (has_frame) {
            const unsigned f = fcol + zc;
            fu[0] = ld(ux, f); fu[1] = ld(uy, f); fu[2] = ld(uz, f);
        }
    };
    load_step(0);
    const int nsteps = TZ + 8;

    for (int k = 0; k < nsteps; ++k) {
        const R cur_u[3] = {nu[0], nu[1], nu[2]};
        const R cur_p = np, cur_P1 = nP1;
        const R cur_fu[3] = {fu[0], fu[1], fu[2]};
        const R cur_v[3] = {nv[0], nv[1], nv[2]};
        const R cur_j[3] = {nj[0], nj[1], nj[2]};
        const R cur_rho = nrho;
        if (k + 1 < nsteps) load_step(k + 1);
        // 1. lead plane of the u ring at this thread's point
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) ur[s][a] = ur[s + 1][a];
#pragma unroll
        for (int a = 0; a < 3; ++a) ur[4][a] = cur_u[a];
        // 2. u plane c = lead-2 into LDS: own point and frame point
#pragma unroll
        for (int a = 0; a < 3; ++a) su[a][ly + 2][lx + 2] = ur[2][a];
        if (has_frame) {
#pragma unroll
            for (int a = 0; a < 3; ++a) su[a][fy][fx] = cur_fu[a];
        }
        __syncthreads();
        // 3. q at plane c
        if (k >= 4) {
            R G[3][3];   // G[a][b] = d_a u_b
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                G[0][b] = d1<R>(su[b][ly + 2][lx], su[b][ly + 2][lx + 1], su[b][ly + 2][lx + 3],
                                su[b][ly + 2][lx + 4]);
                G[1][b] = d1<R>(su[b][ly][lx + 2], su[b][ly + 1][lx + 2], su[b][ly + 3][lx + 2],
                                su[b][ly + 4][lx + 2]);
                G[2][b] = d1<R>(ur[0][b], ur[1][b], ur[3][b], ur[4][b]);
            }
            const R X = cur_P1 * (G[0][0] + G[1][1] + G[2][2]);
            const R p2 = R(2) * cur_p;
            const R qxz = cur_p * (G[0][2] + G[2][0]);
            const R qyz = cur_p * (G[1][2] + G[2][1]);
            sq[0][ly][lx] = X + p2 * G[0][0];
            sq[1][ly][lx] = X + p2 * G[1][1];
            sq[2][ly][lx] = cur_p * (G[0][1] + G[1][0]);
            sq[3][ly][lx] = qxz;
            sq[4][ly][lx] = qyz;
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int a = 0; a < 3; ++a) qz[s][a] = qz[s + 1][a];
            qz[4][0] = qxz; qz[4][1] = qyz; qz[4][2] = X + p2 * G[2][2];
        }
        __syncthreads();
        // 4. the next iterate at plane c-2 = z0 + k - 8
        if (k >= 4 && interior) {
            const int px = lx, py = ly;
#pragma unroll
            for (int a = 0; a < 3; ++a) { sd[0][a] = sd[1][a]; sd[1][a] = sd[2][a]; }
            // a = x: d_x q_xx + d_y q_xy ; a = y: d_x q_xy + d_y q_yy ; a = z: d_x q_xz + d_y q_yz
            sd[2][0] = d1<R>(sq[0][py][px - 2], sq[0][py][px - 1], sq[0][py][px + 1], sq[0][py][px + 2]) +
                       d1<R>(sq[2][py - 2][px], sq[2][py - 1][px], sq[2][py + 1][px], sq[2][py + 2][px]);
            sd[2][1] = d1<R>(sq[2][py][px - 2], sq[2][py][px - 1], sq[2][py][px + 1], sq[2][py][px + 2]) +
                       d1<R>(sq[1][py - 2][px], sq[1][py - 1][px], sq[1][py + 1][px], sq[1][py + 2][px]);
            sd[2][2] = d1<R>(sq[3][py][px - 2], sq[3][py][px - 1], sq[3][py][px + 1], sq[3][py][px + 2]) +
                       d1<R>(sq[4][py - 2][px], sq[4][py - 1][px], sq[4][py + 1][px], sq[4][py + 2][px]);
            const int zo = z0 + k - 8;
            if (k >= 8 && owned && zo < z0 + TZ && zo < nz) {
                const unsigned i = col + plane * (unsigned)zo;
                const R ri = R(1) / cur_rho;
                R un[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const R dz = d1<R>(qz[0][a], qz[1][a], qz[3][a], qz[4][a]);
                    const R gv = -(sd[0][a] + dz) * c12;          // G(x_k)_a
                    // item 6: |G(x_k) - x_k| with x_k = rho u_k - j0'
                    const R d = fabs(gv + cur_j[a] - cur_rho * ur[0][a]);
                    dmax = fmax(dmax, d);
                    dsum += d;
                    // item 3 of the next pass: u = (j0' + G)/rho
                    const R gu = (cur_j[a] + gv) * ri;
                    un[a] = CHEB ? next_iterate<R>(gu, ur[0][a], cur_v[a], omega, gam, it == 0) : gu;
                }
                st(vx, i, un[0]); st(vy, i, un[1]); st(vz, i, un[2]);
            }
        }
    }
    block_max_part(ic.part, dsum == dsum ? (double)dmax : (double)dsum);
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

}  // namespace lb2p
