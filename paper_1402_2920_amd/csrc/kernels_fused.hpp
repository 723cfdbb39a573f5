// kernels_fused.hpp -- one kernel per pass of the correction-current
// iteration (Supplemental items 3-6) for D3Q59.
//
// A block owns a TX x TY tile of an xy plane and marches through TZ planes of
// z.  Its threads are the (TX+4) x (TY+4) points where q is needed (the tile
// and a 2-wide frame for the outer first derivative).  Each thread keeps, in
// registers, the last five planes of u at its point (z-derivatives of u) and
// of q_az (z-derivative in d_b q_ab); LDS holds one u plane (tile + 4-wide
// frame) and one q plane (tile + 2-wide frame) for the x and y derivatives.
// Per pass every site reads j~, j0' and rho once from HBM and writes j~new.
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

template <class R, int TX, int TY>
__global__ void __launch_bounds__((TX + 4) * (TY + 4))
k_iter_fused3(const Domain* __restrict__ tab, const Tile* __restrict__ tiles, IterCtl ic, int it,
              const R* __restrict__ rho, const R* __restrict__ j0p, const R* __restrict__ jt_old,
              R* __restrict__ jt_new)
{
    constexpr int QX = TX + 4, QY = TY + 4;   // q points
    constexpr int UX = TX + 8, UY = TY + 8;   // u points
    constexpr int NFRAME = UX * UY - QX * QY;
    static_assert(NFRAME <= QX * QY, "frame larger than the block");
    __shared__ R su[3][UY][UX];
    __shared__ R sq[6][QY][QX];

    const Tile tl = tiles[blockIdx.x];
    if (tl.dom < 0 || iter_skip(ic, tl.dom, it)) return;   // uniform per block
    const Domain& dm = tab[tl.dom];
    const Geom g = dm.g;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const long long N = g.S;   // component stride
    const long long plane = (long long)nx * ny;
    // this domain's part of the packed arrays
    rho += dm.off; j0p += dm.off; jt_old += dm.off; jt_new += dm.off;
    const Coef& cf = dm.cf;
    const int lx = threadIdx.x, ly = threadIdx.y;
    const int tid = lx + QX * ly;
    const int x0 = tl.x0, y0 = tl.y0, z0 = tl.z0, TZ = tl.len;
    const int gx = wrapmod(x0 + lx - 2, nx), gy = wrapmod(y0 + ly - 2, ny);
    const long long col = gx + (long long)nx * gy;
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
    const long long fcol = has_frame
        ? wrapmod(x0 + fx - 4, nx) + (long long)nx * wrapmod(y0 + fy - 4, ny) : 0;

    R ur[5][3];        // u at planes lead-4 .. lead
    R rr[3];           // rho at planes lead-2 .. lead
    R qz[5][3];        // q_xz, q_yz, q_zz at planes c-4 .. c
    R sd[3][3];        // x,y part of d_b q_ab at planes c-2 .. c
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) { ur[k][a] = R(0); qz[k][a] = R(0); }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        rr[k] = R(1);
#pragma unroll
        for (int a = 0; a < 3; ++a) sd[k][a] = R(0);
    }
    double dmax = 0.0;
    const R c12 = R(1.0 / 12.0);

    // one-plane lookahead: the inputs of step k+1 are loaded while step k
    // computes (own point at the lead plane, frame point at the centre plane)
    // (raw values are kept: combining them at load time would make the
    // compiler wait for the loads right away)
    R nr = R(1), nj[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    R fr = R(1), fj[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    R no[3] = {R(0), R(0), R(0)};   // j~ at the output plane of that step
    auto load_step = [&](int k) {
        if (k >= 8 && owned && z0 + k - 8 < nz) {
            const long long io = col + plane * (z0 + k - 8);
#pragma unroll
            for (int a = 0; a < 3; ++a) no[a] = jt_old[a * N + io];
        }
        const long long i = col + plane * wrap3(z0 - 4 + k, nz);
        nr = rho[i];
#pragma unroll
        for (int a = 0; a < 3; ++a) { nj[a] = j0p[a * N + i]; nj[3 + a] = jt_old[a * N + i]; }
        if (has_frame) {
            const long long f = fcol + plane * wrap3(z0 - 6 + k, nz);
            fr = rho[f];
#pragma unroll
            for (int a = 0; a < 3; ++a) { fj[a] = j0p[a * N + f]; fj[3 + a] = jt_old[a * N + f]; }
        }
    };
    load_step(0);

    for (int k = 0; k < TZ + 8; ++k) {
        // 1. lead plane at this thread's point: u = (j0' + j~)/rho
        const R r = nr;
        const R cur_j[3] = {nj[0] + nj[3], nj[1] + nj[4], nj[2] + nj[5]};
        const R cur_fr = fr;
        const R cur_fj[3] = {fj[0] + fj[3], fj[1] + fj[4], fj[2] + fj[5]};
        const R cur_o[3] = {no[0], no[1], no[2]};
        if (k + 1 < TZ + 8) load_step(k + 1);
        {
            const R inv = R(1) / r;
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int a = 0; a < 3; ++a) ur[s][a] = ur[s + 1][a];
#pragma unroll
            for (int a = 0; a < 3; ++a) ur[4][a] = cur_j[a] * inv;
            rr[0] = rr[1]; rr[1] = rr[2]; rr[2] = r;
        }
        // 2. u plane c = lead-2 into LDS: own point and frame point
#pragma unroll
        for (int a = 0; a < 3; ++a) su[a][ly + 2][lx + 2] = ur[2][a];
        if (has_frame) {
            const R inv = R(1) / cur_fr;
#pragma unroll
            for (int a = 0; a < 3; ++a) su[a][fy][fx] = cur_fj[a] * inv;
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
            const R trG = G[0][0] + G[1][1] + G[2][2];
            const EosVal<R> e = eos_all<R>(cf.eos, rr[0]);
            const R qxx = e.P1 * trG + R(2) * e.p * G[0][0];
            const R qyy = e.P1 * trG + R(2) * e.p * G[1][1];
            const R qzz = e.P1 * trG + R(2) * e.p * G[2][2];
            const R qxy = e.p * (G[0][1] + G[1][0]);
            const R qxz = e.p * (G[0][2] + G[2][0]);
            const R qyz = e.p * (G[1][2] + G[2][1]);
            sq[0][ly][lx] = qxx; sq[1][ly][lx] = qyy; sq[2][ly][lx] = qzz;
            sq[3][ly][lx] = qxy; sq[4][ly][lx] = qxz; sq[5][ly][lx] = qyz;
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int a = 0; a < 3; ++a) qz[s][a] = qz[s + 1][a];
            qz[4][0] = qxz; qz[4][1] = qyz; qz[4][2] = qzz;
        }
        __syncthreads();
        // 4. j~new at plane c-2 = z0 + k - 8
        if (k >= 4 && interior) {
            // x,y part at plane c: sym2 index of (a, x) and (a, y)
            const int px = lx, py = ly;
            R S[3];
            // a = x: d_x q_xx + d_y q_xy ; a = y: d_x q_xy + d_y q_yy ; a = z: d_x q_xz + d_y q_yz
            S[0] = d1<R>(sq[0][py][px - 2], sq[0][py][px - 1], sq[0][py][px + 1], sq[0][py][px + 2]) +
                   d1<R>(sq[3][py - 2][px], sq[3][py - 1][px], sq[3][py + 1][px], sq[3][py + 2][px]);
            S[1] = d1<R>(sq[3][py][px - 2], sq[3][py][px - 1], sq[3][py][px + 1], sq[3][py][px + 2]) +
                   d1<R>(sq[1][py - 2][px], sq[1][py - 1][px], sq[1][py + 1][px], sq[1][py + 2][px]);
            S[2] = d1<R>(sq[4][py][px - 2], sq[4][py][px - 1], sq[4][py][px + 1], sq[4][py][px + 2]) +
                   d1<R>(sq[5][py - 2][px], sq[5][py - 1][px], sq[5][py + 1][px], sq[5][py + 2][px]);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                sd[0][a] = sd[1][a];
                sd[1][a] = sd[2][a];
                sd[2][a] = S[a];
            }
            const int zo = z0 + k - 8;
            if (k >= 8 && owned && zo < z0 + TZ && zo < nz) {
                const long long i = col + plane * zo;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const R dz = d1<R>(qz[0][a], qz[1][a], qz[3][a], qz[4][a]);
                    const R jn = -(sd[0][a] + dz) * c12;
                    dmax = fmax(dmax, fabs((double)(jn - cur_o[a])));
                    jt_new[a * N + i] = jn;
                }
            }
        }
    }
    block_max_to(ic.res + (long long)tl.dom * ic.stride + it, dmax);
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

}  // namespace lb2p
