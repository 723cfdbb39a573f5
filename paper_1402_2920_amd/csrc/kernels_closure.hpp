// kernels_closure.hpp -- the closure kernels (items 9-11): for D3Q59 as
// z-marches, k_closure1_zm (the level-1 fields X, T, Y and Xi' from first
// derivatives of u, p and per-site products) and k_closure2_zm (Sigma from the
// derivatives of X, T, Y); for D2Q21 on LDS tiles, k_closure1_t2 and
// k_closure2_t2 (at the end of this file).  The force kernels of item 2,
// k_force_zm (3D) and k_force_t2 (2D), are here too.
//
// A block owns a TX x TY tile of an xy plane (one thread per tile point) and
// marches through TZ planes of z, like the fused solve pass.  Each thread
// keeps, in registers, five planes (c-2 .. c+2) of the fields whose z
// derivative is taken at its point; one plane of the fields with x or y
// derivatives (tile + 2-wide frame) sits in LDS.  Every input word is then
// read once per launch (plus the frame), where a per-site kernel issues four
// neighbour loads per field and direction (70 to 150 loads per site).
#pragma once

#include "kernels_fused.hpp"

namespace lb2p {

// Inputs of one z step.
template <class R>
struct C2In {
    R lead[11];   // own point, lead plane c+2: X, Txz, Tyz, Tzz, Yx, Yy, Yz, rho, ux, uy, uz
    R own[3];     // own point, centre plane: Txx, Txy, Tyy (no z derivative)
    R fr[13];     // frame point, centre plane: X, Txx, Txy, Tyy, Txz, Tyz, Yx, Yy, Yz, rho, ux, uy, uz
};

template <class R, int TX, int TY>
__global__ void __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 1)))
k_closure2_zm(const Domain* __restrict__ tab, const Tile* __restrict__ tiles, const R* __restrict__ rho,
              const R* __restrict__ u, const R* __restrict__ X, const R* __restrict__ T,
              const R* __restrict__ Y, R* __restrict__ Sig, const int* __restrict__ go)
{
    constexpr int UX = TX + 4, UY = TY + 4;   // tile + 2-wide frame
    constexpr int NFRAME = UX * UY - TX * TY;
    static_assert(NFRAME <= TX * TY, "frame larger than the block");
    // planar fields: X, Txx, Txy, Tyy, Txz, Tyz, Yx, Yy, Yz, rho ux, rho uy, ux, uy, uz
    __shared__ R sl[14][UY][UX];

    if (*go == 0) return;   // the solve is not finished (launched ahead of the host's check)
    const Tile tl = tiles[blockIdx.x];
    if (tl.dom < 0) return;   // uniform per block
    const Domain& dm = tab[tl.dom];
    const int nx = dm.g.nx, ny = dm.g.ny, nz = dm.g.nz;
    const long long N = dm.g.S;
    const unsigned plane = (unsigned)nx * (unsigned)ny;
    const unsigned bytes = (unsigned)dm.g.N * (unsigned)sizeof(R);
    const unsigned OUT = bytes;
    const long long o = dm.off;
    const PlaneBuf bX = plane_buf(X + o, bytes);
    // T and Sigma components: xx yy zz xy xz yz
    const PlaneBuf bT[6] = {plane_buf(T + o, bytes), plane_buf(T + o + N, bytes), plane_buf(T + o + 2 * N, bytes),
                            plane_buf(T + o + 3 * N, bytes), plane_buf(T + o + 4 * N, bytes),
                            plane_buf(T + o + 5 * N, bytes)};
    const PlaneBuf bY[3] = {plane_buf(Y + o, bytes), plane_buf(Y + o + N, bytes), plane_buf(Y + o + 2 * N, bytes)};
    const PlaneBuf bR = plane_buf(rho + o, bytes);
    const PlaneBuf bU[3] = {plane_buf(u + o, bytes), plane_buf(u + o + N, bytes), plane_buf(u + o + 2 * N, bytes)};
    const PlaneBuf bS[6] = {plane_buf(Sig + o, bytes), plane_buf(Sig + o + N, bytes),
                            plane_buf(Sig + o + 2 * N, bytes), plane_buf(Sig + o + 3 * N, bytes),
                            plane_buf(Sig + o + 4 * N, bytes), plane_buf(Sig + o + 5 * N, bytes)};

    const int lx = threadIdx.x, ly = threadIdx.y;
    const int tid = lx + TX * ly;
    const int x0 = tl.x0, y0 = tl.y0, z0 = tl.z0, TZ = tl.len;
    const unsigned col = (unsigned)wrapmod(x0 + lx, nx) + (unsigned)nx * (unsigned)wrapmod(y0 + ly, ny);
    const bool owned = (x0 + lx < nx) && (y0 + ly < ny);

    // this thread's frame point (2-wide ring of the UX x UY region)
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
            const int c = t % 4;
            fy = 2 + t / 4;
            fx = c < 2 ? c : UX - 4 + c;
        }
    }
    const unsigned fcol = has_frame
        ? (unsigned)wrapmod(x0 + fx - 2, nx) + (unsigned)nx * (unsigned)wrapmod(y0 + fy - 2, ny) : 0u;

    // Step k: lead plane z0-2+k, centre plane c = z0-4+k, output at c for
    // 4 <= k < TZ+4.  The ring holds planes c-2 .. c+2 after the shift.
    const int nsteps = TZ + 4;
    auto load_lead = [&](int k, C2In<R>& in) {
        const unsigned i = k < nsteps ? (col + plane * (unsigned)wrap3(z0 - 2 + k, nz)) * (unsigned)sizeof(R) : OUT;
        in.lead[0] = bload<R>(bX, i);
        in.lead[1] = bload<R>(bT[4], i);
        in.lead[2] = bload<R>(bT[5], i);
        in.lead[3] = bload<R>(bT[2], i);
#pragma unroll
        for (int b = 0; b < 3; ++b) in.lead[4 + b] = bload<R>(bY[b], i);
        in.lead[7] = bload<R>(bR, i);
#pragma unroll
        for (int b = 0; b < 3; ++b) in.lead[8 + b] = bload<R>(bU[b], i);
    };
    auto load_centre = [&](int k, C2In<R>& in) {
        const bool live = k >= 4 && k < nsteps;   // LDS is read from step 4 on
        const unsigned zc = plane * (unsigned)wrap3(z0 - 4 + k, nz);
        const unsigned i = live ? (col + zc) * (unsigned)sizeof(R) : OUT;
        in.own[0] = bload<R>(bT[0], i);
        in.own[1] = bload<R>(bT[3], i);
        in.own[2] = bload<R>(bT[1], i);
        const unsigned f = live && has_frame ? (fcol + zc) * (unsigned)sizeof(R) : OUT;
        in.fr[0] = bload<R>(bX, f);
        in.fr[1] = bload<R>(bT[0], f);
        in.fr[2] = bload<R>(bT[3], f);
        in.fr[3] = bload<R>(bT[1], f);
        in.fr[4] = bload<R>(bT[4], f);
        in.fr[5] = bload<R>(bT[5], f);
#pragma unroll
        for (int b = 0; b < 3; ++b) in.fr[6 + b] = bload<R>(bY[b], f);
        in.fr[9] = bload<R>(bR, f);
#pragma unroll
        for (int b = 0; b < 3; ++b) in.fr[10 + b] = bload<R>(bU[b], f);
    };

    R rg[5][11];
#pragma unroll
    for (int s = 0; s < 5; ++s)
#pragma unroll
        for (int f = 0; f < 11; ++f) rg[s][f] = R(0);

    const R gm = R(dm.cf.gamma);
    const R KS1 = R(-0.25) * (gm + R(1)) * (gm + R(1)) / (gm - R(1));
    const R KS2 = (gm * gm + R(4) * gm + R(1)) / (R(6) * (gm - R(1)));

    C2In<R> in;
    load_lead(0, in);
    for (int k = 0; k < nsteps; ++k) {
        // centre-plane inputs of this step (the lead plane was loaded one step
        // ahead; holding these across a step as well costs registers that
        // would spill)
        load_centre(k, in);
        // 1. ring shift; the lead plane comes in
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int f = 0; f < 11; ++f) rg[s][f] = rg[s + 1][f];
#pragma unroll
        for (int f = 0; f < 11; ++f) rg[4][f] = in.lead[f];
        load_lead(k + 1, in);
        // 2. the centre plane into LDS: own point and frame point
        {
            const int py = ly + 2, px = lx + 2;
            sl[0][py][px] = rg[2][0];
            sl[1][py][px] = in.own[0];
            sl[2][py][px] = in.own[1];
            sl[3][py][px] = in.own[2];
            sl[4][py][px] = rg[2][1];
            sl[5][py][px] = rg[2][2];
            sl[6][py][px] = rg[2][4];
            sl[7][py][px] = rg[2][5];
            sl[8][py][px] = rg[2][6];
            sl[9][py][px] = rg[2][7] * rg[2][8];
            sl[10][py][px] = rg[2][7] * rg[2][9];
            sl[11][py][px] = rg[2][8];
            sl[12][py][px] = rg[2][9];
            sl[13][py][px] = rg[2][10];
        }
        if (has_frame) {
#pragma unroll
            for (int f = 0; f < 9; ++f) sl[f][fy][fx] = in.fr[f];
            sl[9][fy][fx] = in.fr[9] * in.fr[10];
            sl[10][fy][fx] = in.fr[9] * in.fr[11];
#pragma unroll
            for (int b = 0; b < 3; ++b) sl[11 + b][fy][fx] = in.fr[10 + b];
        }
        __syncthreads();
        // 3. Sigma at the centre plane (item 11)
        const bool out = owned && k >= 4 && z0 + k - 4 < nz;
        R sg[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
        if (k >= 4) {
            const int py = ly + 2, px = lx + 2;
            auto dx = [&](int f) {
                return d1<R>(sl[f][py][px - 2], sl[f][py][px - 1], sl[f][py][px + 1], sl[f][py][px + 2]);
            };
            auto dy = [&](int f) {
                return d1<R>(sl[f][py - 2][px], sl[f][py - 1][px], sl[f][py + 1][px], sl[f][py + 2][px]);
            };
            auto dz = [&](int f) { return d1<R>(rg[0][f], rg[1][f], rg[3][f], rg[4][f]); };
            // (groups of derivatives are kept apart, so that the LDS reads
            // of one group are not all hoisted ahead and held in registers)
            const R r = rg[2][7];
            const EosVal<R> e = eos_all<R>(dm.cf.eos, r);
            __builtin_amdgcn_sched_barrier(0);
            const R DX[3] = {dx(0), dy(0), dz(0)};
            R DT[3];
            DT[0] = dx(1) + dy(2) + dz(1);
            DT[1] = dx(2) + dy(3) + dz(2);
            DT[2] = dx(4) + dy(5) + dz(3);
            __builtin_amdgcn_sched_barrier(0);
            R DY[3][3];   // DY[a][b] = d_a Y_b
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                DY[0][b] = dx(6 + b);
                DY[1][b] = dy(6 + b);
                DY[2][b] = dz(4 + b);
            }
            __builtin_amdgcn_sched_barrier(0);
            const R trJ = dx(9) + dy(10) +
                          d1<R>(rg[0][7] * rg[0][10], rg[1][7] * rg[1][10], rg[3][7] * rg[3][10],
                                rg[4][7] * rg[4][10]);
            R G[3][3];    // G[a][b] = d_a u_b
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                G[0][b] = dx(11 + b);
                G[1][b] = dy(11 + b);
                G[2][b] = dz(8 + b);
            }
            __builtin_amdgcn_sched_barrier(0);
            const R us[3] = {rg[2][8], rg[2][9], rg[2][10]};
            const R trG = G[0][0] + G[1][1] + G[2][2];
            const R trDY = DY[0][0] + DY[1][1] + DY[2][2];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = a; b < 3; ++b) {
                    const R br1 = us[a] * DX[b] + us[b] * DX[a] + us[b] * DT[a] + us[a] * DT[b];
                    R br2 = -e.dp * trJ * (G[a][b] + G[b][a]) - e.p * (DY[a][b] + DY[b][a]);
                    if (a == b) br2 += -e.P1 * trDY + e.P2 * trG * trJ;
                    sg[sym2<3>(a, b)] = KS1 * br1 + KS2 * br2;
                }
        }
        // every lane stores; lanes without an output point write nowhere
        const unsigned io = out ? (col + plane * (unsigned)(z0 + k - 4)) * (unsigned)sizeof(R) : OUT;
#pragma unroll
        for (int s = 0; s < 6; ++s) bstore<R>(bS[s], io, sg[s]);
        __syncthreads();
    }
}

// Items 9-10 and the Xi' part of item 11: per site X = P1 d_g u_g,
// T_ag = p (d_a u_g + d_g u_a), Y_b = rho^-1 d_b p + u_g d_g u_b and Xi'
// from d_a (p u_b u_g), d_a (p/rho) and j~ (per site, the same terms in the
// same order as the 2D k_closure1_t2).
template <class R>
struct C1In {
    R lead[5];    // own point, lead plane c+2: ux, uy, uz, p - p_ref, c_s^2 - c_s^2_ref
    R own[6];     // own point, centre plane: P1, then rho and j0' (form) or j~, then 1/rho
    R fr[5];      // frame point, centre plane: ux, uy, uz, p - p_ref, c_s^2 - c_s^2_ref
};

template <class R, int TX, int TY>
__global__ void __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 1)))
k_closure1_zm(const Domain* __restrict__ tab, const Tile* __restrict__ tiles,
              const SolveInfo* __restrict__ info, const R* __restrict__ pf, const R* __restrict__ rho,
              const R* __restrict__ j0p, R* u0, const R* u1, R* jtA, R* jtB, R* __restrict__ X,
              R* __restrict__ T, R* __restrict__ Y, R* __restrict__ Xi, int form,
              const int* __restrict__ go)
{
    if (*go == 0) return;   // the solve is not finished (launched ahead of the host's check)
    // form = 1 (after a velocity-form solve): the final iterate is u in u0
    // or u1 (by the pass count); j~ = rho u - j0' is formed here at each site
    // (item 7) and stored in the j~ buffer the pass count selects, and u is
    // copied to u0 when it ended in u1.  form = 0: u0 and that j~ buffer
    // already hold the final values.
    constexpr int UX = TX + 4, UY = TY + 4;   // tile + 2-wide frame
    constexpr int NFRAME = UX * UY - TX * TY;
    static_assert(NFRAME <= TX * TY, "frame larger than the block");
    // planar fields: ux, uy, uz, p, p/rho, then p u_b u_c for (b,c) = xx xy xz yy yz zz
    __shared__ R sl[11][UY][UX];

    const Tile tl = tiles[blockIdx.x];
    if (tl.dom < 0) return;   // uniform per block
    const Domain& dm = tab[tl.dom];
    const int nx = dm.g.nx, ny = dm.g.ny, nz = dm.g.nz;
    const long long N = dm.g.S;
    const unsigned plane = (unsigned)nx * (unsigned)ny;
    const unsigned bytes = (unsigned)dm.g.N * (unsigned)sizeof(R);
    const unsigned OUT = bytes;
    const long long o = dm.off;
    const bool odd = info[tl.dom].final_buf != 0;   // uniform per block
    R* const jt = odd ? jtB : jtA;
    const R* const u = (form && odd) ? u1 : u0;
    const PlaneBuf bU[3] = {plane_buf(u + o, bytes), plane_buf(u + o + N, bytes), plane_buf(u + o + 2 * N, bytes)};
    const PlaneBuf bP = plane_buf(pf + o, bytes);             // p - p_ref
    const PlaneBuf bP1 = plane_buf(pf + o + N, bytes);
    const PlaneBuf bRi = plane_buf(pf + o + 2 * N, bytes);
    const PlaneBuf bC = plane_buf(pf + o + 3 * N, bytes);     // c_s^2 - c_s^2_ref
    const R pref = R(dm.cf.pref);
    const PlaneBuf bJ[3] = {plane_buf(jt + o, bytes), plane_buf(jt + o + N, bytes), plane_buf(jt + o + 2 * N, bytes)};
    const PlaneBuf bRho = plane_buf(rho + o, bytes);
    const PlaneBuf bJ0[3] = {plane_buf(j0p + o, bytes), plane_buf(j0p + o + N, bytes),
                             plane_buf(j0p + o + 2 * N, bytes)};
    const PlaneBuf bU0[3] = {plane_buf(u0 + o, bytes), plane_buf(u0 + o + N, bytes), plane_buf(u0 + o + 2 * N, bytes)};
    const PlaneBuf bX = plane_buf(X + o, bytes);
    const PlaneBuf bT[6] = {plane_buf(T + o, bytes), plane_buf(T + o + N, bytes), plane_buf(T + o + 2 * N, bytes),
                            plane_buf(T + o + 3 * N, bytes), plane_buf(T + o + 4 * N, bytes),
                            plane_buf(T + o + 5 * N, bytes)};
    const PlaneBuf bY[3] = {plane_buf(Y + o, bytes), plane_buf(Y + o + N, bytes), plane_buf(Y + o + 2 * N, bytes)};
    PlaneBuf bXi[10];
#pragma unroll
    for (int s = 0; s < 10; ++s) bXi[s] = plane_buf(Xi + o + s * N, bytes);

    const int lx = threadIdx.x, ly = threadIdx.y;
    const int tid = lx + TX * ly;
    const int x0 = tl.x0, y0 = tl.y0, z0 = tl.z0, TZ = tl.len;
    const unsigned col = (unsigned)wrapmod(x0 + lx, nx) + (unsigned)nx * (unsigned)wrapmod(y0 + ly, ny);
    const bool owned = (x0 + lx < nx) && (y0 + ly < ny);

    int fx = 0, fy = 0;
    const bool has_frame = tid < NFRAME;
    if (has_frame) {
        if (tid < 2 * UX) {
            fy = tid / UX; fx = tid % UX;
        } else if (tid < 4 * UX) {
            const int t = tid - 2 * UX;
            fy = UY - 2 + t / UX; fx = t % UX;
        } else {
            const int t = tid - 4 * UX;
            const int c = t % 4;
            fy = 2 + t / 4;
            fx = c < 2 ? c : UX - 4 + c;
        }
    }
    const unsigned fcol = has_frame
        ? (unsigned)wrapmod(x0 + fx - 2, nx) + (unsigned)nx * (unsigned)wrapmod(y0 + fy - 2, ny) : 0u;

    const int nsteps = TZ + 4;
    auto load_lead = [&](int k, C1In<R>& in) {
        const unsigned i = k < nsteps ? (col + plane * (unsigned)wrap3(z0 - 2 + k, nz)) * (unsigned)sizeof(R) : OUT;
#pragma unroll
        for (int b = 0; b < 3; ++b) in.lead[b] = bload<R>(bU[b], i);
        in.lead[3] = bload<R>(bP, i);
        in.lead[4] = bload<R>(bC, i);
    };
    auto load_centre = [&](int k, C1In<R>& in) {
        const bool live = k >= 4 && k < nsteps;
        const unsigned zc = plane * (unsigned)wrap3(z0 - 4 + k, nz);
        const unsigned i = live ? (col + zc) * (unsigned)sizeof(R) : OUT;
        in.own[0] = bload<R>(bP1, i);
        if (form) {
            in.own[1] = bload<R>(bRho, i);
#pragma unroll
            for (int b = 0; b < 3; ++b) in.own[2 + b] = bload<R>(bJ0[b], i);
        } else {
#pragma unroll
            for (int b = 0; b < 3; ++b) in.own[1 + b] = bload<R>(bJ[b], i);
            in.own[4] = R(0);
        }
        in.own[5] = bload<R>(bRi, i);
        const unsigned f = live && has_frame ? (fcol + zc) * (unsigned)sizeof(R) : OUT;
#pragma unroll
        for (int b = 0; b < 3; ++b) in.fr[b] = bload<R>(bU[b], f);
        in.fr[3] = bload<R>(bP, f);
        in.fr[4] = bload<R>(bC, f);
    };
    // planar LDS fields of one point (pd = p - p_ref, cd = c_s^2 - c_s^2_ref:
    // first derivatives of p and p/rho are those of the deviations)
    auto put = [&](int py, int px, R ux, R uy, R uz, R pd, R cd) {
        const R p = pref + pd;
        sl[0][py][px] = ux;
        sl[1][py][px] = uy;
        sl[2][py][px] = uz;
        sl[3][py][px] = pd;
        sl[4][py][px] = cd;
        sl[5][py][px] = p * ux * ux;
        sl[6][py][px] = p * ux * uy;
        sl[7][py][px] = p * ux * uz;
        sl[8][py][px] = p * uy * uy;
        sl[9][py][px] = p * uy * uz;
        sl[10][py][px] = p * uz * uz;
    };

    R rg[5][5];   // ux, uy, uz, p - p_ref, c_s^2 - c_s^2_ref at planes c-2 .. c+2
#pragma unroll
    for (int s = 0; s < 5; ++s)
#pragma unroll
        for (int f = 0; f < 5; ++f) rg[s][f] = R(0);

    const R gm = R(dm.cf.gamma);
    const R KX = (gm * gm + R(4) * gm + R(1)) / (R(3) * (gm + R(1)));
    const R KJ = (R(1) - gm) * R(dm.cf.c0sq);

    C1In<R> in;
    load_lead(0, in);
    load_centre(0, in);
    for (int k = 0; k < nsteps; ++k) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int f = 0; f < 5; ++f) rg[s][f] = rg[s + 1][f];
#pragma unroll
        for (int f = 0; f < 5; ++f) rg[4][f] = in.lead[f];
        load_lead(k + 1, in);
        put(ly + 2, lx + 2, rg[2][0], rg[2][1], rg[2][2], rg[2][3], rg[2][4]);
        if (has_frame) put(fy, fx, in.fr[0], in.fr[1], in.fr[2], in.fr[3], in.fr[4]);
        // the centre-plane inputs of the next step load while this one computes
        const R own[6] = {in.own[0], in.own[1], in.own[2], in.own[3], in.own[4], in.own[5]};
        load_centre(k + 1, in);
        __syncthreads();
        const bool out = owned && k >= 4 && z0 + k - 4 < nz;
        R oX = R(0), oT[6] = {}, oY[3] = {}, oXi[10] = {}, oJ[3] = {};
        if (k >= 4) {
            const int py = ly + 2, px = lx + 2;
            auto dxl = [&](int f) {
                return d1<R>(sl[f][py][px - 2], sl[f][py][px - 1], sl[f][py][px + 1], sl[f][py][px + 2]);
            };
            auto dyl = [&](int f) {
                return d1<R>(sl[f][py - 2][px], sl[f][py - 1][px], sl[f][py + 1][px], sl[f][py + 2][px]);
            };
            // z derivatives from the ring; products formed per plane (items 9-10)
            auto dzr = [&](int f) { return d1<R>(rg[0][f], rg[1][f], rg[3][f], rg[4][f]); };
            auto dzm = [&](int b, int c) {
                return d1<R>((pref + rg[0][3]) * rg[0][b] * rg[0][c], (pref + rg[1][3]) * rg[1][b] * rg[1][c],
                             (pref + rg[3][3]) * rg[3][b] * rg[3][c], (pref + rg[4][3]) * rg[4][b] * rg[4][c]);
            };
            R G[3][3];      // d_a u_b
            R M[3][3][3];   // d_a (p u_b u_c)
            R Pg[3], C[3];  // d_a p, d_a (p/rho)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                G[0][b] = dxl(b);
                G[1][b] = dyl(b);
                G[2][b] = dzr(b);
            }
            Pg[0] = dxl(3); Pg[1] = dyl(3); Pg[2] = dzr(3);
            C[0] = dxl(4); C[1] = dyl(4); C[2] = dzr(4);
            constexpr int PI[3][3] = {{5, 6, 7}, {6, 8, 9}, {7, 9, 10}};
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int c = b; c < 3; ++c) {
                    const R mx = dxl(PI[b][c]), my = dyl(PI[b][c]), mz = dzm(b, c);
                    M[0][b][c] = mx; M[0][c][b] = mx;
                    M[1][b][c] = my; M[1][c][b] = my;
                    M[2][b][c] = mz; M[2][c][b] = mz;
                }
            const R ep = pref + rg[2][3], inv = own[5], eP1 = own[0];
            const R us[3] = {rg[2][0], rg[2][1], rg[2][2]};
            const R trG = G[0][0] + G[1][1] + G[2][2];
            oX = eP1 * trG;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int c = a; c < 3; ++c) oT[sym2<3>(a, c)] = ep * (G[a][c] + G[c][a]);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                R acc = Pg[b] * inv;
#pragma unroll
                for (int c = 0; c < 3; ++c) acc += us[c] * G[c][b];
                oY[b] = acc;
            }
            R jts[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                // item 7: j~ = j - j0' with j = rho u
                jts[a] = form ? own[1] * us[a] - own[2 + a] : own[1 + a];
                oJ[a] = jts[a];
            }
            R V[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) V[a] = ep * C[a] + eP1 * us[a] * trG;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = a; b < 3; ++b)
#pragma unroll
                    for (int c = b; c < 3; ++c) {
                        R br = M[c][a][b] + M[b][a][c] + M[a][b][c];
                        R dj = R(0);
                        if (a == b) { br += V[c]; dj += jts[c]; }
                        if (a == c) { br += V[b]; dj += jts[b]; }
                        if (b == c) { br += V[a]; dj += jts[a]; }
                        oXi[sym3<3>(a, b, c)] = KX * br + KJ * dj;
                    }
        }
        const unsigned io = out ? (col + plane * (unsigned)(z0 + k - 4)) * (unsigned)sizeof(R) : OUT;
        bstore<R>(bX, io, oX);
#pragma unroll
        for (int s = 0; s < 6; ++s) bstore<R>(bT[s], io, oT[s]);
#pragma unroll
        for (int b = 0; b < 3; ++b) bstore<R>(bY[b], io, oY[b]);
#pragma unroll
        for (int s = 0; s < 10; ++s) bstore<R>(bXi[s], io, oXi[s]);
        {
            const unsigned ij = form ? io : OUT, iu = (form && odd) ? io : OUT;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                bstore<R>(bJ[a], ij, oJ[a]);
                bstore<R>(bU0[a], iu, rg[2][a]);
            }
        }
        __syncthreads();
    }
}

// Item 2 for D3Q59 as a z-march: f = kappa rho (sum over the force stencil of
// Table III of tau_i d_i rho(r + d_i)), j0' = j0 + f/2 and the start of the
// iteration (per site, the same terms as k_force_t2 in 2D).  The stencil reaches (+-1, 0, 0), (+-1, +-1, 0)
// and (+-2, 0, 0) and their permutations, so three planes of rho (c-1, c,
// c+1, tile + 2-wide frame) sit in LDS and the column's rho at c-2 .. c+2 in
// registers.
template <class R, int TX, int TY>
__global__ void __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 1)))
k_force_zm(const Domain* __restrict__ tab, const Tile* __restrict__ tiles, IterCtl ic,
           const double* __restrict__ mass, const R* __restrict__ j0, R* __restrict__ f, R* __restrict__ j0p,
           R* __restrict__ u, const R* jt_prevA, const R* jt_prevB, const SolveInfo* prev_info, R* jt0,
           R* hist, R* hist2, int order)
{
    constexpr int UX = TX + 4, UY = TY + 4;
    constexpr int NFRAME = UX * UY - TX * TY;
    static_assert(NFRAME <= TX * TY, "frame larger than the block");
    // The stencil runs in FP64 on the FP64 mass of item 1: the force is a
    // third derivative of a field of size 1 whose differences are small, so
    // an FP32 rho (or its FP32 deviation) would leave rounding noise of the
    // size of the force's own FP32 resolution in every step's momentum.
    __shared__ double sr[3][UY][UX];   // rho at planes (slot = plane mod 3)

    const Tile tl = tiles[blockIdx.x];
    double amax = 0.0;
    if (tl.dom >= 0) {
        const Domain& dm = tab[tl.dom];
        const int nx = dm.g.nx, ny = dm.g.ny, nz = dm.g.nz;
        const long long N = dm.g.S;
        const unsigned plane = (unsigned)nx * (unsigned)ny;
        const unsigned bytes = (unsigned)dm.g.N * (unsigned)sizeof(R);
        const unsigned OUT = bytes;
        const long long o = dm.off;
        const unsigned mbytes = (unsigned)dm.g.N * 8u;
        const PlaneBuf bM = plane_buf(mass + o, mbytes);
        const R* prev = nullptr;
        if (prev_info) prev = prev_info[tl.dom].final_buf ? jt_prevB : jt_prevA;

        const int lx = threadIdx.x, ly = threadIdx.y;
        const int tid = lx + TX * ly;
        const int x0 = tl.x0, y0 = tl.y0, z0 = tl.z0, TZ = tl.len;
        const unsigned col = (unsigned)wrapmod(x0 + lx, nx) + (unsigned)nx * (unsigned)wrapmod(y0 + ly, ny);
        const bool owned = (x0 + lx < nx) && (y0 + ly < ny);
        int fx = 0, fy = 0;
        const bool has_frame = tid < NFRAME;
        if (has_frame) {
            if (tid < 2 * UX) {
                fy = tid / UX; fx = tid % UX;
            } else if (tid < 4 * UX) {
                const int t = tid - 2 * UX;
                fy = UY - 2 + t / UX; fx = t % UX;
            } else {
                const int t = tid - 4 * UX;
                const int c = t % 4;
                fy = 2 + t / 4;
                fx = c < 2 ? c : UX - 4 + c;
            }
        }
        const unsigned fcol = has_frame
            ? (unsigned)wrapmod(x0 + fx - 2, nx) + (unsigned)nx * (unsigned)wrapmod(y0 + fy - 2, ny) : 0u;

        // Step k: the column's lead plane z0-2+k enters the ring, plane
        // c+1 = z0-3+k enters LDS, output at c = z0-4+k for 4 <= k < TZ+4.
        const int nsteps = TZ + 4;
        auto lead_off = [&](int k) {
            return k < nsteps ? (col + plane * (unsigned)wrap3(z0 - 2 + k, nz)) * 8u : mbytes;
        };
        auto frame_off = [&](int k) {
            return has_frame && k >= 2 && k < nsteps
                ? (fcol + plane * (unsigned)wrap3(z0 - 3 + k, nz)) * 8u : mbytes;
        };
        double rg[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // the column's rho at c-2 .. c+2
        // own-point inputs of step k (j0 and the previous j~ at plane c),
        // loaded a step ahead like rho
        const PlaneBuf bJ0[3] = {plane_buf(j0 + o, bytes), plane_buf(j0 + o + N, bytes),
                                 plane_buf(j0 + o + 2 * N, bytes)};
        const R* const pv = prev ? prev : j0;   // any valid plane when there is no previous j~
        const PlaneBuf bPv[3] = {plane_buf(pv + o, bytes), plane_buf(pv + o + N, bytes),
                                 plane_buf(pv + o + 2 * N, bytes)};
        auto own_off = [&](int k) {
            return owned && k >= 4 && k < nsteps && z0 + k - 4 < nz
                ? (col + plane * (unsigned)(z0 + k - 4)) * (unsigned)sizeof(R) : OUT;
        };
        R nj[3], np_[3];
        auto load_own = [&](int k) {
            const unsigned i = own_off(k);
            const unsigned ip = prev ? i : OUT;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                nj[a] = bload<R>(bJ0[a], i);
                np_[a] = bload<R>(bPv[a], ip);
            }
        };
        double nlead = bload<double>(bM, lead_off(0));
        double nfr = bload<double>(bM, frame_off(0));
        load_own(0);
        for (int k = 0; k < nsteps; ++k) {
#pragma unroll
            for (int s = 0; s < 4; ++s) rg[s] = rg[s + 1];
            rg[4] = nlead;
            const double fr = nfr;
            const R cj[3] = {nj[0], nj[1], nj[2]}, cp[3] = {np_[0], np_[1], np_[2]};
            nlead = bload<double>(bM, lead_off(k + 1));
            nfr = bload<double>(bM, frame_off(k + 1));
            load_own(k + 1);
            // plane c+1 = z0-3+k into its LDS slot
            const int slot = (k + 3) % 3;   // (z0 - 3 + k) mod 3 relative to z0: slots follow k
            sr[slot][ly + 2][lx + 2] = rg[3];
            if (has_frame) sr[slot][fy][fx] = fr;
            __syncthreads();
            const int zc = z0 + k - 4;
            if (k >= 4 && owned && zc < nz) {
                const int sc = (k + 2) % 3, sm = (k + 1) % 3, sp = slot;   // planes c, c-1, c+1
                const int py = ly + 2, px = lx + 2;
                auto RH = [&](int dx, int dy, int dz) -> double {
                    if (dz == 0) return sr[sc][py + dy][px + dx];
                    if (dz == 1) return (dx == 0 && dy == 0) ? rg[3] : sr[sp][py + dy][px + dx];
                    if (dz == -1) return (dx == 0 && dy == 0) ? rg[1] : sr[sm][py + dy][px + dx];
                    return dz == 2 ? rg[4] : rg[0];
                };
                double fa[3];
                // (100): tau -3 ; (110): tau 1/2 ; (200): tau 1/4 (Table III)
                fa[0] = -3.0 * (RH(1, 0, 0) - RH(-1, 0, 0)) +
                        0.5 * (RH(1, 1, 0) + RH(1, -1, 0) + RH(1, 0, 1) + RH(1, 0, -1) -
                               RH(-1, 1, 0) - RH(-1, -1, 0) - RH(-1, 0, 1) - RH(-1, 0, -1)) +
                        0.5 * (RH(2, 0, 0) - RH(-2, 0, 0));
                fa[1] = -3.0 * (RH(0, 1, 0) - RH(0, -1, 0)) +
                        0.5 * (RH(1, 1, 0) + RH(-1, 1, 0) + RH(0, 1, 1) + RH(0, 1, -1) -
                               RH(1, -1, 0) - RH(-1, -1, 0) - RH(0, -1, 1) - RH(0, -1, -1)) +
                        0.5 * (RH(0, 2, 0) - RH(0, -2, 0));
                fa[2] = -3.0 * (RH(0, 0, 1) - RH(0, 0, -1)) +
                        0.5 * (RH(1, 0, 1) + RH(-1, 0, 1) + RH(0, 1, 1) + RH(0, -1, 1) -
                               RH(1, 0, -1) - RH(-1, 0, -1) - RH(0, 1, -1) - RH(0, -1, -1)) +
                        0.5 * (RH(0, 0, 2) - RH(0, 0, -2));
                const double r64 = rg[2];
                const double kr = dm.cf.kappa * r64;
                const R inv = R(1) / R(r64);   // as the 1/rho plane of item 1
                const long long i0 = o + col + (long long)plane * zc;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const long long ia = i0 + a * N;
                    const R fv = R(kr * fa[a]);
                    const R jp = cj[a] + R(0.5) * fv;
                    R jt = prev ? cp[a] : R(0);
                    if (hist) {
                        const R y1 = jt;
                        const R y2 = hist[ia];
                        hist[ia] = y1;
                        R y3 = R(0);
                        if (hist2) {
                            y3 = hist2[ia];
                            hist2[ia] = y2;
                        }
                        if (order == 2)
                            jt = y3 + R(3) * (y1 - y2);
                        else if (order == 1)
                            jt = R(2) * y1 - y2;
                    }
                    f[ia] = fv;
                    j0p[ia] = jp;
                    if (jt0) jt0[ia] = jt;
                    u[ia] = (jp + jt) * inv;
                    amax = fmax(amax, fabs((double)jp));
                }
            }
            __syncthreads();
        }
    }
    block_max_part(ic.part, amax);
}


// ---------------------------------------------------------------------------
// The closure kernels for D2Q21 on TX x TY tiles of a domain.  A block first
// copies the fields whose first derivatives it takes into LDS, for its tile
// and a 2-wide frame (one global load per field and point, where a per-site
// kernel loads every stencil neighbour: 4 per field and axis), then each
// thread evaluates its site from LDS.  Per site, the terms and their order
// are those of the per-site forms, so the results round the same way.
// ---------------------------------------------------------------------------

// Domain index of point k of the (TX+4) x (TY+4) tile-plus-frame region
// (periodic; a tile may reach past the domain's edge).
template <int UX>
__device__ __forceinline__ unsigned frame_site(int k, int x0, int y0, int nx, int ny)
{
    const int lx = k % UX, ly = k / UX;
    return (unsigned)wrapmod(x0 + lx - 2, nx) + (unsigned)nx * (unsigned)wrapmod(y0 + ly - 2, ny);
}

// Items 9-11, first part (see k_closure1_zm for the fields): X, T, Y and Xi'.
// With `form` set (after the velocity-form solve) the kernel also forms
// j~ = rho u - j0' from the final iterate (u1 when the pass count left it
// there, else u0), stores it in the j~ buffer the pass count selects and
// copies a final u1 to u0, as k_jt_final does; otherwise it reads u0 and
// that j~ buffer.
template <class R, int TX, int TY>
__global__ void __launch_bounds__(TX * TY)
k_closure1_t2(const Domain* __restrict__ tab, const Tile* __restrict__ tiles, const SolveInfo* __restrict__ info,
              const R* __restrict__ pf, const R* __restrict__ rho, const R* __restrict__ j0p, R* u0,
              const R* __restrict__ u1, R* __restrict__ jtA, R* __restrict__ jtB, R* __restrict__ X,
              R* __restrict__ T, R* __restrict__ Y, R* __restrict__ Xi, int form,
              const int* __restrict__ go)
{
    constexpr int D = 2;
    constexpr int UX = TX + 4, UY = TY + 4;
    __shared__ R sl[4][UY][UX];   // p - p_ref, c_s^2 - c_s^2_ref, ux, uy

    if (*go == 0) return;   // the solve is not finished (launched ahead of the host's check)
    const Tile tl = tiles[blockIdx.x];
    if (tl.dom < 0) return;   // uniform per block
    const Domain& dm = tab[tl.dom];
    const int nx = dm.g.nx, ny = dm.g.ny;
    const long long o = dm.off, St = dm.g.S;
    const R* const pp = pf + o;            // p - p_ref
    const R* const pri = pf + o + 2 * St;  // 1/rho
    const R* const pc = pf + o + 3 * St;   // c_s^2 - c_s^2_ref
    const R pref = R(dm.cf.pref);
    const bool odd = info[tl.dom].final_buf != 0;   // uniform per block
    // the final iterate; with odd && form, u0 is only written (own points)
    const R* const uo = (form && odd ? u1 : u0) + o;
    const int tid = threadIdx.x + TX * threadIdx.y;
    for (int k = tid; k < UX * UY; k += TX * TY) {
        const unsigned t = frame_site<UX>(k, tl.x0, tl.y0, nx, ny);
        R* const sp = &sl[0][0][0] + k;
        sp[0] = ldo(pp, t);
        sp[UX * UY] = ldo(pc, t);
        sp[2 * UX * UY] = ldo(uo, t);
        sp[3 * UX * UY] = ldo(uo + St, t);
    }
    __syncthreads();
    const int x = tl.x0 + (int)threadIdx.x, y = tl.y0 + (int)threadIdx.y;
    if (x >= nx || y >= ny) return;
    const unsigned i0 = (unsigned)x + (unsigned)nx * (unsigned)y;
    const int cx = (int)threadIdx.x + 2, cy = (int)threadIdx.y + 2;
    // field f at the k-th neighbour (-2, -1, +1, +2) along axis a
    auto at = [&](int f, int a, int k) -> R {
        const int d = k < 2 ? k - 2 : k - 1;
        return a == 0 ? sl[f][cy][cx + d] : sl[f][cy + d][cx];
    };
    R* const jt = (odd ? jtB : jtA) + o;

    R G[3][3] = {};    // d_a u_b
    R M[3][3][3] = {}; // d_a (p u_b u_g)
    R Pg[3] = {}, C[3] = {};  // d_a p, d_a (p/rho)
#pragma unroll
    for (int a = 0; a < D; ++a) {
        R pv[4], cv[4], uv[4][3];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            pv[k] = at(0, a, k);
            cv[k] = at(1, a, k);
#pragma unroll
            for (int b = 0; b < D; ++b) uv[k][b] = at(2 + b, a, k);
        }
        Pg[a] = d1<R>(pv[0], pv[1], pv[2], pv[3]);
        C[a] = d1<R>(cv[0], cv[1], cv[2], cv[3]);
#pragma unroll
        for (int b = 0; b < D; ++b) {
            G[a][b] = d1<R>(uv[0][b], uv[1][b], uv[2][b], uv[3][b]);
#pragma unroll
            for (int c = b; c < D; ++c) {
                R m = d1<R>((pref + pv[0]) * uv[0][b] * uv[0][c], (pref + pv[1]) * uv[1][b] * uv[1][c],
                            (pref + pv[2]) * uv[2][b] * uv[2][c], (pref + pv[3]) * uv[3][b] * uv[3][c]);
                M[a][b][c] = m;
                M[a][c][b] = m;
            }
        }
    }
    const R ep = pref + sl[0][cy][cx], eP1 = ldo(pf + o + St, i0), inv = ldo(pri, i0);
    R us[3] = {sl[2][cy][cx], sl[3][cy][cx], R(0)};
    R trG = R(0);
#pragma unroll
    for (int a = 0; a < D; ++a) trG += G[a][a];

    sto(X + o, i0, eP1 * trG);
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int c = a; c < D; ++c) sto(T + o + sym2<D>(a, c) * St, i0, ep * (G[a][c] + G[c][a]));
#pragma unroll
    for (int b = 0; b < D; ++b) {
        R acc = Pg[b] * inv;
#pragma unroll
        for (int c = 0; c < D; ++c) acc += us[c] * G[c][b];
        sto(Y + o + b * St, i0, acc);
    }

    const R gm = R(dm.cf.gamma);
    const R KX = (gm * gm + R(4) * gm + R(1)) / (R(3) * (gm + R(1)));
    const R KJ = (R(1) - gm) * R(dm.cf.c0sq);
    R jts[3] = {R(0), R(0), R(0)};
    if (form) {
        const R r = ldo(rho + o, i0);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            jts[a] = r * us[a] - ldo(j0p + o + a * St, i0);
            sto(jt + a * St, i0, jts[a]);
            if (odd) sto(u0 + o + a * St, i0, us[a]);
        }
    } else {
#pragma unroll
        for (int a = 0; a < D; ++a) jts[a] = ldo(jt + a * St, i0);
    }
    R V[3];
#pragma unroll
    for (int a = 0; a < D; ++a) V[a] = ep * C[a] + eP1 * us[a] * trG;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a; b < D; ++b)
#pragma unroll
            for (int c = b; c < D; ++c) {
                R br = M[c][a][b] + M[b][a][c] + M[a][b][c];
                R dj = R(0);
                if (a == b) { br += V[c]; dj += jts[c]; }
                if (a == c) { br += V[b]; dj += jts[b]; }
                if (b == c) { br += V[a]; dj += jts[a]; }
                sto(Xi + o + sym3<D>(a, b, c) * St, i0, KX * br + KJ * dj);
            }
}

// Item 11, second part: Sigma from the derivatives of X, T, Y, j = rho u and
// u (see k_closure2_zm).
template <class R, int TX, int TY>
__global__ void __launch_bounds__(TX * TY)
k_closure2_t2(const Domain* __restrict__ tab, const Tile* __restrict__ tiles, const R* __restrict__ rho,
              const R* __restrict__ u, const R* __restrict__ X, const R* __restrict__ T,
              const R* __restrict__ Y, R* __restrict__ Sig, const int* __restrict__ go)
{
    constexpr int D = 2;
    constexpr int UX = TX + 4, UY = TY + 4;
    // X, Txx, Tyy, Txy, Yx, Yy, rho ux, rho uy, ux, uy
    __shared__ R sl[10][UY][UX];

    if (*go == 0) return;   // the solve is not finished (launched ahead of the host's check)
    const Tile tl = tiles[blockIdx.x];
    if (tl.dom < 0) return;   // uniform per block
    const Domain& dm = tab[tl.dom];
    const int nx = dm.g.nx, ny = dm.g.ny;
    const long long o = dm.off, St = dm.g.S;
    const R* const rh = rho + o;
    const R* const uo = u + o;
    const int tid = threadIdx.x + TX * threadIdx.y;
    for (int k = tid; k < UX * UY; k += TX * TY) {
        const unsigned t = frame_site<UX>(k, tl.x0, tl.y0, nx, ny);
        R* const sp = &sl[0][0][0] + k;
        constexpr int P = UX * UY;
        sp[0] = ldo(X + o, t);
#pragma unroll
        for (int c = 0; c < 3; ++c) sp[(1 + c) * P] = ldo(T + o + c * St, t);
        sp[4 * P] = ldo(Y + o, t);
        sp[5 * P] = ldo(Y + o + St, t);
        const R r = ldo(rh, t), ux = ldo(uo, t), uy = ldo(uo + St, t);
        sp[6 * P] = r * ux;
        sp[7 * P] = r * uy;
        sp[8 * P] = ux;
        sp[9 * P] = uy;
    }
    __syncthreads();
    const int x = tl.x0 + (int)threadIdx.x, y = tl.y0 + (int)threadIdx.y;
    if (x >= nx || y >= ny) return;
    const unsigned i0 = (unsigned)x + (unsigned)nx * (unsigned)y;
    const int cx = (int)threadIdx.x + 2, cy = (int)threadIdx.y + 2;
    // D1 of LDS field f along axis a
    auto dd = [&](int f, int a) -> R {
        return a == 0 ? d1<R>(sl[f][cy][cx - 2], sl[f][cy][cx - 1], sl[f][cy][cx + 1], sl[f][cy][cx + 2])
                      : d1<R>(sl[f][cy - 2][cx], sl[f][cy - 1][cx], sl[f][cy + 1][cx], sl[f][cy + 2][cx]);
    };
    R DX[3] = {}, DT[3] = {}, DY[3][3] = {}, G[3][3] = {};
    R trJ = R(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        DX[a] = dd(0, a);
#pragma unroll
        for (int c = 0; c < D; ++c) DT[a] += dd(1 + sym2<D>(a, c), c);
#pragma unroll
        for (int b = 0; b < D; ++b) DY[a][b] = dd(4 + b, a);
        trJ += dd(6 + a, a);
#pragma unroll
        for (int b = 0; b < D; ++b) G[a][b] = dd(8 + b, a);
    }
    const R r = ldo(rh, i0);
    const EosVal<R> e = eos_all<R>(dm.cf.eos, r);
    R us[3] = {sl[8][cy][cx], sl[9][cy][cx], R(0)};
    R trG = R(0), trDY = R(0);
#pragma unroll
    for (int a = 0; a < D; ++a) { trG += G[a][a]; trDY += DY[a][a]; }
    const R gm = R(dm.cf.gamma);
    const R KS1 = R(-0.25) * (gm + R(1)) * (gm + R(1)) / (gm - R(1));
    const R KS2 = (gm * gm + R(4) * gm + R(1)) / (R(6) * (gm - R(1)));
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a; b < D; ++b) {
            const R br1 = us[a] * DX[b] + us[b] * DX[a] + us[b] * DT[a] + us[a] * DT[b];
            R br2 = -e.dp * trJ * (G[a][b] + G[b][a]) - e.p * (DY[a][b] + DY[b][a]);
            if (a == b) br2 += -e.P1 * trDY + e.P2 * trG * trJ;
            sto(Sig + o + sym2<D>(a, b) * St, i0, KS1 * br1 + KS2 * br2);
        }
}


// Item 2 for D2Q21 on LDS tiles: f = kappa rho d_a d_b d_b rho (Sec. IV E,
// Table III), j0' = j0 + f/2; the planes p, P1 and 1/rho of the iteration;
// its start j~ (zero, the previous step's, or extrapolated from the previous
// steps: linear 2 y1 - y2 or quadratic y3 + 3 (y1 - y2), with hist and hist2
// keeping y1 and y2 for the next step when non-null); u = (j0' + j~)/rho;
// and per-block maxima of |j0'| for the stop rule.  rho is staged in LDS for
// the tile and a 2-wide frame; the rest is per site.
template <class R, int TX, int TY>
__global__ void __launch_bounds__(TX * TY)
k_force_t2(const Domain* __restrict__ tab, const Tile* __restrict__ tiles, IterCtl ic, const double* __restrict__ mass,
           const R* __restrict__ j0, R* __restrict__ f, R* __restrict__ j0p, R* __restrict__ u,
           const R* jt_prevA, const R* jt_prevB, const SolveInfo* prev_info, R* jt0,
           R* hist, R* hist2, int order)
{
    constexpr int UX = TX + 4, UY = TY + 4;
    __shared__ double sr[UY][UX];   // FP64 rho (the stencil runs in FP64, as in k_force_zm)

    const Tile tl = tiles[blockIdx.x];
    if (tl.dom < 0) return;   // uniform per block (padding: no slot)
    const Domain& dm = tab[tl.dom];
    const int nx = dm.g.nx, ny = dm.g.ny;
    const long long o = dm.off, St = dm.g.S;
    const double* const mh = mass + o;
    const int tid = threadIdx.x + TX * threadIdx.y;
    for (int k = tid; k < UX * UY; k += TX * TY)
        (&sr[0][0])[k] = ldo(mh, frame_site<UX>(k, tl.x0, tl.y0, nx, ny));
    __syncthreads();
    double amax = 0.0;
    const int x = tl.x0 + (int)threadIdx.x, y = tl.y0 + (int)threadIdx.y;
    if (x < nx && y < ny) {
        const unsigned i0 = (unsigned)x + (unsigned)nx * (unsigned)y;
        const int cx = (int)threadIdx.x + 2, cy = (int)threadIdx.y + 2;
        auto RH = [&](int dx, int dy) -> double { return sr[cy + dy][cx + dx]; };
        const double r64 = RH(0, 0);
        // (10): tau -2 ; (11): tau 1/2 ; (20): tau 1/4
        double fa[2];
        fa[0] = -2.0 * (RH(1, 0) - RH(-1, 0)) + 0.5 * (RH(1, 1) + RH(1, -1) - RH(-1, 1) - RH(-1, -1)) +
                0.5 * (RH(2, 0) - RH(-2, 0));
        fa[1] = -2.0 * (RH(0, 1) - RH(0, -1)) + 0.5 * (RH(1, 1) + RH(-1, 1) - RH(1, -1) - RH(-1, -1)) +
                0.5 * (RH(0, 2) - RH(0, -2));
        const double kr = dm.cf.kappa * r64;
        const R inv = R(1) / R(r64);   // as the 1/rho plane of item 1
        const R* prev = nullptr;
        if (prev_info) prev = prev_info[tl.dom].final_buf ? jt_prevB : jt_prevA;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const R fv = R(kr * fa[a]);
            const R jp = ldo(j0 + o + a * St, i0) + R(0.5) * fv;
            R jt = prev ? ldo(prev + o + a * St, i0) : R(0);
            if (hist) {
                const R y1 = jt;
                const R y2 = ldo(hist + o + a * St, i0);
                sto(hist + o + a * St, i0, y1);
                R y3 = R(0);
                if (hist2) {
                    y3 = ldo(hist2 + o + a * St, i0);
                    sto(hist2 + o + a * St, i0, y2);
                }
                if (order == 2)
                    jt = y3 + R(3) * (y1 - y2);
                else if (order == 1)
                    jt = R(2) * y1 - y2;
            }
            sto(f + o + a * St, i0, fv);
            sto(j0p + o + a * St, i0, jp);
            if (jt0) sto(jt0 + o + a * St, i0, jt);   // the velocity-form solve needs only u
            sto(u + o + a * St, i0, (jp + jt) * inv);
            amax = fmax(amax, fabs((double)jp));
        }
    }
    block_max_part(ic.part, amax);
}

// ---------------------------------------------------------------------------
// Sigma in the stencil formulation (LB2P_FLAG_STENCIL_CLOSURE), per site.
// The derivatives of item 11 are taken with the outer operator carried
// through the products (the Supplemental preamble allows moving the
// operators), so that every second derivative acts on p or on u alone and
// takes the Table III stencils for d_a d_a (Sec. IV C) and the traceless
// d_a d_b (Sec. IV D):
//   d_a X     = (d_a P1) tr G + P1 d_a d_g u_g
//   d_g T_ag  = (d_g p)(G_ag + G_ga) + p (d_a d_g u_g + d_g d_g u_a)
//   d_a Y_b   = -rho^-2 (d_a rho)(d_b p) + rho^-1 d_a d_b p + G_ag G_gb + u_g d_a d_g u_b
// with first derivatives by the stencil of Sec. IV B; Sigma then as in
// k_closure2_zm / k_closure2_t2.  p enters as p - p_ref (the per-step plane)
// and rho as the FP64 mass of item 1.
// ---------------------------------------------------------------------------

// d_a d_b F at one site from the compact stencils: Laplacian (rest -2D,
// shell (100) 1) and traceless part (shell (100) tau1, shell (110) 1/4).
template <int D, class R, class F>
__device__ __forceinline__ void hess_compact(F at, R H[3][3])
{
    constexpr double tau1 = D == 3 ? 0.5 : 1.0, tau2 = 0.25;
    const R c0 = at(0, 0, 0);
    R lap = R(-2 * D) * c0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) H[a][b] = R(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const int e[3] = {a == 0, a == 1, a == 2};
        const R sp = at(e[0], e[1], e[2]), sm = at(-e[0], -e[1], -e[2]);
        lap += sp + sm;
        // traceless (d_c d_c - |d|^2 / D) on the diagonal: 1 - 1/D for c = a, -1/D otherwise
#pragma unroll
        for (int c = 0; c < D; ++c) H[c][c] += R(tau1 * ((c == a ? 1.0 : 0.0) - 1.0 / D)) * (sp + sm);
    }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a + 1; b < D; ++b) {
            int e1[3] = {0, 0, 0}, e2[3] = {0, 0, 0};
            e1[a] = 1; e2[b] = 1;
            // the four vectors +-e_a +-e_b: d_a d_b = +1 for (+,+), (-,-), -1 otherwise
            const R pp = at(e1[0] + e2[0], e1[1] + e2[1], e1[2] + e2[2]);
            const R mm = at(-e1[0] - e2[0], -e1[1] - e2[1], -e1[2] - e2[2]);
            const R pm = at(e1[0] - e2[0], e1[1] - e2[1], e1[2] - e2[2]);
            const R mp = at(-e1[0] + e2[0], -e1[1] + e2[1], -e1[2] + e2[2]);
            const R sum = pp + mm + pm + mp;
            H[a][b] += R(tau2) * ((pp + mm) - (pm + mp));
#pragma unroll
            for (int c = 0; c < D; ++c)
                H[c][c] += R(tau2 * ((c == a || c == b ? 1.0 : 0.0) - 2.0 / D)) * sum;
        }
#pragma unroll
    for (int a = 0; a < D; ++a) {
        H[a][a] += lap * R(1.0 / D);
#pragma unroll
        for (int b = 0; b < a; ++b) H[a][b] = H[b][a];
    }
}

template <int Q, class R>
__global__ void __launch_bounds__(256) k_sigma_stencil(const Domain* __restrict__ tab,
                                                       const Tile* __restrict__ tiles,
                                                       const R* __restrict__ pf, const double* __restrict__ mass,
                                                       const R* __restrict__ u, R* __restrict__ Sig,
                                                       const int* __restrict__ go)
{
    using L = Lattice<Q>;
    constexpr int D = L::D;
    if (*go == 0) return;   // the solve is not finished (launched ahead of the host's check)
    const Where w = locate(tab, tiles);
    if (!w.ok) return;
    const Domain& dm = tab[w.dom];
    const long long o = dm.off, St = dm.g.S;
    const NbP nb = make_nbp(dm.g, w.x, w.y, w.z);
    const unsigned i0 = nb.i0;
    const R* const pdev = pf + o;
    const R* const pP1 = pf + o + St;
    const double* const ms = mass + o;
    const R* const uo = u + o;
    auto at3 = [&](int dx, int dy, int dz) { return nb.at(dx, dy, D == 3 ? dz : 0); };
    // first derivatives (Sec. IV B) along axis a of a field given by value(index)
    auto d1f = [&](auto value, int a) {
        const int e[3] = {a == 0, a == 1, a == 2};
        return d1<R>(value(at3(-2 * e[0], -2 * e[1], -2 * e[2])), value(at3(-e[0], -e[1], -e[2])),
                     value(at3(e[0], e[1], e[2])), value(at3(2 * e[0], 2 * e[1], 2 * e[2])));
    };
    R G[3][3] = {}, Pg[3] = {}, DP1[3] = {}, Drho[3] = {}, trJ = R(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
#pragma unroll
        for (int b = 0; b < D; ++b) G[a][b] = d1f([&](unsigned t) { return ldo(uo + b * St, t); }, a);
        Pg[a] = d1f([&](unsigned t) { return ldo(pdev, t); }, a);
        DP1[a] = d1f([&](unsigned t) { return ldo(pP1, t); }, a);
        Drho[a] = R(d1<double>(ldo(ms, at3(a == 0 ? -2 : 0, a == 1 ? -2 : 0, a == 2 ? -2 : 0)),
                               ldo(ms, at3(a == 0 ? -1 : 0, a == 1 ? -1 : 0, a == 2 ? -1 : 0)),
                               ldo(ms, at3(a == 0 ? 1 : 0, a == 1 ? 1 : 0, a == 2 ? 1 : 0)),
                               ldo(ms, at3(a == 0 ? 2 : 0, a == 1 ? 2 : 0, a == 2 ? 2 : 0))));
        // d_a j_a with j = rho u
        trJ += d1f([&](unsigned t) { return R(ldo(ms, t)) * ldo(uo + a * St, t); }, a);
    }
    R Hu[3][3][3], Hp[3][3];
#pragma unroll
    for (int c = 0; c < D; ++c)
        hess_compact<D, R>([&](int dx, int dy, int dz) { return ldo(uo + c * St, at3(dx, dy, dz)); }, Hu[c]);
    hess_compact<D, R>([&](int dx, int dy, int dz) { return ldo(pdev, at3(dx, dy, dz)); }, Hp);

    const R r = R(ldo(ms, i0));
    const R ri = R(1) / r;
    const EosVal<R> e = eos_all<R>(dm.cf.eos, r);
    const R us[3] = {ldo(uo, i0), ldo(uo + St, i0), D == 3 ? ldo(uo + 2 * St, i0) : R(0)};
    R trG = R(0);
#pragma unroll
    for (int a = 0; a < D; ++a) trG += G[a][a];
    R DX[3] = {}, DT[3] = {}, DY[3][3] = {};
#pragma unroll
    for (int a = 0; a < D; ++a) {
        R ddiv = R(0), lapu = R(0);
#pragma unroll
        for (int c = 0; c < D; ++c) {
            ddiv += Hu[c][a][c];
            lapu += Hu[a][c][c];
        }
        DX[a] = DP1[a] * trG + e.P1 * ddiv;
        R dt = e.p * (ddiv + lapu);
#pragma unroll
        for (int c = 0; c < D; ++c) dt += Pg[c] * (G[a][c] + G[c][a]);
        DT[a] = dt;
#pragma unroll
        for (int b = 0; b < D; ++b) {
            R v = -Drho[a] * Pg[b] * ri * ri + Hp[a][b] * ri;
#pragma unroll
            for (int c = 0; c < D; ++c) v += G[a][c] * G[c][b] + us[c] * Hu[b][a][c];
            DY[a][b] = v;
        }
    }
    R trDY = R(0);
#pragma unroll
    for (int a = 0; a < D; ++a) trDY += DY[a][a];
    const R gm = R(dm.cf.gamma);
    const R KS1 = R(-0.25) * (gm + R(1)) * (gm + R(1)) / (gm - R(1));
    const R KS2 = (gm * gm + R(4) * gm + R(1)) / (R(6) * (gm - R(1)));
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a; b < D; ++b) {
            const R br1 = us[a] * DX[b] + us[b] * DX[a] + us[b] * DT[a] + us[a] * DT[b];
            R br2 = -e.dp * trJ * (G[a][b] + G[b][a]) - e.p * DY[a][b] - e.p * DY[b][a];
            if (a == b) br2 += -e.P1 * trDY + e.P2 * trG * trJ;
            sto(Sig + o + sym2<D>(a, b) * St, i0, KS1 * br1 + KS2 * br2);
        }
}

}  // namespace lb2p
