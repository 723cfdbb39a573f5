// lattice.hpp -- compile-time velocity sets, shell weights, stencil
// coefficients and the equation of state for the gfx950 kernels.
//
// D3Q59 (Table I) and D2Q21 (Table II).  Velocities are stored as the rest
// vector followed by antipodal pairs (c, -c): index 2p+1 holds c and 2p+2
// holds -c, so a collision loop can form the even and odd parts of each pair
// once.  Within a shell the first member of each pair is the vector with the
// first non-zero component positive.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace lb2p {

struct VelSet {
    int q;             // number of velocities
    int d;             // dimension
    int nshell;
    int c[64][3];
    int shell[64];
    int shell_size[8];
};

// Candidate vectors of a shell: absolute components are a permutation of rep.
constexpr bool member(const int v[3], const int rep[3], int d)
{
    int a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
    for (int k = 0; k < d; ++k) {
        a[k] = v[k] < 0 ? -v[k] : v[k];
        b[k] = rep[k];
    }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j + 1 < d - i; ++j) {
            if (a[j] < a[j + 1]) { int t = a[j]; a[j] = a[j + 1]; a[j + 1] = t; }
            if (b[j] < b[j + 1]) { int t = b[j]; b[j] = b[j + 1]; b[j + 1] = t; }
        }
    for (int k = 0; k < d; ++k)
        if (a[k] != b[k]) return false;
    return true;
}

constexpr bool first_nonzero_positive(const int v[3])
{
    for (int k = 0; k < 3; ++k)
        if (v[k] != 0) return v[k] > 0;
    return false;
}

constexpr VelSet make_set(int d, int nshell, const int (*reps)[3])
{
    VelSet s{};
    s.d = d;
    s.nshell = nshell;
    int n = 0;
    for (int k = 0; k < nshell; ++k) {
        int cnt = 0;
        const int zr = d == 3 ? 4 : 0;
        for (int z = zr; z >= -zr; --z)
            for (int y = 4; y >= -4; --y)
                for (int x = 4; x >= -4; --x) {
                    int v[3] = {x, y, z};
                    if (!member(v, reps[k], d)) continue;
                    bool rest = (x == 0 && y == 0 && z == 0);
                    if (!rest && !first_nonzero_positive(v)) continue;
                    s.c[n][0] = x; s.c[n][1] = y; s.c[n][2] = z;
                    s.shell[n] = k;
                    ++n; ++cnt;
                    if (!rest) {
                        s.c[n][0] = -x; s.c[n][1] = -y; s.c[n][2] = -z;
                        s.shell[n] = k;
                        ++n; ++cnt;
                    }
                }
        s.shell_size[k] = cnt;
    }
    s.q = n;
    return s;
}

constexpr int kRep3[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {1, 1, 1},
                             {2, 0, 0}, {2, 2, 0}, {2, 2, 2}, {4, 0, 0}};
constexpr int kRep2[6][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {2, 0, 0},
                             {2, 2, 0}, {4, 0, 0}};

constexpr VelSet kD3Q59 = make_set(3, 8, kRep3);
constexpr VelSet kD2Q21 = make_set(2, 6, kRep2);
static_assert(kD3Q59.q == 59, "D3Q59 must have 59 velocities");
static_assert(kD2Q21.q == 21, "D2Q21 must have 21 velocities");

template <int Q> struct Lattice;

template <> struct Lattice<59> {
    static constexpr int Q = 59, D = 3, NSHELL = 8, NPAIR = 29;
    static constexpr int NSIG = 6, NXI = 10;
    __host__ __device__ static constexpr int cx(int i) { return kD3Q59.c[i][0]; }
    __host__ __device__ static constexpr int cy(int i) { return kD3Q59.c[i][1]; }
    __host__ __device__ static constexpr int cz(int i) { return kD3Q59.c[i][2]; }
    __host__ __device__ static constexpr int shell(int i) { return kD3Q59.shell[i]; }
};

template <> struct Lattice<21> {
    static constexpr int Q = 21, D = 2, NSHELL = 6, NPAIR = 10;
    static constexpr int NSIG = 3, NXI = 4;
    __host__ __device__ static constexpr int cx(int i) { return kD2Q21.c[i][0]; }
    __host__ __device__ static constexpr int cy(int i) { return kD2Q21.c[i][1]; }
    __host__ __device__ static constexpr int cz(int) { return 0; }
    __host__ __device__ static constexpr int shell(int i) { return kD2Q21.shell[i]; }
};

// Shell weights w_k(s), s = c_s^2, Tables I and II.  The D3Q59 rest weight
// follows from sum_i w_i = 1: the printed Table I w0 violates that condition
// and the printed upper positivity bound 1.1917145 of Sec. III, while the
// normalised one satisfies both.
template <int Q, class R>
__host__ __device__ inline void shell_weights(R s, R* w)
{
    // The polynomials of Tables I and II with every constant divisor folded
    // into a reciprocal coefficient (a division by a constant is not a
    // multiplication in IEEE arithmetic and costs a full divide sequence).
    if constexpr (Q == 59) {
        const R base = s * (R(8.0 / 45.0) - s * R(1.0 / 3.0) + s * s * R(1.0 / 6.0));
        w[1] = R(2) * base;
        w[2] = base;
        w[3] = s * R(1.0 / 12.0) * (R(-16.0 / 15.0) + R(4) * s - R(2.5) * s * s);
        w[4] = s * R(1.0 / 96.0) * (R(-24.0 / 5.0) + R(17) * s - R(9) * s * s);
        w[5] = s * R(1.0 / 192.0) * (R(-8.0 / 15.0) + s + s * s);
        w[6] = s * R(1.0 / 192.0) * (R(4.0 / 15.0) - s + s * s);
        w[7] = s * R(1.0 / 384.0) * (R(4.0 / 15.0) - s + s * s);
        w[0] = R(1) - (R(6) * w[1] + R(12) * w[2] + R(8) * w[3] + R(6) * w[4] +
                       R(12) * w[5] + R(8) * w[6] + R(6) * w[7]);
    } else {
        w[0] = R(1) - R(22.5) * s * (R(7.0 / 60.0) - R(7.0 / 48.0) * s + s * s * R(1.0 / 16.0));
        w[1] = s * R(1.0 / 3.0) * (R(32.0 / 15.0) - R(4) * s + R(2) * s * s);
        w[2] = s * (s * R(1.0 / 3.0) - s * s * R(0.25));
        w[3] = s * (R(-1.0 / 18.0) + R(3.0 / 16.0) * s - s * s * R(1.0 / 12.0));
        w[4] = s * R(1.0 / 96.0) * (R(-0.5) * s + R(1.5) * s * s);
        w[5] = s * R(1.0 / 384.0) * (R(4.0 / 15.0) - s + s * s);
    }
}

// Weight of one shell K >= 1 (the other shells fold away when inlined).
template <int Q, int K, class R>
__host__ __device__ inline R shell_weight(R s)
{
    R w[8];
    shell_weights<Q, R>(s, w);
    return w[K];
}

// Equation of state of App. B, the quantities of Supplemental item 1.
struct EosParams {
    double rho1, rho3, inv_delta_pi;   // pi/(rho2-rho1)
    double A, cs2_1, a_delta_over_pi;  // A (rho2-rho1)/pi
};

template <class R>
struct EosVal {
    R cs2, p, dp, P1, P2;
};

template <class R>
__device__ __host__ inline R eos_cos(R x);
template <>
__device__ __host__ inline float eos_cos<float>(float x) { return cosf(x); }
template <>
__device__ __host__ inline double eos_cos<double>(double x) { return cos(x); }
template <class R>
__device__ __host__ inline R eos_sin(R x);
template <>
__device__ __host__ inline float eos_sin<float>(float x) { return sinf(x); }
template <>
__device__ __host__ inline double eos_sin<double>(double x) { return sin(x); }
template <class R>
__device__ __host__ inline R eos_exp(R x);
template <>
__device__ __host__ inline float eos_exp<float>(float x) { return expf(x); }
template <>
__device__ __host__ inline double eos_exp<double>(double x) { return exp(x); }

// c_s^2 only (n_eq weights).
template <class R>
__device__ __host__ inline R eos_cs2(const EosParams& e, R rho)
{
    if (rho > R(e.rho1) && rho < R(e.rho3)) {
        R th = (rho - R(e.rho1)) * R(e.inv_delta_pi);
        return R(e.cs2_1) * eos_exp<R>(R(e.a_delta_over_pi) * (R(1) - eos_cos<R>(th)));
    }
    return R(e.cs2_1);
}

// psi = A sin(pi (rho - rho1)/(rho2 - rho1)) on (rho1, rho3), zero outside.
template <class R>
__device__ __host__ inline R eos_psi(const EosParams& e, R rho)
{
    if (rho > R(e.rho1) && rho < R(e.rho3)) return R(e.A) * eos_sin<R>((rho - R(e.rho1)) * R(e.inv_delta_pi));
    return R(0);
}

// c_s^2, p, dp/drho, p - rho dp/drho, rho d2p/drho2 (psi' jumps at the ends
// of (rho1, rho3); outside the interval psi = psi' = 0).
template <class R>
__device__ __host__ inline EosVal<R> eos_all(const EosParams& e, R rho)
{
    R cs2 = R(e.cs2_1), psi = R(0), dpsi = R(0);
    if (rho > R(e.rho1) && rho < R(e.rho3)) {
        R th = (rho - R(e.rho1)) * R(e.inv_delta_pi);
        R c = eos_cos<R>(th), s = eos_sin<R>(th);
        cs2 = R(e.cs2_1) * eos_exp<R>(R(e.a_delta_over_pi) * (R(1) - c));
        psi = R(e.A) * s;
        dpsi = R(e.A) * R(e.inv_delta_pi) * c;
    }
    EosVal<R> v;
    v.cs2 = cs2;
    v.p = rho * cs2;
    v.dp = cs2 * (R(1) + rho * psi);
    v.P1 = -rho * rho * cs2 * psi;                       // p - rho dp/drho
    v.P2 = rho * cs2 * (psi * (R(2) + rho * psi) + rho * dpsi);
    return v;
}

// First-derivative stencil of Sec. IV B along one axis:
// d g = 2/3 (g[+1] - g[-1]) - 1/12 (g[+2] - g[-2]).
template <class R>
__device__ __host__ inline R d1(R m2, R m1, R p1, R p2)
{
    return R(2.0 / 3.0) * (p1 - m1) - R(1.0 / 12.0) * (p2 - m2);
}

}  // namespace lb2p
