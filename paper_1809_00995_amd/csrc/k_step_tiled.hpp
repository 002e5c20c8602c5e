// k_step_tiled.hpp -- the tiled step kernel for gfx950, with the network
// diagnostics fused in.
//
// Same update as k_step_plain (Sec. 2, Eqs. (4)-(7)), organised for the
// memory system:
//  - A block is TY wavefronts; wavefront ly owns the 64 consecutive x-sites of
//    row y0 + ly of a 64 x TY tile, so every global load and store of a plane
//    is a 256 B (FP32) or 512 B (FP64) contiguous segment.  The block walks a
//    chunk of z-planes of its tile.
//  - For each plane the link phasors U_i = e^{iA_i} (one sincos per link) and
//    phi are computed once per site and staged in LDS, together with a one-site
//    halo ring that a few wavefronts compute for the neighbouring tiles; the
//    planes are double-buffered (plane z and z+1 live at once).
//  - Plaquette sines come from products of the four link phasors,
//    sin Xi_ij = Im[U_i(s) U_j(s+i) conj(U_i(s+j)) conj(U_j(s))] (Eq. (3)),
//    so the update makes no further transcendental call; the yz and zx
//    plaquettes of plane z-1 and the phi, U_z of z-1 stay in registers.
//  - Workgroups are dispatched round-robin over the 8 XCDs; tile numbers are
//    remapped so each XCD walks a contiguous run of neighbouring tiles and
//    the halo reads of adjacent tiles meet in the same L2.
//
// Modes: MODE_STEP advances S_n -> S_{n+1}; MODE_STEP_MEASURE also measures
// S_n (the state it reads) on the way (the read-only measuring pass is
// k_measure_tiled.hpp).  The measuring mode stages arg(phi) in FP32 and the
// raw link angles A_i next to the phasors, and counts the winding of each
// plaquette from the wrap counts of its four links: with
// m_i(s) = floor((theta(s+i) - theta(s) + A_i(s) + pi) / 2 pi) the [.]_pi of
// Eq. (11) subtracts 2 pi m_i, the phase differences cancel around the
// plaquette, and W_ij = -(m_i(x) + m_j(x+i) - m_i(x+j) - m_j(x)) exactly.
// Each in-plane link's count is formed once, by the thread that stages its
// site, one plane ahead, and shared through LDS; a site forms the z-link
// counts of itself and of its x and y neighbours.
#pragma once

#include <type_traits>

#include "ah_device.hpp"

namespace ah {

enum : int { MODE_STEP = 0, MODE_STEP_MEASURE = 1 };

// quantities staged per site in LDS
enum : int { Q_PR, Q_PI, Q_UXC, Q_UXS, Q_UYC, Q_UYS, Q_UZC, Q_UZS, Q_COUNT };

template <int TY> struct TileGeom {
    static constexpr int W = 66;              // 64 sites + 1 halo site each side
    static constexpr int H = TY + 2;
    static constexpr int S = W * H;
    static constexpr int HALO = 2 * 64 + 2 * H;   // halo ring, corners included
    static constexpr int HALO_FWD = 65 + TY;      // the row above (with its right end) and
                                                  // the column to the right
    static __device__ __forceinline__ int li(int lx, int ly) { return (ly + 1) * W + (lx + 1); }
    static __device__ __forceinline__ void halo_fwd(int h, int &lx, int &ly) {
        if (h < 65) {
            lx = h;
            ly = TY;
        } else {
            lx = 64;
            ly = h - 65;
        }
    }
    static __device__ __forceinline__ void halo(int h, int &lx, int &ly) {
        if (h < 64) {
            lx = h;
            ly = -1;
        } else if (h < 128) {
            lx = h - 64;
            ly = TY;
        } else if (h < 128 + H) {
            lx = -1;
            ly = h - 128 - 1;
        } else {
            lx = 64;
            ly = h - 128 - H - 1;
        }
    }
};

// sin Xi_ij(s) = Im[U_i(s) U_j(s+i) conj(U_i(s+j)) conj(U_j(s))], phasors as
// (cos, sin).  Written with explicit fused multiply-adds so that its rounding
// does not depend on where the compiler inlines it: the same plaquette is
// formed in the chunk prologue and in the main loop, and results must not
// depend on the z-chunk.
template <typename T>
__device__ __forceinline__ T plaq_sin(T aic, T ais, T bjc, T bjs, T cic, T cis, T djc, T djs) {
    const T wr = fma(aic, djc, ais * djs), wi = fma(ais, djc, -(aic * djs));  // U_i(s) conj(U_j(s))
    const T vr = fma(bjc, cic, bjs * cis), vi = fma(bjs, cic, -(bjc * cis));  // U_j(s+i) conj(U_i(s+j))
    return fma(wr, vi, wi * vr);
}

// 1 - cos Xi_ij(s) = |conj(w) - v|^2 / 2 with w, v as in plaq_sin (|w v| = 1);
// this form keeps its relative accuracy for small Xi.
template <typename T>
__device__ __forceinline__ T plaq_omc(T aic, T ais, T bjc, T bjs, T cic, T cis, T djc, T djs) {
    const T wr = fma(aic, djc, ais * djs), wi = fma(ais, djc, -(aic * djs));
    const T vr = fma(bjc, cic, bjs * cis), vi = fma(bjs, cic, -(bjc * cis));
    const T a = wr - vr, b = wi + vi;
    return (T)0.5 * fma(a, a, b * b);
}

// wrap count of a link: [u]_pi = u - 2 pi m (Eq. (11)), computed in FP64.
// The quotient by 2 pi is taken as a product with its reciprocal (one FP64
// multiply instead of a ~10-instruction correctly rounded division); the
// two differ only when (u + pi) / 2 pi lies within an ulp of an integer,
// i.e. u within ~1e-15 of an odd multiple of pi, where the phase
// difference of the link is ambiguous anyway.
constexpr double kInvTwoPi = 0.15915494309189533576888376337251436;

__device__ __forceinline__ int wrap_count(double u) {
    return (int)floor((u + kPi) * kInvTwoPi);
}

// The measuring kernels take each wrap count from FP32 phases (phase_f32,
// error below 5e-7) in FP32 arithmetic: ta, tb are the phases at the start and
// end of the link and a its raw angle.  False when the FP64 phases (atan2)
// must decide instead: the quotient (u + pi) / 2 pi within the margin of an
// integer, a phase not a number, or |a| > 32.  For |a| <= 32 the four
// roundings move the quotient by at most 1.3e-6 and the phase errors by
// 1.6e-7 more, so outside the margin the integer is the one FP64 phases give.
constexpr float kWrapMarginF = 4e-6f;

__device__ __forceinline__ bool wrap_count_f32(float ta, float tb, float a, int &m) {
    const float u = (tb - ta) + a;
    const float w = (u + 3.1415927e+00f) * 1.5915494e-01f;
    const float f = __builtin_floorf(w);
    m = (int)f;
    const float fr = w - f;
    return fr > kWrapMarginF && fr < 1.0f - kWrapMarginF && __builtin_fabsf(a) <= 32.0f;
}

// FP64 phase of phi = (pr, pi), as the oracle takes it.
template <typename T> __device__ __forceinline__ double phase64(T pr, T pi) {
    return atan2((double)pi, (double)pr);
}

// Wrap count of one link from the FP32 phases ta, tb of its ends and its raw
// angle a; dphase() gives the FP64 phase difference when those must decide.
template <typename T, typename F>
__device__ __forceinline__ int wrap_count_link(float ta, float tb, T a, F dphase) {
    int m;
    if (!wrap_count_f32(ta, tb, (float)a, m))
        m = wrap_count(dphase() + (double)a);
    return m;
}

template <typename T> struct SiteV {
    T pr, pm, ax, ay, az, uxc, uxs, uyc, uys, uzc, uzs;
    float th;   // FP32 phase (measuring kernels)
};

// Everything the update of one site x reads (Eqs. (4)-(7)), gathered by the
// kernel: phi, A and the link phasors U_i = e^{iA_i} at x, the momenta at x,
// phi at the six neighbours, the backward links U_j(x-j), and the sines of
// the nine plaquettes that contain a link of x (Eq. (3)).  Suffixes name the
// site: _xp is x+x, _ym is x-y, and so on.
template <typename T> struct Stencil {
    T pr, pm, ax, ay, az, uxc, uxs, uyc, uys, uzc, uzs;
    T pr0, pi0, ex0, ey0, ez0;
    T pr_xp, pi_xp, pr_xm, pi_xm, pr_yp, pi_yp, pr_ym, pi_ym, pr_zp, pi_zp, pr_zm, pi_zm;
    T uxc_xm, uxs_xm, uyc_ym, uys_ym, uzc_zm, uzs_zm;
    T pxy, pxy_xm, pxy_ym, pyz, pyz_ym, pyz_zm, pzx, pzx_xm, pzx_zm;
};

// New values of the site: Pi^{n+1/2}, E^{n+1/2}, phi^{n+1}, A^{n+1}.
template <typename T> struct SiteNew {
    T pr, pi, ex, ey, ez, qr, qi, ax, ay, az;
};

// Step coefficients of Eqs. (4)-(5) in the stencil's precision.
template <typename T> struct StepK {
    T c1, c2, c3, d1, d2, d3, dt, s2;
};

template <typename T> __device__ __forceinline__ StepK<T> step_k(const RealDesc &d, const Coef &c) {
    return StepK<T>{ (T)c.c1, (T)c.c2, (T)c.c3, (T)c.d1, (T)c.d2, (T)c.d3, (T)d.dt,
                     (T)(d.sigma * d.sigma) };
}

// The leapfrog update of one site, Eqs. (4)-(7).  Contraction is off and
// every fused multiply-add is written out, so the rounding is the same in
// every kernel that calls it: the tiled kernels of any tile shape, and the
// two-steps-per-pass kernel, agree bit for bit.
template <typename T>
__device__ __forceinline__ SiteNew<T> leapfrog_site(const Stencil<T> &s, const StepK<T> &k) {
#pragma clang fp contract(off)
    // Eq. (4): sum_j [U_j(x) phi(x+j) + conj(U_j(x-j)) phi(x-j)] - 6 phi(x)
    T lr = (T)-6 * s.pr, li = (T)-6 * s.pm;
    lr = fma(s.uxc, s.pr_xp, lr);    lr = fma(-s.uxs, s.pi_xp, lr);
    li = fma(s.uxc, s.pi_xp, li);    li = fma(s.uxs, s.pr_xp, li);
    lr = fma(s.uxc_xm, s.pr_xm, lr); lr = fma(s.uxs_xm, s.pi_xm, lr);
    li = fma(s.uxc_xm, s.pi_xm, li); li = fma(-s.uxs_xm, s.pr_xm, li);
    lr = fma(s.uyc, s.pr_yp, lr);    lr = fma(-s.uys, s.pi_yp, lr);
    li = fma(s.uyc, s.pi_yp, li);    li = fma(s.uys, s.pr_yp, li);
    lr = fma(s.uyc_ym, s.pr_ym, lr); lr = fma(s.uys_ym, s.pi_ym, lr);
    li = fma(s.uyc_ym, s.pi_ym, li); li = fma(-s.uys_ym, s.pr_ym, li);
    lr = fma(s.uzc, s.pr_zp, lr);    lr = fma(-s.uzs, s.pi_zp, lr);
    li = fma(s.uzc, s.pi_zp, li);    li = fma(s.uzs, s.pr_zp, li);
    lr = fma(s.uzc_zm, s.pr_zm, lr); lr = fma(s.uzs_zm, s.pi_zm, lr);
    li = fma(s.uzc_zm, s.pi_zm, li); li = fma(-s.uzs_zm, s.pr_zm, li);
    const T v = fma(s.pr, s.pr, s.pm * s.pm) - k.s2;
    const T cv = k.c3 * v;
    SiteNew<T> o;
    o.pr = fma(k.c1, s.pr0, fma(k.c2, lr, -(cv * s.pr)));
    o.pi = fma(k.c1, s.pi0, fma(k.c2, li, -(cv * s.pm)));

    // Eq. (5): current Im[conj(phi(x+i)) conj(U_i(x)) phi(x)] and the lattice curl
    const T wxr = fma(s.uxc, s.pr, s.uxs * s.pm), wxi = fma(s.uxc, s.pm, -(s.uxs * s.pr));
    const T wyr = fma(s.uyc, s.pr, s.uys * s.pm), wyi = fma(s.uyc, s.pm, -(s.uys * s.pr));
    const T wzr = fma(s.uzc, s.pr, s.uzs * s.pm), wzi = fma(s.uzc, s.pm, -(s.uzs * s.pr));
    const T jx = fma(s.pr_xp, wxi, -(s.pi_xp * wxr));
    const T jy = fma(s.pr_yp, wyi, -(s.pi_yp * wyr));
    const T jz = fma(s.pr_zp, wzi, -(s.pi_zp * wzr));
    const T curl_x = (s.pxy - s.pxy_ym) - (s.pzx - s.pzx_zm);
    const T curl_y = (s.pyz - s.pyz_zm) - (s.pxy - s.pxy_xm);
    const T curl_z = (s.pzx - s.pzx_xm) - (s.pyz - s.pyz_ym);
    o.ex = fma(k.d1, s.ex0, fma(k.d3, jx, -(k.d2 * curl_x)));
    o.ey = fma(k.d1, s.ey0, fma(k.d3, jy, -(k.d2 * curl_y)));
    o.ez = fma(k.d1, s.ez0, fma(k.d3, jz, -(k.d2 * curl_z)));

    // Eqs. (6)-(7)
    o.qr = fma(k.dt, o.pr, s.pr);
    o.qi = fma(k.dt, o.pi, s.pm);
    o.ax = fma(k.dt, o.ex, s.ax);
    o.ay = fma(k.dt, o.ey, s.ay);
    o.az = fma(k.dt, o.ez, s.az);
    return o;
}

__device__ __forceinline__ int wrap_mod(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// Per-thread FP64 accumulators of one measurement of S_n (Eqs. (9)-(12)),
// with the a-dependent weights of the conformal densities.
struct MeasAcc {
    double s[A_COUNT];
    int c[C_COUNT];        // per thread at most 3 per plane of one column: 32 bits suffice
    double a2, g, h, idx2, s2;
};

__device__ __forceinline__ void meas_init(MeasAcc &m, const RealDesc &d, const Coef &c) {
    for (int k = 0; k < A_COUNT; ++k)
        m.s[k] = 0.0;
    for (int k = 0; k < C_COUNT; ++k)
        m.c[k] = 0;
    m.a2 = c.a_0 * c.a_0;
    m.g = pow(c.a_0, 2.0 * (1.0 - c.s_0)) / (2.0 * d.e0 * d.e0);
    m.h = d.lambda0 * pow(c.a_0, 2.0 + 2.0 * c.s_0);
    m.idx2 = 1.0 / (d.dx * d.dx);
    m.s2 = d.sigma * d.sigma;
}

// What the densities of site x read: its fields and phasors, phi at x+x,
// x+y, x+z, and the phasors of the other links of its three forward
// plaquettes.
template <typename T> struct MeasSite {
    T pr, pm, pr0, pi0, ax, ay, az, ex0, ey0, ez0;
    T uxc, uxs, uyc, uys, uzc, uzs;
    T pr_xp, pi_xp, pr_yp, pi_yp, pr_zp, pi_zp;
    T uyc_xp, uys_xp, uzc_xp, uzs_xp, uxc_yp, uxs_yp, uzc_yp, uzs_yp, uxc_zp, uxs_zp, uyc_zp, uys_zp;
};

// Add site x of S_n to the accumulators: the densities of Eqs. (9)-(10) and
// the pressure of Eq. (12), formed in the storage precision T and summed in
// FP64.  Returns false (and counts the site) when a field is not finite.
// The pressure is linear in the five parts of the energy density, so its sum
// is formed from theirs when the measurement is finalised.
template <typename T>
__device__ __forceinline__ bool measure_densities(MeasAcc &m, const MeasSite<T> &v) {
    // every multiply-add written out and contraction off: the per-site values
    // are bitwise the same in every kernel that measures (the fused measuring
    // step, the read-only pass, the batched kernel)
#pragma clang fp contract(off)
    const bool finite = __builtin_isfinite(v.pr) && __builtin_isfinite(v.pm) &&
                        __builtin_isfinite(v.pr0) && __builtin_isfinite(v.pi0) &&
                        __builtin_isfinite(v.ax) && __builtin_isfinite(v.ay) &&
                        __builtin_isfinite(v.az) && __builtin_isfinite(v.ex0) &&
                        __builtin_isfinite(v.ey0) && __builtin_isfinite(v.ez0);
    if (!finite) {
        m.c[C_NONFIN] += 1;
        return false;
    }
    const T pr = v.pr, pm = v.pm;
    // e^{iA_i} phi(x+i) - phi(x)
    const T gxr = fma(v.uxc, v.pr_xp, fma(-v.uxs, v.pi_xp, -pr));
    const T gxi = fma(v.uxc, v.pi_xp, fma(v.uxs, v.pr_xp, -pm));
    const T gyr = fma(v.uyc, v.pr_yp, fma(-v.uys, v.pi_yp, -pr));
    const T gyi = fma(v.uyc, v.pi_yp, fma(v.uys, v.pr_yp, -pm));
    const T gzr = fma(v.uzc, v.pr_zp, fma(-v.uzs, v.pi_zp, -pr));
    const T gzi = fma(v.uzc, v.pi_zp, fma(v.uzs, v.pr_zp, -pm));
    const T idx2 = (T)m.idx2, a2 = (T)m.a2, g = (T)m.g, h = (T)m.h;
    const T K = fma(v.pr0, v.pr0, v.pi0 * v.pi0);
    const T gs = fma(gxr, gxr, fma(gxi, gxi, fma(gyr, gyr, fma(gyi, gyi, fma(gzr, gzr, gzi * gzi)))));
    const T Gr = idx2 * gs;
    const T EE = idx2 * fma(v.ex0, v.ex0, fma(v.ey0, v.ey0, v.ez0 * v.ez0));
    const T oxy = plaq_omc(v.uxc, v.uxs, v.uyc_xp, v.uys_xp, v.uxc_yp, v.uxs_yp, v.uyc, v.uys);
    const T oyz = plaq_omc(v.uyc, v.uys, v.uzc_yp, v.uzs_yp, v.uyc_zp, v.uys_zp, v.uzc, v.uzs);
    const T ozx = plaq_omc(v.uzc, v.uzs, v.uxc_zp, v.uxs_zp, v.uzc_xp, v.uzs_xp, v.uxc, v.uxs);
    const T BB = ((T)2 * idx2 * idx2) * ((oxy + oyz) + ozx);
    // |phi|^2 - sigma^2 in FP64: near the vacuum it is a small difference of
    // numbers near sigma^2, which the storage precision would not resolve
    const double vv = fma((double)pr, (double)pr, fma((double)pm, (double)pm, -m.s2));
    const T V = (T)(0.25 * (vv * vv));
    const T kin = a2 * K, grad = a2 * Gr, elec = g * EE, mag = g * BB, pot = h * V;
    const T lag = ((kin - grad) + (elec - mag)) - pot;
    const T rho = ((kin + grad) + (elec + mag)) + pot;
    const T third = (T)(1.0 / 3.0);
    const T pres = fma(elec + mag, third, fma(-grad, third, kin)) - pot;
    m.s[A_KIN] += (double)kin;
    m.s[A_GRAD] += (double)grad;
    m.s[A_ELEC] += (double)elec;
    m.s[A_MAG] += (double)mag;
    m.s[A_POT] += (double)pot;
    m.s[A_LAG] += (double)lag;
    m.s[A_NUM_L] += (double)(K * lag);
    m.s[A_NUM_V] += (double)(K * V);
    m.s[A_NUM_R] += (double)(K * rho);
    m.s[A_DEN_L] += (double)(Gr * lag);
    m.s[A_DEN_V] += (double)(Gr * V);
    m.s[A_DEN_R] += (double)(Gr * rho);
    m.s[A_PRES_L] += (double)(pres * lag);
    m.s[A_RHO_L] += (double)(rho * lag);
    return true;
}

// Add the windings of the three forward plaquettes of a site (Eq. (11)) to
// the counters.
__device__ __forceinline__ void count_windings(MeasAcc &m, const int (&w3)[3]) {
    for (int k = 0; k < 3; ++k) {
        m.c[C_W0 + k] += w3[k];
        m.c[C_N0 + k] += w3[k] < 0 ? -w3[k] : w3[k];
        m.c[C_PIERCED] += w3[k] != 0 ? 1 : 0;
    }
}

// Block-wide reduction of the accumulators into the measurement slot; every
// thread of the block (NW wavefronts) calls it.
template <int NW>
__device__ __forceinline__ void meas_commit(MeasAcc &m, Slot *slot, const Coef &c, bool first) {
    if (first && threadIdx.x == 0) {
        slot->c = c;
        slot->measured = 1;
    }
    unsigned long long cnt64[C_COUNT];
    for (int k = 0; k < C_COUNT; ++k)
        cnt64[k] = (unsigned long long)(long long)m.c[k];   // two's complement for W sums
    block_accumulate<A_COUNT, C_COUNT, NW>(m.s, cnt64, slot->acc.s, slot->acc.c);
    __syncthreads();   // the reduction's LDS is reused by the next tile of a batch
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b on XCD
// b % 8).  This bijection of [0, nb) gives XCD i the contiguous run
// [start_i, start_i + count_i) of tile numbers, so tiles that share halo rows
// run on one XCD and meet in its L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int xcd = b & 7, per = nb >> 3, rem = nb & 7;
    return xcd * per + min(xcd, rem) + (b >> 3);
}

// One tile (64 x TY sites, planes [z0, z0 + cz)) of one realization, tiles
// numbered x-fastest, then y, then z-chunk.  Every thread of the block calls
// it with the same arguments.
template <typename T, int TY, int MODE>
__device__ __forceinline__ void tiled_tile(const RealDesc &d, const Coef &c, int tile, int cz,
                                           Slot *slot) {
    constexpr bool MEAS = MODE != MODE_STEP;
    using G = TileGeom<TY>;
    constexpr int SM = MEAS ? G::S : 1;
    __shared__ T lds[2][Q_COUNT][G::S];
    __shared__ float lth[2][SM];       // FP32 phase of phi (measuring modes)
    __shared__ T lar[2][3][SM];        // raw link angles (measuring modes)
    __shared__ int lcnt[2][2][SM];     // wrap counts of the x and y links (measuring modes)

    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const int ntx = nx >> 6, nty = (ny + TY - 1) / TY;
    const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
    const int x0 = tx << 6, y0 = ty * TY, z0 = tz * cz;
    const int z1 = min(z0 + cz, nz);

    const int t = threadIdx.x, lx = t & 63, ly = t >> 6;
    const int gx = x0 + lx;
    const bool owner = (y0 + ly) < ny;       // rows past a ragged tile edge only stage data
    const int gy = wrap_mod(y0 + ly, ny);
    const int q = G::li(lx, ly);

    const int par = c.parity, L = d.layout;
    const gptr<const T> phr = gplane<const T>(d, field_plane(0, par, L));
    const gptr<const T> phi = gplane<const T>(d, field_plane(1, par, L));
    const gptr<const T> A0 = gplane<const T>(d, field_plane(4, par, L));
    const gptr<const T> A1 = gplane<const T>(d, field_plane(5, par, L));
    const gptr<const T> A2 = gplane<const T>(d, field_plane(6, par, L));
    const gptr<const T> pir = gplane<const T>(d, field_plane(2, par, L));
    const gptr<const T> pii = gplane<const T>(d, field_plane(3, par, L));
    const gptr<const T> E0 = gplane<const T>(d, field_plane(7, par, L));
    const gptr<const T> E1 = gplane<const T>(d, field_plane(8, par, L));
    const gptr<const T> E2 = gplane<const T>(d, field_plane(9, par, L));
    // the new state: phi, A always to the other copy; Pi, E in place in the
    // 15-plane layout (each thread reads them only at its own site)
    gptr<T> o[10];
    for (int f = 0; f < 10; ++f)
        o[f] = gplane<T>(d, field_plane(f, par ^ 1, L));

    const StepK<T> K = step_k<T>(d, c);

    // per-thread FP64 accumulators of the measuring modes
    MeasAcc macc;
    if (MEAS)
        meas_init(macc, d, c);

    auto load_site = [&](int s, SiteV<T> &v) {
        v.pr = phr[s];
        v.pm = phi[s];
        v.ax = A0[s];
        v.ay = A1[s];
        v.az = A2[s];
        sincos_t(v.ax, &v.uxs, &v.uxc);
        sincos_t(v.ay, &v.uys, &v.uyc);
        sincos_t(v.az, &v.uzs, &v.uzc);
        if (MEAS)
            v.th = phase_f32((float)v.pm, (float)v.pr);
    };
    auto put = [&](int bf, int k, const SiteV<T> &v) {
        lds[bf][Q_PR][k] = v.pr;
        lds[bf][Q_PI][k] = v.pm;
        lds[bf][Q_UXC][k] = v.uxc;
        lds[bf][Q_UXS][k] = v.uxs;
        lds[bf][Q_UYC][k] = v.uyc;
        lds[bf][Q_UYS][k] = v.uys;
        lds[bf][Q_UZC][k] = v.uzc;
        lds[bf][Q_UZS][k] = v.uzs;
        if (MEAS) {
            lth[bf][k] = v.th;
            lar[bf][0][k] = v.ax;
            lar[bf][1][k] = v.ay;
            lar[bf][2][k] = v.az;
        }
    };
    auto stage_halo = [&](int bf, int z) {
        for (int h = t; h < G::HALO; h += 64 * TY) {
            int hx, hy;
            G::halo(h, hx, hy);
            const int s = wrap_mod(x0 + hx, nx) + nx * (wrap_mod(y0 + hy, ny) + ny * z);
            SiteV<T> v;
            load_site(s, v);
            put(bf, G::li(hx, hy), v);
        }
    };
    auto own = [&](int z) { return gx + nx * (gy + ny * z); };

    // Wrap count of the link from LDS site ka to kb (same buffer bf) with raw
    // angle a: FP32 phases, FP64 phases when the quotient is too close to call.
    auto link_count = [&](int bf, int ka, int kb, T a) {
        int m;
        if (!wrap_count_f32(lth[bf][ka], lth[bf][kb], (float)a, m))
            m = wrap_count(phase64(lds[bf][Q_PR][kb], lds[bf][Q_PI][kb]) -
                           phase64(lds[bf][Q_PR][ka], lds[bf][Q_PI][ka]) + (double)a);
        return m;
    };
    // In-plane wrap counts of plane buffer bf: this thread's own site (x and y
    // links, raw angles ax, ay) and the halo sites it staged whose links the
    // tile's plaquettes use (the x link of the row above, the y link of the
    // column to the right).  Returns the own counts.
    auto plane_counts = [&](int bf, T ax, T ay, int &mx, int &my) {
        int cx, cy;
        const bool sx = wrap_count_f32(lth[bf][q], lth[bf][q + 1], (float)ax, cx);
        const bool sy = wrap_count_f32(lth[bf][q], lth[bf][q + G::W], (float)ay, cy);
        if (!(sx && sy)) {
            const double e = phase64(lds[bf][Q_PR][q], lds[bf][Q_PI][q]);
            cx = wrap_count(phase64(lds[bf][Q_PR][q + 1], lds[bf][Q_PI][q + 1]) - e + (double)ax);
            cy = wrap_count(phase64(lds[bf][Q_PR][q + G::W], lds[bf][Q_PI][q + G::W]) - e +
                            (double)ay);
        }
        lcnt[bf][0][q] = cx;
        lcnt[bf][1][q] = cy;
        mx = cx;
        my = cy;
        for (int h = t; h < G::HALO; h += 64 * TY) {
            int hx, hy;
            G::halo(h, hx, hy);
            const int k = G::li(hx, hy);
            if (hy == TY && hx >= 0 && hx < 64)
                lcnt[bf][0][k] = link_count(bf, k, k + 1, lar[bf][0][k]);
            else if (hx == 64 && hy >= 0 && hy < TY)
                lcnt[bf][1][k] = link_count(bf, k, k + G::W, lar[bf][1][k]);
        }
    };

    // prologue: planes z0-1 (buffer 1) and z0 (buffer 0); z below is
    // slab-relative, zmap gives the stored plane
    const int zm0 = zmap(d, z0 - 1), zc0 = zmap(d, z0);
    SiteV<T> prv, cur, nxt;
    load_site(own(zm0), prv);
    put(1, q, prv);
    stage_halo(1, zm0);
    load_site(own(zc0), cur);
    put(0, q, cur);
    stage_halo(0, zc0);
    __syncthreads();
    // yz and zx plaquettes of plane z0-1 at this column
    T pyz_m = plaq_sin(prv.uyc, prv.uys, lds[1][Q_UZC][q + G::W], lds[1][Q_UZS][q + G::W],
                       cur.uyc, cur.uys, prv.uzc, prv.uzs);
    T pzx_m = plaq_sin(prv.uzc, prv.uzs, cur.uxc, cur.uxs, lds[1][Q_UZC][q + 1],
                       lds[1][Q_UZS][q + 1], prv.uxc, prv.uxs);
    T phr_m = prv.pr, phi_m = prv.pm, uzc_m = prv.uzc, uzs_m = prv.uzs;
    // wrap counts of the in-plane links of plane z0
    int mx_c = 0, my_c = 0;
    if (MEAS)
        plane_counts(0, cur.ax, cur.ay, mx_c, my_c);
    __syncthreads();

    for (int z = z0; z < z1; ++z) {
        const int cb = (z - z0) & 1, nb_ = cb ^ 1;
        const int zp = zmap(d, z + 1);
        const int s = own(zmap(d, z));
        // the momenta are read once, by this thread only: streaming loads
        const T pr0 = __builtin_nontemporal_load(pir + s), pi0 = __builtin_nontemporal_load(pii + s);
        const T ex0 = __builtin_nontemporal_load(E0 + s), ey0 = __builtin_nontemporal_load(E1 + s);
        const T ez0 = __builtin_nontemporal_load(E2 + s);
        load_site(own(zp), nxt);
        put(nb_, q, nxt);
        stage_halo(nb_, zp);
        __syncthreads();

        const T(*L)[G::S] = lds[cb];
        const T(*Ln)[G::S] = lds[nb_];
        // phi neighbours in the plane
        const T pr_xp = L[Q_PR][q + 1], pi_xp = L[Q_PI][q + 1];
        const T pr_xm = L[Q_PR][q - 1], pi_xm = L[Q_PI][q - 1];
        const T pr_yp = L[Q_PR][q + G::W], pi_yp = L[Q_PI][q + G::W];
        const T pr_ym = L[Q_PR][q - G::W], pi_ym = L[Q_PI][q - G::W];
        // link phasors around the site
        const T uxc_xm = L[Q_UXC][q - 1], uxs_xm = L[Q_UXS][q - 1];
        const T uxc_yp = L[Q_UXC][q + G::W], uxs_yp = L[Q_UXS][q + G::W];
        const T uxc_xmyp = L[Q_UXC][q - 1 + G::W], uxs_xmyp = L[Q_UXS][q - 1 + G::W];
        const T uxc_ym = L[Q_UXC][q - G::W], uxs_ym = L[Q_UXS][q - G::W];
        const T uyc_xp = L[Q_UYC][q + 1], uys_xp = L[Q_UYS][q + 1];
        const T uyc_ym = L[Q_UYC][q - G::W], uys_ym = L[Q_UYS][q - G::W];
        const T uyc_xm = L[Q_UYC][q - 1], uys_xm = L[Q_UYS][q - 1];
        const T uyc_xpym = L[Q_UYC][q + 1 - G::W], uys_xpym = L[Q_UYS][q + 1 - G::W];
        const T uzc_xp = L[Q_UZC][q + 1], uzs_xp = L[Q_UZS][q + 1];
        const T uzc_yp = L[Q_UZC][q + G::W], uzs_yp = L[Q_UZS][q + G::W];
        const T uzc_xm = L[Q_UZC][q - 1], uzs_xm = L[Q_UZS][q - 1];
        const T uzc_ym = L[Q_UZC][q - G::W], uzs_ym = L[Q_UZS][q - G::W];
        const T uxc_xmzp = Ln[Q_UXC][q - 1], uxs_xmzp = Ln[Q_UXS][q - 1];
        const T uyc_ymzp = Ln[Q_UYC][q - G::W], uys_ymzp = Ln[Q_UYS][q - G::W];

        // plaquette sines (Eq. (3))
        const T pxy = plaq_sin(cur.uxc, cur.uxs, uyc_xp, uys_xp, uxc_yp, uxs_yp, cur.uyc, cur.uys);
        const T pxy_xm = plaq_sin(uxc_xm, uxs_xm, cur.uyc, cur.uys, uxc_xmyp, uxs_xmyp, uyc_xm, uys_xm);
        const T pxy_ym = plaq_sin(uxc_ym, uxs_ym, uyc_xpym, uys_xpym, cur.uxc, cur.uxs, uyc_ym, uys_ym);
        const T pyz = plaq_sin(cur.uyc, cur.uys, uzc_yp, uzs_yp, nxt.uyc, nxt.uys, cur.uzc, cur.uzs);
        const T pyz_ym = plaq_sin(uyc_ym, uys_ym, cur.uzc, cur.uzs, uyc_ymzp, uys_ymzp, uzc_ym, uzs_ym);
        const T pzx = plaq_sin(cur.uzc, cur.uzs, nxt.uxc, nxt.uxs, uzc_xp, uzs_xp, cur.uxc, cur.uxs);
        const T pzx_xm = plaq_sin(uzc_xm, uzs_xm, uxc_xmzp, uxs_xmzp, cur.uzc, cur.uzs, uxc_xm, uxs_xm);

        const T pr = cur.pr, pm = cur.pm;
        {
            Stencil<T> st;
            st.pr = pr; st.pm = pm; st.ax = cur.ax; st.ay = cur.ay; st.az = cur.az;
            st.uxc = cur.uxc; st.uxs = cur.uxs; st.uyc = cur.uyc; st.uys = cur.uys;
            st.uzc = cur.uzc; st.uzs = cur.uzs;
            st.pr0 = pr0; st.pi0 = pi0; st.ex0 = ex0; st.ey0 = ey0; st.ez0 = ez0;
            st.pr_xp = pr_xp; st.pi_xp = pi_xp; st.pr_xm = pr_xm; st.pi_xm = pi_xm;
            st.pr_yp = pr_yp; st.pi_yp = pi_yp; st.pr_ym = pr_ym; st.pi_ym = pi_ym;
            st.pr_zp = nxt.pr; st.pi_zp = nxt.pm; st.pr_zm = phr_m; st.pi_zm = phi_m;
            st.uxc_xm = uxc_xm; st.uxs_xm = uxs_xm; st.uyc_ym = uyc_ym; st.uys_ym = uys_ym;
            st.uzc_zm = uzc_m; st.uzs_zm = uzs_m;
            st.pxy = pxy; st.pxy_xm = pxy_xm; st.pxy_ym = pxy_ym;
            st.pyz = pyz; st.pyz_ym = pyz_ym; st.pyz_zm = pyz_m;
            st.pzx = pzx; st.pzx_xm = pzx_xm; st.pzx_zm = pzx_m;
            const SiteNew<T> nw = leapfrog_site(st, K);
            if (owner) {
                // streaming stores: the new state is not read again in this launch
                __builtin_nontemporal_store(nw.pr, o[2] + s);
                __builtin_nontemporal_store(nw.pi, o[3] + s);
                __builtin_nontemporal_store(nw.ex, o[7] + s);
                __builtin_nontemporal_store(nw.ey, o[8] + s);
                __builtin_nontemporal_store(nw.ez, o[9] + s);
                __builtin_nontemporal_store(nw.qr, o[0] + s);
                __builtin_nontemporal_store(nw.qi, o[1] + s);
                __builtin_nontemporal_store(nw.ax, o[4] + s);
                __builtin_nontemporal_store(nw.ay, o[5] + s);
                __builtin_nontemporal_store(nw.az, o[6] + s);
            }
        }

        if (MEAS) {
            // wrap counts: the in-plane links of plane z+1 (this column and
            // the halo), the z links of plane z at x, x+x and x+y
            int mx_n, my_n;
            plane_counts(nb_, nxt.ax, nxt.ay, mx_n, my_n);
            int mz, mz_xp, mz_yp;
            const bool s0 = wrap_count_f32(cur.th, nxt.th, (float)cur.az, mz);
            const bool s1 = wrap_count_f32(lth[cb][q + 1], lth[nb_][q + 1],
                                           (float)lar[cb][2][q + 1], mz_xp);
            const bool s2 = wrap_count_f32(lth[cb][q + G::W], lth[nb_][q + G::W],
                                           (float)lar[cb][2][q + G::W], mz_yp);
            if (!(s0 && s1 && s2)) {
                mz = wrap_count(phase64(nxt.pr, nxt.pm) - phase64(pr, pm) + (double)cur.az);
                mz_xp = wrap_count(phase64(Ln[Q_PR][q + 1], Ln[Q_PI][q + 1]) -
                                   phase64(pr_xp, pi_xp) + (double)lar[cb][2][q + 1]);
                mz_yp = wrap_count(phase64(Ln[Q_PR][q + G::W], Ln[Q_PI][q + G::W]) -
                                   phase64(pr_yp, pi_yp) + (double)lar[cb][2][q + G::W]);
            }
            const int my_xp = lcnt[cb][1][q + 1], mx_yp = lcnt[cb][0][q + G::W];
            if (owner) {
                // Eqs. (9)-(12) for the site of S_n read above
                MeasSite<T> mv;
                mv.pr = pr; mv.pm = pm; mv.pr0 = pr0; mv.pi0 = pi0;
                mv.ax = cur.ax; mv.ay = cur.ay; mv.az = cur.az;
                mv.ex0 = ex0; mv.ey0 = ey0; mv.ez0 = ez0;
                mv.uxc = cur.uxc; mv.uxs = cur.uxs; mv.uyc = cur.uyc; mv.uys = cur.uys;
                mv.uzc = cur.uzc; mv.uzs = cur.uzs;
                mv.pr_xp = pr_xp; mv.pi_xp = pi_xp; mv.pr_yp = pr_yp; mv.pi_yp = pi_yp;
                mv.pr_zp = nxt.pr; mv.pi_zp = nxt.pm;
                mv.uyc_xp = uyc_xp; mv.uys_xp = uys_xp; mv.uzc_xp = uzc_xp; mv.uzs_xp = uzs_xp;
                mv.uxc_yp = uxc_yp; mv.uxs_yp = uxs_yp; mv.uzc_yp = uzc_yp; mv.uzs_yp = uzs_yp;
                mv.uxc_zp = nxt.uxc; mv.uxs_zp = nxt.uxs; mv.uyc_zp = nxt.uyc; mv.uys_zp = nxt.uys;
                int w3[3] = { 0, 0, 0 };
                if (measure_densities(macc, mv)) {
                    // Eq. (11): W_ij = -(m_i(x) + m_j(x+i) - m_i(x+j) - m_j(x))
                    w3[0] = -(mx_c + my_xp - mx_yp - my_c);
                    w3[1] = -(my_c + mz_yp - my_n - mz);
                    w3[2] = -(mz + mx_n - mz_xp - mx_c);
                    count_windings(macc, w3);
                }
            }
            mx_c = mx_n;
            my_c = my_n;
        }

        phr_m = pr;
        phi_m = pm;
        uzc_m = cur.uzc;
        uzs_m = cur.uzs;
        pyz_m = pyz;
        pzx_m = pzx;
        cur = nxt;
        __syncthreads();
    }

    if (MEAS)
        meas_commit<TY>(macc, slot, c, tile == 0);
}

// One realization: one block per tile, tiles [tile0, tile0 + gridDim.x).
template <typename T, int TY, int MODE>
__global__ void __launch_bounds__(64 * TY)
k_step_tiled(const RealDesc *descs, const Coef *coefs, int r, int cz, Slot *slot, int tile0) {
    const RealDesc d = descs[r];
    const Coef c = coefs[r];
    if (!c.active)
        return;
    tiled_tile<T, TY, MODE>(d, c, tile0 + xcd_remap(blockIdx.x, gridDim.x), cz, slot);
}

// Many realizations in one launch: a persistent grid walks the item list in
// rounds of gridDim.x items; within a round the XCD remap keeps consecutive
// items (neighbouring tiles of one realization) on one XCD.  Realizations
// that reached their n_end are skipped.  In the measuring mode every active
// realization r measures into slots[r].
template <typename T, int TY, int MODE>
__global__ void __launch_bounds__(64 * TY)
k_step_batch(const RealDesc *descs, const Coef *coefs, const BatchItem *items, int n_items,
             Slot *slots) {
    const int g = gridDim.x;
    const int b = xcd_remap(blockIdx.x, g);
    for (int base = 0; base < n_items; base += g) {
        const int it = base + b;
        if (it >= n_items)
            break;
        const BatchItem item = items[it];
        const Coef c = coefs[item.r];
        if (!c.active)
            continue;
        const RealDesc d = descs[item.r];
        tiled_tile<T, TY, MODE>(d, c, item.tile, item.cz,
                                MODE == MODE_STEP ? nullptr : slots + item.r);
    }
}

} // namespace ah
