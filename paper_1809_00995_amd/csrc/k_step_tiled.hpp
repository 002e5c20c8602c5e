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
// S_n (the state it reads) on the way; MODE_MEASURE only measures (and can
// write the per-plaquette winding map).  The measuring modes stage arg(phi)
// in FP64 and the raw link angles A_i next to the phasors, and count the
// winding of each plaquette from the wrap counts of its four links:
// with m_i(s) = floor((theta(s+i) - theta(s) + A_i(s) + pi) / 2 pi) the
// [.]_pi of Eq. (11) subtracts 2 pi m_i, the phase differences cancel around
// the plaquette, and W_ij = -(m_i(x) + m_j(x+i) - m_i(x+j) - m_j(x)) exactly.
#pragma once

#include <type_traits>

#include "ah_device.hpp"

namespace ah {

enum : int { MODE_STEP = 0, MODE_STEP_MEASURE = 1, MODE_MEASURE = 2 };

// quantities staged per site in LDS
enum : int { Q_PR, Q_PI, Q_UXC, Q_UXS, Q_UYC, Q_UYS, Q_UZC, Q_UZS, Q_COUNT };

template <int TY> struct TileGeom {
    static constexpr int W = 66;              // 64 sites + 1 halo site each side
    static constexpr int H = TY + 2;
    static constexpr int S = W * H;
    static constexpr int HALO = 2 * 64 + 2 * H;   // halo ring, corners included
    static __device__ __forceinline__ int li(int lx, int ly) { return (ly + 1) * W + (lx + 1); }
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

// The measuring kernels decide wrap counts on FP32 phases (phase_f32, error
// below 5e-7) and fall back to FP64 phases (atan2) for every link of a site
// when any of its quotients (u + pi) / 2 pi lies within kWrapMargin of an
// integer: the two sets of phases move a quotient by at most ~1.6e-7, so
// outside the margin both give the same integer, and the counts equal those
// of FP64 phases everywhere.
constexpr double kWrapMargin = 4e-6;

// m = wrap_count(u) from FP32 phases; false when the FP64 phases must decide
// (u within the margin of a boundary, or not a number).
__device__ __forceinline__ bool wrap_count_sure(double u, int &m) {
    const double w = (u + kPi) * kInvTwoPi;
    const double f = floor(w);
    m = (int)f;
    const double fr = w - f;
    return fr > kWrapMargin && fr < 1.0 - kWrapMargin;
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

// What the measurement of site x reads: its fields and phasors, phi at
// x+x, x+y, x+z, the phasors of the other links of its three forward
// plaquettes, and the FP32 phases of phi and the raw link angles at the
// corners of those plaquettes.
template <typename T> struct MeasSite {
    T pr, pm, pr0, pi0, ax, ay, az, ex0, ey0, ez0;
    T uxc, uxs, uyc, uys, uzc, uzs;
    T pr_xp, pi_xp, pr_yp, pi_yp, pr_zp, pi_zp;
    T uyc_xp, uys_xp, uzc_xp, uzs_xp, uxc_yp, uxs_yp, uzc_yp, uzs_yp, uxc_zp, uxs_zp, uyc_zp, uys_zp;
    float th, th_xp, th_yp, th_xpyp, th_zp, th_xpzp, th_ypzp;
    double ay_xp, az_xp, ax_yp, az_yp, ax_zp, ay_zp;
};

// phi at the corners x+x+y, x+x+z, x+y+z of the forward plaquettes (read
// only when the winding falls back to FP64 phases).
template <typename T> struct Corners {
    T pr_xpyp, pi_xpyp, pr_xpzp, pi_xpzp, pr_ypzp, pi_ypzp;
};

// Add site x of S_n to the accumulators: the densities of Eqs. (9)-(10), the
// pressure of Eq. (12), and the windings of its xy, yz, zx plaquettes
// (Eq. (11)) from the wrap counts of their links; w3 receives the windings.
// corners() returns the Corners of the site.
template <typename T, typename CornersFn>
__device__ __forceinline__ void measure_site(MeasAcc &m, const MeasSite<T> &v, int (&w3)[3],
                                             CornersFn corners) {
    const bool finite = __builtin_isfinite(v.pr) && __builtin_isfinite(v.pm) &&
                        __builtin_isfinite(v.pr0) && __builtin_isfinite(v.pi0) &&
                        __builtin_isfinite(v.ax) && __builtin_isfinite(v.ay) &&
                        __builtin_isfinite(v.az) && __builtin_isfinite(v.ex0) &&
                        __builtin_isfinite(v.ey0) && __builtin_isfinite(v.ez0);
    w3[0] = w3[1] = w3[2] = 0;
    if (!finite) {
        m.c[C_NONFIN] += 1;
        return;
    }
    const T pr = v.pr, pm = v.pm;
    const T gxr = v.uxc * v.pr_xp - v.uxs * v.pi_xp - pr;
    const T gxi = v.uxc * v.pi_xp + v.uxs * v.pr_xp - pm;
    const T gyr = v.uyc * v.pr_yp - v.uys * v.pi_yp - pr;
    const T gyi = v.uyc * v.pi_yp + v.uys * v.pr_yp - pm;
    const T gzr = v.uzc * v.pr_zp - v.uzs * v.pi_zp - pr;
    const T gzi = v.uzc * v.pi_zp + v.uzs * v.pr_zp - pm;
    const double idx2 = m.idx2, ma2 = m.a2, mg = m.g, mh = m.h;
    const double K = (double)v.pr0 * v.pr0 + (double)v.pi0 * v.pi0;
    const double Gr = idx2 * ((double)gxr * gxr + (double)gxi * gxi + (double)gyr * gyr +
                              (double)gyi * gyi + (double)gzr * gzr + (double)gzi * gzi);
    const double EE = idx2 * ((double)v.ex0 * v.ex0 + (double)v.ey0 * v.ey0 + (double)v.ez0 * v.ez0);
    const T oxy = plaq_omc(v.uxc, v.uxs, v.uyc_xp, v.uys_xp, v.uxc_yp, v.uxs_yp, v.uyc, v.uys);
    const T oyz = plaq_omc(v.uyc, v.uys, v.uzc_yp, v.uzs_yp, v.uyc_zp, v.uys_zp, v.uzc, v.uzs);
    const T ozx = plaq_omc(v.uzc, v.uzs, v.uxc_zp, v.uxs_zp, v.uzc_xp, v.uzs_xp, v.uxc, v.uxs);
    const double BB = 2.0 * idx2 * idx2 * ((double)oxy + (double)oyz + (double)ozx);
    const double vv = (double)pr * pr + (double)pm * pm - m.s2;
    const double V = 0.25 * vv * vv;
    const double lag = ma2 * K - ma2 * Gr + mg * (EE - BB) - mh * V;
    const double rho = ma2 * K + ma2 * Gr + mg * (EE + BB) + mh * V;
    // the thirds as products with 1/3 (two FP64 divisions per site saved; the
    // results differ from the quotients by at most an ulp of each term)
    constexpr double kThird = 1.0 / 3.0;
    const double pres = ma2 * K - (ma2 * Gr) * kThird + (mg * (EE + BB)) * kThird - mh * V;
    m.s[A_KIN] += ma2 * K;
    m.s[A_GRAD] += ma2 * Gr;
    m.s[A_ELEC] += mg * EE;
    m.s[A_MAG] += mg * BB;
    m.s[A_POT] += mh * V;
    m.s[A_LAG] += lag;
    m.s[A_NUM_L] += K * lag;
    m.s[A_NUM_V] += K * V;
    m.s[A_NUM_R] += K * rho;
    m.s[A_DEN_L] += Gr * lag;
    m.s[A_DEN_V] += Gr * V;
    m.s[A_DEN_R] += Gr * rho;
    m.s[A_PRES] += pres;
    m.s[A_PRES_L] += pres * lag;
    m.s[A_RHO_L] += rho * lag;

    // winding (Eq. (11)) from link wrap counts: FP32 phases, FP64 near a boundary
    const double ax = v.ax, ay = v.ay, az = v.az;
    const double t = v.th, t_xp = v.th_xp, t_yp = v.th_yp, t_zp = v.th_zp;
    const double t_xpyp = v.th_xpyp, t_xpzp = v.th_xpzp, t_ypzp = v.th_ypzp;
    int mx, my, mz, my_xp, mx_yp, mz_yp, my_zp, mx_zp, mz_xp;
    bool sure = wrap_count_sure(t_xp - t + ax, mx);
    sure &= wrap_count_sure(t_yp - t + ay, my);
    sure &= wrap_count_sure(t_zp - t + az, mz);
    sure &= wrap_count_sure(t_xpyp - t_xp + v.ay_xp, my_xp);
    sure &= wrap_count_sure(t_xpyp - t_yp + v.ax_yp, mx_yp);
    sure &= wrap_count_sure(t_ypzp - t_yp + v.az_yp, mz_yp);
    sure &= wrap_count_sure(t_ypzp - t_zp + v.ay_zp, my_zp);
    sure &= wrap_count_sure(t_xpzp - t_zp + v.ax_zp, mx_zp);
    sure &= wrap_count_sure(t_xpzp - t_xp + v.az_xp, mz_xp);
    if (!sure) {
        const Corners<T> k = corners();
        const double e = atan2((double)v.pm, (double)v.pr);
        const double e_xp = atan2((double)v.pi_xp, (double)v.pr_xp);
        const double e_yp = atan2((double)v.pi_yp, (double)v.pr_yp);
        const double e_zp = atan2((double)v.pi_zp, (double)v.pr_zp);
        const double e_xpyp = atan2((double)k.pi_xpyp, (double)k.pr_xpyp);
        const double e_xpzp = atan2((double)k.pi_xpzp, (double)k.pr_xpzp);
        const double e_ypzp = atan2((double)k.pi_ypzp, (double)k.pr_ypzp);
        mx = wrap_count(e_xp - e + ax);
        my = wrap_count(e_yp - e + ay);
        mz = wrap_count(e_zp - e + az);
        my_xp = wrap_count(e_xpyp - e_xp + v.ay_xp);
        mx_yp = wrap_count(e_xpyp - e_yp + v.ax_yp);
        mz_yp = wrap_count(e_ypzp - e_yp + v.az_yp);
        my_zp = wrap_count(e_ypzp - e_zp + v.ay_zp);
        mx_zp = wrap_count(e_xpzp - e_zp + v.ax_zp);
        mz_xp = wrap_count(e_xpzp - e_xp + v.az_xp);
    }
    w3[0] = -(mx + my_xp - mx_yp - my);
    w3[1] = -(my + mz_yp - my_zp - mz);
    w3[2] = -(mz + mx_zp - mz_xp - mx);
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
                                           Slot *slot, int8_t *wind) {
    constexpr bool MEAS = MODE != MODE_STEP;
    constexpr bool UPD = MODE != MODE_MEASURE;
    using G = TileGeom<TY>;
    constexpr int SM = MEAS ? G::S : 1;
    __shared__ T lds[2][Q_COUNT][G::S];
    __shared__ float lth[2][SM];       // FP32 phase of phi (measuring modes)
    __shared__ T lar[2][3][SM];        // raw link angles (measuring modes)

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
        if (UPD) {
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

        if (MEAS && owner) {
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
            mv.th = cur.th; mv.th_xp = lth[cb][q + 1]; mv.th_yp = lth[cb][q + G::W];
            mv.th_xpyp = lth[cb][q + 1 + G::W];
            mv.th_zp = nxt.th; mv.th_xpzp = lth[nb_][q + 1]; mv.th_ypzp = lth[nb_][q + G::W];
            mv.ay_xp = lar[cb][1][q + 1]; mv.az_xp = lar[cb][2][q + 1];
            mv.ax_yp = lar[cb][0][q + G::W]; mv.az_yp = lar[cb][2][q + G::W];
            mv.ax_zp = nxt.ax; mv.ay_zp = nxt.ay;
            int w3[3];
            measure_site(macc, mv, w3, [&]() {
                Corners<T> k;
                k.pr_xpyp = L[Q_PR][q + 1 + G::W];
                k.pi_xpyp = L[Q_PI][q + 1 + G::W];
                k.pr_xpzp = Ln[Q_PR][q + 1];
                k.pi_xpzp = Ln[Q_PI][q + 1];
                k.pr_ypzp = Ln[Q_PR][q + G::W];
                k.pi_ypzp = Ln[Q_PI][q + G::W];
                return k;
            });
            if (MODE == MODE_MEASURE && wind)
                for (int k = 0; k < 3; ++k)
                    wind[(size_t)k * (size_t)d.N + s] = (int8_t)w3[k];
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
// The FP32 read-only measuring kernel at 4-row tiles needs 169 VGPRs unhinted (two
// wavefronts per SIMD); asked for three it fits in 168 with one register spilled and runs
// 17 % faster (2.78 -> 2.30 ms at 512^3).  The fused measuring step would spill
// under the same request (3.70 -> 4.33 ms), so it keeps the compiler's choice.
template <typename T, int TY, int MODE>
__global__ void __launch_bounds__(64 * TY)
__attribute__((amdgpu_waves_per_eu(std::is_same<T, float>::value && MODE == MODE_MEASURE &&
                                           TY == 4 ? 3 : 1)))
k_step_tiled(const RealDesc *descs, const Coef *coefs, int r, int cz, Slot *slot, int8_t *wind,
             int tile0) {
    const RealDesc d = descs[r];
    const Coef c = coefs[r];
    if (MODE != MODE_MEASURE && !c.active)
        return;
    tiled_tile<T, TY, MODE>(d, c, tile0 + xcd_remap(blockIdx.x, gridDim.x), cz, slot, wind);
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
                                MODE == MODE_STEP ? nullptr : slots + item.r, nullptr);
    }
}

} // namespace ah
