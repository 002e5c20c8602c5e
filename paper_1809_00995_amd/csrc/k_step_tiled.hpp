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

// wrap count of a link: [u]_pi = u - 2 pi m (Eq. (11)), computed in FP64
__device__ __forceinline__ int wrap_count(double u) {
    return (int)floor((u + kPi) / kTwoPi);
}

template <typename T> struct SiteV {
    T pr, pm, ax, ay, az, uxc, uxs, uyc, uys, uzc, uzs;
    double th;
};

__device__ __forceinline__ int wrap_mod(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
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
    __shared__ double lth[2][SM];      // arg phi (measuring modes)
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

    const int par = c.parity;
    const T *phr = plane<T>(d, field_plane(0, par));
    const T *phi = plane<T>(d, field_plane(1, par));
    const T *A0 = plane<T>(d, field_plane(4, par));
    const T *A1 = plane<T>(d, field_plane(5, par));
    const T *A2 = plane<T>(d, field_plane(6, par));
    T *pir = plane<T>(d, P_PIR), *pii = plane<T>(d, P_PII);
    T *E0 = plane<T>(d, P_EX), *E1 = plane<T>(d, P_EX + 1), *E2 = plane<T>(d, P_EX + 2);
    T *ophr = plane<T>(d, field_plane(0, par ^ 1));
    T *ophi = plane<T>(d, field_plane(1, par ^ 1));
    T *oA0 = plane<T>(d, field_plane(4, par ^ 1));
    T *oA1 = plane<T>(d, field_plane(5, par ^ 1));
    T *oA2 = plane<T>(d, field_plane(6, par ^ 1));

    const T c1 = (T)c.c1, c2 = (T)c.c2, c3 = (T)c.c3;
    const T d1 = (T)c.d1, d2 = (T)c.d2, d3 = (T)c.d3;
    const T dt = (T)d.dt, s2 = (T)(d.sigma * d.sigma);

    // measurement constants and per-thread FP64 accumulators
    double msum[A_COUNT];
    int mcnt[C_COUNT];       // per thread at most 3 per plane of one column: 32 bits suffice
    double ma2 = 0.0, mg = 0.0, mh = 0.0, idx2 = 0.0;
    if (MEAS) {
        for (int k = 0; k < A_COUNT; ++k)
            msum[k] = 0.0;
        for (int k = 0; k < C_COUNT; ++k)
            mcnt[k] = 0;
        ma2 = c.a_0 * c.a_0;
        mg = pow(c.a_0, 2.0 * (1.0 - c.s_0)) / (2.0 * d.e0 * d.e0);
        mh = d.lambda0 * pow(c.a_0, 2.0 + 2.0 * c.s_0);
        idx2 = 1.0 / (d.dx * d.dx);
    }

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
            v.th = atan2((double)v.pm, (double)v.pr);
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

    // prologue: planes z0-1 (buffer 1) and z0 (buffer 0)
    const int zm0 = z0 == 0 ? nz - 1 : z0 - 1;
    SiteV<T> prv, cur, nxt;
    load_site(own(zm0), prv);
    put(1, q, prv);
    stage_halo(1, zm0);
    load_site(own(z0), cur);
    put(0, q, cur);
    stage_halo(0, z0);
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
        const int zp = z + 1 == nz ? 0 : z + 1;
        const int s = own(z);
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
            // Eq. (4): sum_j [U_j(x) phi(x+j) + conj(U_j(x-j)) phi(x-j)] - 6 phi
            T lr = (T)-6 * pr, lim = (T)-6 * pm;
            lr += cur.uxc * pr_xp - cur.uxs * pi_xp + uxc_xm * pr_xm + uxs_xm * pi_xm;
            lim += cur.uxc * pi_xp + cur.uxs * pr_xp + uxc_xm * pi_xm - uxs_xm * pr_xm;
            lr += cur.uyc * pr_yp - cur.uys * pi_yp + uyc_ym * pr_ym + uys_ym * pi_ym;
            lim += cur.uyc * pi_yp + cur.uys * pr_yp + uyc_ym * pi_ym - uys_ym * pr_ym;
            lr += cur.uzc * nxt.pr - cur.uzs * nxt.pm + uzc_m * phr_m + uzs_m * phi_m;
            lim += cur.uzc * nxt.pm + cur.uzs * nxt.pr + uzc_m * phi_m - uzs_m * phr_m;
            const T v = pr * pr + pm * pm - s2;
            const T pnr = c1 * pr0 + c2 * lr - c3 * v * pr;
            const T pni = c1 * pi0 + c2 * lim - c3 * v * pm;

            // Eq. (5): current Im[conj(phi(x+i)) conj(U_i) phi(x)] and the curl
            const T wxr = cur.uxc * pr + cur.uxs * pm, wxi = cur.uxc * pm - cur.uxs * pr;
            const T wyr = cur.uyc * pr + cur.uys * pm, wyi = cur.uyc * pm - cur.uys * pr;
            const T wzr = cur.uzc * pr + cur.uzs * pm, wzi = cur.uzc * pm - cur.uzs * pr;
            const T jx = pr_xp * wxi - pi_xp * wxr;
            const T jy = pr_yp * wyi - pi_yp * wyr;
            const T jz = nxt.pr * wzi - nxt.pm * wzr;
            const T curl_x = (pxy - pxy_ym) - (pzx - pzx_m);
            const T curl_y = (pyz - pyz_m) - (pxy - pxy_xm);
            const T curl_z = (pzx - pzx_xm) - (pyz - pyz_ym);
            const T enx = d1 * ex0 + d3 * jx - d2 * curl_x;
            const T eny = d1 * ey0 + d3 * jy - d2 * curl_y;
            const T enz = d1 * ez0 + d3 * jz - d2 * curl_z;

            if (owner) {
                // streaming stores: the new state is not read again in this launch
                __builtin_nontemporal_store(pnr, pir + s);
                __builtin_nontemporal_store(pni, pii + s);
                __builtin_nontemporal_store(enx, E0 + s);
                __builtin_nontemporal_store(eny, E1 + s);
                __builtin_nontemporal_store(enz, E2 + s);
                __builtin_nontemporal_store((T)(pr + dt * pnr), ophr + s);        // Eq. (6)
                __builtin_nontemporal_store((T)(pm + dt * pni), ophi + s);
                __builtin_nontemporal_store((T)(cur.ax + dt * enx), oA0 + s);    // Eq. (7)
                __builtin_nontemporal_store((T)(cur.ay + dt * eny), oA1 + s);
                __builtin_nontemporal_store((T)(cur.az + dt * enz), oA2 + s);
            }
        }

        if (MEAS && owner) {
            // Eqs. (9)-(12) for the site of S_n read above
            const bool finite = isfinite((double)pr) && isfinite((double)pm) &&
                                isfinite((double)pr0) && isfinite((double)pi0) &&
                                isfinite((double)cur.ax) && isfinite((double)cur.ay) &&
                                isfinite((double)cur.az) && isfinite((double)ex0) &&
                                isfinite((double)ey0) && isfinite((double)ez0);
            int w3[3] = { 0, 0, 0 };
            if (!finite) {
                mcnt[C_NONFIN] += 1;
            } else {
                const T gxr = cur.uxc * pr_xp - cur.uxs * pi_xp - pr;
                const T gxi = cur.uxc * pi_xp + cur.uxs * pr_xp - pm;
                const T gyr = cur.uyc * pr_yp - cur.uys * pi_yp - pr;
                const T gyi = cur.uyc * pi_yp + cur.uys * pr_yp - pm;
                const T gzr = cur.uzc * nxt.pr - cur.uzs * nxt.pm - pr;
                const T gzi = cur.uzc * nxt.pm + cur.uzs * nxt.pr - pm;
                const double K = (double)pr0 * pr0 + (double)pi0 * pi0;
                const double Gr = idx2 * ((double)gxr * gxr + (double)gxi * gxi + (double)gyr * gyr +
                                          (double)gyi * gyi + (double)gzr * gzr + (double)gzi * gzi);
                const double EE = idx2 * ((double)ex0 * ex0 + (double)ey0 * ey0 + (double)ez0 * ez0);
                const T oxy = plaq_omc(cur.uxc, cur.uxs, uyc_xp, uys_xp, uxc_yp, uxs_yp, cur.uyc, cur.uys);
                const T oyz = plaq_omc(cur.uyc, cur.uys, uzc_yp, uzs_yp, nxt.uyc, nxt.uys, cur.uzc, cur.uzs);
                const T ozx = plaq_omc(cur.uzc, cur.uzs, nxt.uxc, nxt.uxs, uzc_xp, uzs_xp, cur.uxc, cur.uxs);
                const double BB = 2.0 * idx2 * idx2 * ((double)oxy + (double)oyz + (double)ozx);
                const double vv = (double)pr * pr + (double)pm * pm - (double)s2;
                const double V = 0.25 * vv * vv;
                const double lag = ma2 * K - ma2 * Gr + mg * (EE - BB) - mh * V;
                const double rho = ma2 * K + ma2 * Gr + mg * (EE + BB) + mh * V;
                const double pres = ma2 * K - ma2 * Gr / 3.0 + mg * (EE + BB) / 3.0 - mh * V;
                msum[A_KIN] += ma2 * K;
                msum[A_GRAD] += ma2 * Gr;
                msum[A_ELEC] += mg * EE;
                msum[A_MAG] += mg * BB;
                msum[A_POT] += mh * V;
                msum[A_LAG] += lag;
                msum[A_NUM_L] += K * lag;
                msum[A_NUM_V] += K * V;
                msum[A_NUM_R] += K * rho;
                msum[A_DEN_L] += Gr * lag;
                msum[A_DEN_V] += Gr * V;
                msum[A_DEN_R] += Gr * rho;
                msum[A_PRES] += pres;
                msum[A_PRES_L] += pres * lag;
                msum[A_RHO_L] += rho * lag;

                // winding (Eq. (11)) from link wrap counts
                const double t0 = cur.th, t_xp = lth[cb][q + 1], t_yp = lth[cb][q + G::W];
                const double t_xpyp = lth[cb][q + 1 + G::W];
                const double t_zp = nxt.th, t_xpzp = lth[nb_][q + 1], t_ypzp = lth[nb_][q + G::W];
                const double ax = cur.ax, ay = cur.ay, az = cur.az;
                const double ay_xp = lar[cb][1][q + 1], az_xp = lar[cb][2][q + 1];
                const double ax_yp = lar[cb][0][q + G::W], az_yp = lar[cb][2][q + G::W];
                const double ax_zp = nxt.ax, ay_zp = nxt.ay;
                const int mx = wrap_count(t_xp - t0 + ax);
                const int my = wrap_count(t_yp - t0 + ay);
                const int mz = wrap_count(t_zp - t0 + az);
                const int my_xp = wrap_count(t_xpyp - t_xp + ay_xp);
                const int mx_yp = wrap_count(t_xpyp - t_yp + ax_yp);
                const int mz_yp = wrap_count(t_ypzp - t_yp + az_yp);
                const int my_zp = wrap_count(t_ypzp - t_zp + ay_zp);
                const int mx_zp = wrap_count(t_xpzp - t_zp + ax_zp);
                const int mz_xp = wrap_count(t_xpzp - t_xp + az_xp);
                w3[0] = -(mx + my_xp - mx_yp - my);
                w3[1] = -(my + mz_yp - my_zp - mz);
                w3[2] = -(mz + mx_zp - mz_xp - mx);
                for (int k = 0; k < 3; ++k) {
                    mcnt[C_W0 + k] += w3[k];
                    mcnt[C_N0 + k] += w3[k] < 0 ? -w3[k] : w3[k];
                    mcnt[C_PIERCED] += w3[k] != 0 ? 1 : 0;
                }
            }
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

    if (MEAS) {
        if (tile == 0 && threadIdx.x == 0) {
            slot->c = c;
            slot->measured = 1;
        }
        unsigned long long cnt64[C_COUNT];
        for (int k = 0; k < C_COUNT; ++k)
            cnt64[k] = (unsigned long long)(long long)mcnt[k];   // two's complement for W sums
        block_accumulate<A_COUNT, C_COUNT, TY>(msum, cnt64, slot->acc.s, slot->acc.c);
        __syncthreads();   // the reduction's LDS is reused by the next tile of a batch
    }
}

// One realization: one block per tile, tiles [tile0, tile0 + gridDim.x).
template <typename T, int TY, int MODE>
__global__ void __launch_bounds__(64 * TY)
k_step_tiled(const RealDesc *descs, const Coef *coefs, int r, int cz, Slot *slot, int8_t *wind,
             int tile0) {
    const RealDesc d = descs[r];
    const Coef c = coefs[r];
    if (MODE != MODE_MEASURE && !c.active)
        return;
    tiled_tile<T, TY, MODE>(d, c, tile0 + xcd_remap(blockIdx.x, gridDim.x), cz, slot, wind);
}

// A work item of the batched kernel: tile `tile` of realization r, with that
// realization's z-chunk cz.
struct BatchItem {
    int32_t r, tile, cz, pad;
};

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

// Tile height and z-chunk used when the caller leaves them at 0.
inline void tiled_defaults(bool fp64, int nx, int ny, int nz, int &ty, int &cz) {
    if (ty <= 0)
        ty = fp64 ? 4 : 8;
    if (cz <= 0) {
        const long tiles_xy = (long)(nx / 64) * ((ny + ty - 1) / ty);
        long chunks = (4096 + tiles_xy - 1) / tiles_xy;       // aim at ~4096 blocks
        const long max_chunks = (nz + 7) / 8;                  // but at least ~8 planes each
        if (chunks > max_chunks)
            chunks = max_chunks;
        if (chunks < 1)
            chunks = 1;
        cz = (int)((nz + chunks - 1) / chunks);
    }
}

template <typename T, int TY, int MODE>
hipError_t launch_tiled_ty(const RealDesc *desc, const Coef *coef, int r, int nx, int ny, int nz,
                           int cz, Slot *slot, int8_t *wind, hipStream_t stream) {
    const long blocks = (long)(nx / 64) * ((ny + TY - 1) / TY) * ((nz + cz - 1) / cz);
    hipLaunchKernelGGL((k_step_tiled<T, TY, MODE>), dim3((unsigned)blocks), dim3(64 * TY), 0,
                       stream, desc, coef, r, cz, slot, wind, 0);
    return hipGetLastError();
}

template <typename T, int MODE>
hipError_t launch_tiled_mode(int ty, const RealDesc *desc, const Coef *coef, int r, int nx, int ny,
                             int nz, int cz, Slot *slot, int8_t *wind, hipStream_t stream) {
    // The measuring modes hold ~220 VGPRs: keep them at tiles that do not
    // spill (FP32 <= 8 rows, FP64 <= 4).  The update is the same arithmetic
    // for every tile height, so this only changes the order of the sums.
    constexpr bool MEAS = MODE != MODE_STEP;
    constexpr int TYMAX = MEAS ? (sizeof(T) == 4 ? 8 : 4) : (sizeof(T) == 4 ? 16 : 8);
    if (ty > TYMAX)
        ty = TYMAX;
    switch (ty) {
    case 2: return launch_tiled_ty<T, 2, MODE>(desc, coef, r, nx, ny, nz, cz, slot, wind, stream);
    case 4: return launch_tiled_ty<T, 4, MODE>(desc, coef, r, nx, ny, nz, cz, slot, wind, stream);
    default:
        if constexpr (TYMAX >= 16)
            if (ty == 16)
                return launch_tiled_ty<T, 16, MODE>(desc, coef, r, nx, ny, nz, cz, slot, wind, stream);
        if constexpr (TYMAX >= 8)
            return launch_tiled_ty<T, 8, MODE>(desc, coef, r, nx, ny, nz, cz, slot, wind, stream);
        return hipErrorInvalidValue;
    }
}

// Valid tile heights: FP32 2, 4, 8, 16; FP64 2, 4, 8.
inline bool tiled_ty_valid(bool fp64, int ty) {
    return ty == 2 || ty == 4 || ty == 8 || (!fp64 && ty == 16);
}

// Launch one tiled kernel (mode MODE_*) for realization r.
inline int launch_step_tiled(bool fp64, int mode, const RealDesc *desc, const Coef *coef, int r,
                             int nx, int ny, int nz, int tile_y, int chunk_z, Slot *slot,
                             int8_t *wind, hipStream_t stream) {
    int ty = tile_y, cz = chunk_z;
    tiled_defaults(fp64, nx, ny, nz, ty, cz);
    if (nx % 64 != 0 || !tiled_ty_valid(fp64, ty) || cz < 1)
        return (int)hipErrorInvalidValue;
    hipError_t e;
    if (fp64) {
        e = mode == MODE_STEP ? launch_tiled_mode<double, MODE_STEP>(ty, desc, coef, r, nx, ny, nz, cz, slot, wind, stream)
          : mode == MODE_STEP_MEASURE ? launch_tiled_mode<double, MODE_STEP_MEASURE>(ty, desc, coef, r, nx, ny, nz, cz, slot, wind, stream)
          : launch_tiled_mode<double, MODE_MEASURE>(ty, desc, coef, r, nx, ny, nz, cz, slot, wind, stream);
    } else {
        e = mode == MODE_STEP ? launch_tiled_mode<float, MODE_STEP>(ty, desc, coef, r, nx, ny, nz, cz, slot, wind, stream)
          : mode == MODE_STEP_MEASURE ? launch_tiled_mode<float, MODE_STEP_MEASURE>(ty, desc, coef, r, nx, ny, nz, cz, slot, wind, stream)
          : launch_tiled_mode<float, MODE_MEASURE>(ty, desc, coef, r, nx, ny, nz, cz, slot, wind, stream);
    }
    return (int)e;
}

// Largest tile height of a mode (the measuring modes hold ~220 VGPRs).
inline int tiled_ty_max(bool fp64, int mode) {
    return mode != MODE_STEP ? (fp64 ? 4 : 8) : (fp64 ? 8 : 16);
}

template <typename T, int TY, int MODE>
hipError_t batch_grid_ty(int *grid) {
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step_batch<T, TY, MODE>, 64 * TY, 0);
    *grid = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
    return e;
}

template <typename T, int TY, int MODE>
hipError_t launch_batch_ty(const RealDesc *desc, const Coef *coef, const BatchItem *items,
                           int n_items, Slot *slots, int grid, hipStream_t stream) {
    if (grid > n_items)
        grid = n_items;
    if (grid < 1)
        return hipSuccess;
    hipLaunchKernelGGL((k_step_batch<T, TY, MODE>), dim3((unsigned)grid), dim3(64 * TY), 0, stream,
                       desc, coef, items, n_items, slots);
    return hipGetLastError();
}

// Dispatch over (precision, tile height, mode) of the batched kernel.  With
// grid_out != NULL only the resident-block count of that kernel is returned
// (occupancy x compute units); otherwise the kernel is launched on `grid`
// blocks.  Tile heights: FP32 2, 4, 8 (16 for MODE_STEP); FP64 2, 4 (8 for
// MODE_STEP).
inline int batch_dispatch(bool fp64, int mode, int ty, const RealDesc *desc, const Coef *coef,
                          const BatchItem *items, int n_items, Slot *slots, int grid,
                          hipStream_t stream, int *grid_out) {
    if (ty > tiled_ty_max(fp64, mode) || !tiled_ty_valid(fp64, ty))
        return (int)hipErrorInvalidValue;
#define AH_BATCH(T, TY_, M)                                                                        \
    (grid_out ? batch_grid_ty<T, TY_, M>(grid_out)                                                 \
              : launch_batch_ty<T, TY_, M>(desc, coef, items, n_items, slots, grid, stream))
    hipError_t e = hipErrorInvalidValue;
    if (fp64) {
        if (mode == MODE_STEP)
            e = ty == 2 ? AH_BATCH(double, 2, MODE_STEP) : ty == 4 ? AH_BATCH(double, 4, MODE_STEP)
                                                                   : AH_BATCH(double, 8, MODE_STEP);
        else
            e = ty == 2 ? AH_BATCH(double, 2, MODE_STEP_MEASURE) : AH_BATCH(double, 4, MODE_STEP_MEASURE);
    } else {
        if (mode == MODE_STEP)
            e = ty == 2 ? AH_BATCH(float, 2, MODE_STEP) : ty == 4 ? AH_BATCH(float, 4, MODE_STEP)
              : ty == 8 ? AH_BATCH(float, 8, MODE_STEP) : AH_BATCH(float, 16, MODE_STEP);
        else
            e = ty == 2 ? AH_BATCH(float, 2, MODE_STEP_MEASURE)
              : ty == 4 ? AH_BATCH(float, 4, MODE_STEP_MEASURE) : AH_BATCH(float, 8, MODE_STEP_MEASURE);
    }
#undef AH_BATCH
    return (int)e;
}

} // namespace ah
