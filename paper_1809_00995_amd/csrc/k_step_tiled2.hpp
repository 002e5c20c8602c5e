// k_step_tiled2.hpp -- two leapfrog steps per pass over memory (temporal
// blocking) in the 20-plane layout.
//
// A single-step pass reads and writes the whole state once per step, and at
// 512^3 that runs at the speed of a device copy.  Here each block advances
// its 64 x TY tile from S_n to S_{n+2} while reading S_n and writing S_{n+2}
// once: the intermediate state S_{n+1} lives in LDS only.
//
// Geometry, per z-plane (R1 = tile + one-site ring, R2 = R1 + one more ring):
//  - S_n (phi and the link phasors) is staged in LDS on R2: the tile's own
//    sites and the R1 ring come from the threads that update them (in
//    registers), the outer ring from the ring wavefronts.
//  - Step one (Eqs. (4)-(7) with the coefficients of step n) is computed on
//    all of R1: TY wavefronts hold the tile's rows (64 sites each, as in the
//    single-step kernel) and NRW ring wavefronts hold the R1 ring.  S_{n+1}'s
//    phi and phasors go to LDS.
//  - Step two (coefficients of step n+1) is computed on the tile, one plane
//    behind step one, and S_{n+2} is written to the other copy.
// The ring costs (66 (TY+2)) / (64 TY) extra site updates of step one.  The
// momenta Pi, E of S_n are read by neighbouring blocks (their R1 ring) while
// this block writes S_{n+2}: that is why every field has two copies.
//
// Per plane there are two barriers, both ordering LDS only: the global reads
// of the next plane are issued one iteration ahead and stay in flight across
// them.  Each site publishes its three forward plaquette sines in LDS (step
// one's while staging, step two's after its S_{n+1} update), and the four it
// needs from x-x and x-y are read there instead of recomputed.
//
// Both steps use leapfrog_site and plaq_sin, so S_{n+2} is bitwise what two
// single-step tiled passes give.  When the second step of the pair is not
// active (the realization reaches n_end after one step), the kernel writes
// S_{n+1} instead.
#pragma once

#include <type_traits>

#include "k_step_tiled.hpp"
#include "k_step_tiled2_api.hpp"

namespace ah {

// R1 and R2 are W x H sites; their LDS rows are P = W + PAD elements apart.
template <int TY, int PAD = 0> struct Tile2Geom {
    static constexpr int W1 = 66, H1 = TY + 2, P1 = W1 + PAD, S1 = P1 * H1;   // R1
    static constexpr int W2 = 68, H2 = TY + 4, P2 = W2 + PAD, S2 = P2 * H2;   // R2
    static constexpr int RING1 = 2 * W1 + 2 * TY;              // R1 minus the tile
    static constexpr int RING2 = 2 * W2 + 2 * H1;              // R2 minus R1
    static constexpr int NRW = (RING1 + 63) / 64;              // ring wavefronts
    static constexpr int NW = TY + NRW;                        // wavefronts per block
    static_assert(RING2 <= 64 * NRW, "the ring wavefronts stage the outer ring");
    static_assert(NW <= 16, "at most 1024 threads per block");
    static __device__ __forceinline__ int i1(int lx, int ly) { return (ly + 1) * P1 + (lx + 1); }
    static __device__ __forceinline__ int i2(int lx, int ly) { return (ly + 2) * P2 + (lx + 2); }
    // h-th site of the R1 ring: rows -1 and TY (x = -1..64), then columns -1 and 64 (y = 0..TY-1)
    static __device__ __forceinline__ void ring1(int h, int &lx, int &ly) {
        if (h < W1) {
            lx = h - 1;
            ly = -1;
        } else if (h < 2 * W1) {
            lx = h - W1 - 1;
            ly = TY;
        } else if (h < 2 * W1 + TY) {
            lx = -1;
            ly = h - 2 * W1;
        } else {
            lx = 64;
            ly = h - 2 * W1 - TY;
        }
    }
    // h-th site of the R2 ring: rows -2 and TY+1 (x = -2..65), then columns -2 and 65 (y = -1..TY)
    static __device__ __forceinline__ void ring2(int h, int &lx, int &ly) {
        if (h < W2) {
            lx = h - 2;
            ly = -2;
        } else if (h < 2 * W2) {
            lx = h - W2 - 2;
            ly = TY + 1;
        } else if (h < 2 * W2 + H1) {
            lx = -2;
            ly = h - 2 * W2 - 1;
        } else {
            lx = 65;
            ly = h - 2 * W2 - H1 - 1;
        }
    }
};

// LDS row padding of the two-step kernel by element type.  FP32 rows take one
// element more: with odd pitches the ring wavefronts' column accesses (lanes one
// row apart) fall in distinct banks.  FP64 has no LDS to spare (159.4 KiB of the
// 160 KiB at TY = 5).
template <typename T> inline constexpr int kTile2Pad = 0;
template <> inline constexpr int kTile2Pad<float> = 1;

// phi and the three link phasors of one site (the LDS record of a state).
template <typename T> struct Phasors {
    T pr, pm, uxc, uxs, uyc, uys, uzc, uzs;
};

// A site's own values carried from plane z-1 to plane z: phi, U_z, and the yz
// and zx plaquettes based at the site.
template <typename T> struct Below {
    T pr, pm, uzc, uzs, pyz, pzx;
};

// The three forward plaquette sines based at site s (Eq. (3)): xy, yz, zx at
// s, from its phasors on plane z (own) and z+1 (up) and those of s+x, s+y on
// plane z (buffer C, row width W).  The argument order is the single-step
// kernel's, so the values are bitwise the same whichever thread forms them.
template <typename T> struct Plaq3 {
    T xy, yz, zx;
};

template <typename T, int W, int S>
__device__ __forceinline__ Plaq3<T> fwd_plaquettes(const T (*C)[S], int q, const Phasors<T> &own,
                                                   const Phasors<T> &up) {
    Plaq3<T> p;
    p.xy = plaq_sin(own.uxc, own.uxs, C[Q_UYC][q + 1], C[Q_UYS][q + 1], C[Q_UXC][q + W],
                    C[Q_UXS][q + W], own.uyc, own.uys);
    p.yz = plaq_sin(own.uyc, own.uys, C[Q_UZC][q + W], C[Q_UZS][q + W], up.uyc, up.uys, own.uzc,
                    own.uzs);
    p.zx = plaq_sin(own.uzc, own.uzs, up.uxc, up.uxs, C[Q_UZC][q + 1], C[Q_UZS][q + 1], own.uxc,
                    own.uxs);
    return p;
}

template <typename T, int S>
__device__ __forceinline__ Phasors<T> get_phasors(const T (*C)[S], int k) {
    Phasors<T> v;
    v.pr = C[Q_PR][k];
    v.pm = C[Q_PI][k];
    v.uxc = C[Q_UXC][k];
    v.uxs = C[Q_UXS][k];
    v.uyc = C[Q_UYC][k];
    v.uys = C[Q_UYS][k];
    v.uzc = C[Q_UZC][k];
    v.uzs = C[Q_UZS][k];
    return v;
}

// Gather the stencil of the site at LDS index q of a state staged with row
// width W on plane z (buffer C).  own/up are the site's values at z and z+1
// (registers), bel its carried values from z-1, pi_e its momenta at z, fp its
// forward plaquettes, and P the forward plaquettes of every site of plane z
// (those of x-x and x-y are read).
template <typename T, int W, int S>
__device__ __forceinline__ Stencil<T> gather(const T (*C)[S], const T (*P)[S], int q,
                                             const Phasors<T> &own, T ax, T ay, T az,
                                             const Phasors<T> &up, const Below<T> &bel,
                                             T pr0, T pi0, T ex0, T ey0, T ez0,
                                             const Plaq3<T> &fp) {
    Stencil<T> st;
    st.pr = own.pr; st.pm = own.pm; st.ax = ax; st.ay = ay; st.az = az;
    st.uxc = own.uxc; st.uxs = own.uxs; st.uyc = own.uyc; st.uys = own.uys;
    st.uzc = own.uzc; st.uzs = own.uzs;
    st.pr0 = pr0; st.pi0 = pi0; st.ex0 = ex0; st.ey0 = ey0; st.ez0 = ez0;
    st.pr_xp = C[Q_PR][q + 1]; st.pi_xp = C[Q_PI][q + 1];
    st.pr_xm = C[Q_PR][q - 1]; st.pi_xm = C[Q_PI][q - 1];
    st.pr_yp = C[Q_PR][q + W]; st.pi_yp = C[Q_PI][q + W];
    st.pr_ym = C[Q_PR][q - W]; st.pi_ym = C[Q_PI][q - W];
    st.pr_zp = up.pr; st.pi_zp = up.pm; st.pr_zm = bel.pr; st.pi_zm = bel.pm;
    st.uxc_xm = C[Q_UXC][q - 1]; st.uxs_xm = C[Q_UXS][q - 1];
    st.uyc_ym = C[Q_UYC][q - W]; st.uys_ym = C[Q_UYS][q - W];
    st.uzc_zm = bel.uzc; st.uzs_zm = bel.uzs;
    st.pxy = fp.xy;
    st.pyz = fp.yz;
    st.pzx = fp.zx;
    st.pxy_xm = P[0][q - 1];
    st.pzx_xm = P[2][q - 1];
    st.pxy_ym = P[0][q - W];
    st.pyz_ym = P[1][q - W];
    st.pyz_zm = bel.pyz;
    st.pzx_zm = bel.pzx;
    return st;
}

// The yz and zx plaquettes based at the site of LDS index q on plane z
// (buffer C), with own/up its values at z and z+1: the carried values of the
// first plane of a chunk.
template <typename T, int W, int S>
__device__ __forceinline__ void base_plaquettes(const T (*C)[S], int q, const Phasors<T> &own,
                                                const Phasors<T> &up, T &pyz, T &pzx) {
    pyz = plaq_sin(own.uyc, own.uys, C[Q_UZC][q + W], C[Q_UZS][q + W], up.uyc, up.uys, own.uzc,
                   own.uzs);
    pzx = plaq_sin(own.uzc, own.uzs, up.uxc, up.uxs, C[Q_UZC][q + 1], C[Q_UZS][q + 1], own.uxc,
                   own.uxs);
}

template <typename T, int S>
__device__ __forceinline__ void put_phasors(T (*B)[S], int k, const Phasors<T> &v) {
    B[Q_PR][k] = v.pr;
    B[Q_PI][k] = v.pm;
    B[Q_UXC][k] = v.uxc;
    B[Q_UXS][k] = v.uxs;
    B[Q_UYC][k] = v.uyc;
    B[Q_UYS][k] = v.uys;
    B[Q_UZC][k] = v.uzc;
    B[Q_UZS][k] = v.uzs;
}

template <typename T>
__device__ __forceinline__ Phasors<T> make_phasors(T pr, T pm, T ax, T ay, T az) {
    Phasors<T> v;
    v.pr = pr;
    v.pm = pm;
    sincos_t(ax, &v.uxs, &v.uxc);
    sincos_t(ay, &v.uys, &v.uyc);
    sincos_t(az, &v.uzs, &v.uzc);
    return v;
}

// One tile (64 x TY sites, planes [z0, z0 + cz)) of one realization: S_n in
// copy c0.parity -> S_{n+2} (or S_{n+1} when c1 is not active) in the other
// copy.  OFF32: every plane is below 4 GiB, so element addresses are one
// 32-bit byte offset shared by all planes from each plane's base (scalar
// registers); otherwise 64-bit addresses.  Every thread of the block calls it
// with the same arguments.
template <typename T, int TY, bool OFF32>
__device__ __forceinline__ void tiled2_tile(const RealDesc &d, const Coef &c0, const Coef &c1,
                                            int tile, int cz) {
    using G = Tile2Geom<TY, kTile2Pad<T>>;
    __shared__ T sa[2][Q_COUNT][G::S2];   // S_n on R2, planes z and z+1
    __shared__ T sb[2][Q_COUNT][G::S1];   // S_{n+1} on R1, two planes
    __shared__ T pa[3][G::S2];            // forward plaquettes of S_n, plane of step one
    __shared__ T pb[3][G::S1];            // forward plaquettes of S_{n+1}, plane of step two

    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const int ntx = nx >> 6, nty = (ny + TY - 1) / TY;
    const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
    const int x0 = tx << 6, y0 = ty * TY, z0 = tz * cz;
    const int z1 = min(z0 + cz, nz);
    const bool two = c1.active != 0;

    const int t = threadIdx.x;
    const bool inner = t < 64 * TY;            // wave-uniform
    int lx, ly;
    bool has1 = true;
    if (inner) {
        lx = t & 63;
        ly = t >> 6;
    } else {
        const int h = t - 64 * TY;
        has1 = h < G::RING1;
        G::ring1(has1 ? h : 0, lx, ly);
    }
    const bool owner = inner && (y0 + ly) < ny;
    const int gx = wrap_mod(x0 + lx, nx), gy = wrap_mod(y0 + ly, ny);
    const int q2 = G::i2(lx, ly), q1 = G::i1(lx, ly);
    // outer-ring staging by the ring wavefronts
    int h2 = inner ? G::RING2 : t - 64 * TY;
    int rx = 0, ry = 0;
    const bool stager = h2 < G::RING2;
    if (stager)
        G::ring2(h2, rx, ry);
    const int rq = G::i2(rx, ry);
    const int rgx = wrap_mod(x0 + rx, nx), rgy = wrap_mod(y0 + ry, ny);
    // forward plaquettes that step one reads at x-x and x-y of the R1 ring
    const bool edge2 = stager && ((rx == -2 && ry >= -1 && ry <= TY) || (ry == -2 && rx >= -1 && rx <= 64));
    // forward plaquettes of S_{n+1} that step two needs: the tile and the
    // ring's column x = -1 and row y = -1 next to it
    const bool need1 = inner || (lx == -1 && ly >= 0 && ly < TY) || (ly == -1 && lx >= 0 && lx < 64);

    const int par = c0.parity, L = d.layout;
    gptr<const T> in[10];
    gptr<T> out[10];
    for (int f = 0; f < 10; ++f) {
        in[f] = gplane<const T>(d, field_plane(f, par, L));
        out[f] = gplane<T>(d, field_plane(f, par ^ 1, L));
    }
    const StepK<T> K0 = step_k<T>(d, c0), K1 = step_k<T>(d, c1);

    auto own_site = [&](int z) { return gx + nx * (gy + ny * z); };
    // z below is slab-relative; zmap gives the stored plane (periodic wrap,
    // or the offset past the halo planes of a slab)
    auto zwrap = [&](int z) { return zmap(d, z); };
    // element s of field f of S_n, and the store of the new state
    auto LD = [&](int f, int s) -> T {
        if constexpr (OFF32)
            return *(gptr<const T>)((gptr<const char>)in[f] + (uint32_t)s * (uint32_t)sizeof(T));
        else
            return in[f][s];
    };
    auto ST = [&](int f, int s, T v) {
        if constexpr (OFF32)
            __builtin_nontemporal_store(
                v, (gptr<T>)((gptr<char>)out[f] + (uint32_t)s * (uint32_t)sizeof(T)));
        else
            __builtin_nontemporal_store(v, out[f] + s);
    };
    // S_n at (own site, z): phi, A and phasors
    struct Raw {
        T pr, pm, ax, ay, az;
    };
    auto load_raw = [&](int s) {
        Raw r;
        r.pr = LD(0, s);
        r.pm = LD(1, s);
        r.ax = LD(4, s);
        r.ay = LD(5, s);
        r.az = LD(6, s);
        return r;
    };
    auto stage_ring = [&](int bf, int z) {
        if (stager) {
            const Raw r = load_raw(rgx + nx * (rgy + ny * z));
            put_phasors<T, G::S2>(sa[bf], rq, make_phasors(r.pr, r.pm, r.ax, r.ay, r.az));
        }
    };

    // ---- prologue: S_n planes z0-2 (buffer 1) and z0-1 (buffer 0)
    const int za = zwrap(z0 - 2), zb = zwrap(z0 - 1);
    Raw rcur;
    Phasors<T> pcur;
    Below<T> bel;
    {
        const Raw rb = load_raw(own_site(za));
        const Phasors<T> pbel = make_phasors(rb.pr, rb.pm, rb.ax, rb.ay, rb.az);
        if (has1)
            put_phasors<T, G::S2>(sa[1], q2, pbel);
        stage_ring(1, za);
        rcur = load_raw(own_site(zb));
        pcur = make_phasors(rcur.pr, rcur.pm, rcur.ax, rcur.ay, rcur.az);
        if (has1)
            put_phasors<T, G::S2>(sa[0], q2, pcur);
        stage_ring(0, zb);
        lds_barrier();
        bel.pyz = bel.pzx = 0;
        if (has1)
            base_plaquettes<T, G::P2, G::S2>(sa[1], q2, pbel, pcur, bel.pyz, bel.pzx);
        bel.pr = pbel.pr;
        bel.pm = pbel.pm;
        bel.uzc = pbel.uzc;
        bel.uzs = pbel.uzs;
        lds_barrier();
    }

    // The global reads of iteration k (S_n at plane zs+1 on the own site and
    // the outer ring, the momenta of S_n at zs) are issued one iteration
    // ahead, so their latency hides behind the previous plane's two steps.
    Raw f_own{}, f_ring{};
    T f_pr0 = 0, f_pi0 = 0, f_ex0 = 0, f_ey0 = 0, f_ez0 = 0;
    auto prefetch = [&](int k) {
        const int zs = zwrap(z0 - 1 + k), zn = zwrap(z0 + k);
        if (has1) {
            const int s = own_site(zs);
            f_pr0 = LD(2, s);
            f_pi0 = LD(3, s);
            f_ex0 = LD(7, s);
            f_ey0 = LD(8, s);
            f_ez0 = LD(9, s);
            f_own = load_raw(own_site(zn));
        }
        if (stager)
            f_ring = load_raw(rgx + nx * (rgy + ny * zn));
    };
    auto store_state = [&](const SiteNew<T> &v, int s) {
        ST(2, s, v.pr);
        ST(3, s, v.pi);
        ST(7, s, v.ex);
        ST(8, s, v.ey);
        ST(9, s, v.ez);
        ST(0, s, v.qr);
        ST(1, s, v.qi);
        ST(4, s, v.ax);
        ST(5, s, v.ay);
        ST(6, s, v.az);
    };

    // Own-site values of one plane: S_n (raw fields and phasors) and S_{n+1}
    // (new values and phasors).  The loop is unrolled by two with the sets
    // alternating roles, so the plane-to-plane hand-over needs no copies and
    // the LDS buffer of each half is a constant.
    struct SnSet {
        Raw r;
        Phasors<T> p;
    };
    struct S1Set {
        SiteNew<T> v;
        Phasors<T> p;
    };
    SnSet sA, sB;
    S1Set uA{}, uB{};
    sA.r = rcur;
    sA.p = pcur;
    Below<T> bel1{};

    // Iteration k: step one on plane zs = z0-1+k (S_n in sa[CB], plane zs+1
    // goes to sa[CB^1]), S_{n+1} of plane zs to sb[CB]; step two on plane zs-1
    // (S_{n+1} in sb[CB^1] and sb[CB]).  cur/nxt: own S_n at zs, zs+1; c1/n1:
    // own S_{n+1} at zs-1, zs.
    const int nk = (z1 - z0) + 2;
    auto body = [&](auto cbc, int k, SnSet &cur, SnSet &nxt, S1Set &c1, S1Set &n1) {
        constexpr int CB = decltype(cbc)::value, NB = CB ^ 1;
        const int zi = z0 - 1 + k, zs = zwrap(zi);
        // (a) stage S_n at zs+1 from the prefetched values; start the next reads
        const T pr0 = f_pr0, pi0 = f_pi0, ex0 = f_ex0, ey0 = f_ey0, ez0 = f_ez0;
        // and form the forward plaquettes of plane zs (complete since the last
        // barrier) for the own site and the outer ring's column and row that
        // step one reads
        nxt.r = f_own;
        Plaq3<T> fp{};
        if (has1) {
            nxt.p = make_phasors(nxt.r.pr, nxt.r.pm, nxt.r.ax, nxt.r.ay, nxt.r.az);
            put_phasors<T, G::S2>(sa[NB], q2, nxt.p);
            fp = fwd_plaquettes<T, G::P2, G::S2>(sa[CB], q2, cur.p, nxt.p);
            pa[0][q2] = fp.xy;
            pa[1][q2] = fp.yz;
            pa[2][q2] = fp.zx;
        }
        if (stager) {
            const Phasors<T> up = make_phasors(f_ring.pr, f_ring.pm, f_ring.ax, f_ring.ay, f_ring.az);
            put_phasors<T, G::S2>(sa[NB], rq, up);
            if (edge2) {
                const Plaq3<T> rp =
                    fwd_plaquettes<T, G::P2, G::S2>(sa[CB], rq, get_phasors<T, G::S2>(sa[CB], rq), up);
                pa[0][rq] = rp.xy;
                pa[1][rq] = rp.yz;
                pa[2][rq] = rp.zx;
            }
        }
        if (k + 1 < nk)
            prefetch(k + 1);
        lds_barrier();

        // (b) step one at (own R1 site, zs); then the forward plaquettes of
        // S_{n+1} at zs-1, which need the own site's S_{n+1} at zs just formed
        Plaq3<T> fp1{};
        if (has1) {
            const Stencil<T> st = gather<T, G::P2, G::S2>(sa[CB], pa, q2, cur.p, cur.r.ax,
                                                          cur.r.ay, cur.r.az, nxt.p, bel, pr0,
                                                          pi0, ex0, ey0, ez0, fp);
            n1.v = leapfrog_site(st, K0);
            bel.pr = cur.p.pr;
            bel.pm = cur.p.pm;
            bel.uzc = cur.p.uzc;
            bel.uzs = cur.p.uzs;
            bel.pyz = fp.yz;
            bel.pzx = fp.zx;
            if (two) {
                n1.p = make_phasors(n1.v.qr, n1.v.qi, n1.v.ax, n1.v.ay, n1.v.az);
                put_phasors<T, G::S1>(sb[CB], q1, n1.p);
                if (need1 && k >= 1) {
                    fp1 = fwd_plaquettes<T, G::P1, G::S1>(sb[NB], q1, c1.p, n1.p);
                    pb[0][q1] = fp1.xy;
                    pb[1][q1] = fp1.yz;
                    pb[2][q1] = fp1.zx;
                }
            }
        }
        if (!two) {
            // one step only: the tile's S_{n+1} is final
            if (owner && k >= 1 && k <= z1 - z0)
                store_state(n1.v, own_site(zs));
            lds_barrier();
            return;
        }
        lds_barrier();

        // (c) step two at (tile site, zs - 1), one plane behind
        if (inner) {
            if (k >= 2) {
                const Stencil<T> st = gather<T, G::P1, G::S1>(sb[NB], pb, q1, c1.p, c1.v.ax,
                                                              c1.v.ay, c1.v.az, n1.p, bel1,
                                                              c1.v.pr, c1.v.pi, c1.v.ex,
                                                              c1.v.ey, c1.v.ez, fp1);
                const SiteNew<T> n2 = leapfrog_site(st, K1);
                if (owner)
                    store_state(n2, own_site(zwrap(zi - 1)));
            }
            if (k >= 1) {
                // plane zs-1 is below the next plane of step two
                bel1.pr = c1.p.pr;
                bel1.pm = c1.p.pm;
                bel1.uzc = c1.p.uzc;
                bel1.uzs = c1.p.uzs;
                bel1.pyz = fp1.yz;
                bel1.pzx = fp1.zx;
            }
        }
    };
    using C0 = std::integral_constant<int, 0>;
    using C1 = std::integral_constant<int, 1>;
    prefetch(0);
    int k = 0;
    for (; k + 1 < nk; k += 2) {
        body(C0{}, k, sA, sB, uB, uA);
        body(C1{}, k + 1, sB, sA, uA, uB);
    }
    if (k < nk)
        body(C0{}, k, sA, sB, uB, uA);
}

// One realization: one block per tile.  coefs[r] describes step n,
// coefs[nreal + r] step n+1.
template <typename T, int TY, bool OFF32>
__global__ void __launch_bounds__(64 * Tile2Geom<TY>::NW)
k_step_tiled2(const RealDesc *descs, const Coef *coefs, int r, int nreal, int cz) {
    const RealDesc d = descs[r];
    const Coef c0 = coefs[r];
    if (!c0.active)
        return;
    const Coef c1 = coefs[nreal + r];
    tiled2_tile<T, TY, OFF32>(d, c0, c1, xcd_remap(blockIdx.x, gridDim.x), cz);
}

// Many realizations in one launch (the ensemble form): a persistent grid
// walks the item list (every realization's tiles in the two-step tile shape)
// in rounds of gridDim.x items, with the XCD remap within a round.
// Realizations that reached n_end are skipped; one with a single step left
// takes one step.
template <typename T, int TY, bool OFF32>
__global__ void __launch_bounds__(64 * Tile2Geom<TY>::NW)
k_step_batch2(const RealDesc *descs, const Coef *coefs, const BatchItem *items, int n_items,
              int nreal) {
    const int g = gridDim.x;
    const int b = xcd_remap(blockIdx.x, g);
    for (int base = 0; base < n_items; base += g) {
        const int it = base + b;
        if (it >= n_items)
            break;
        const BatchItem item = items[it];
        const Coef c0 = coefs[item.r];
        if (!c0.active)
            continue;
        const RealDesc d = descs[item.r];
        tiled2_tile<T, TY, OFF32>(d, c0, coefs[nreal + item.r], item.tile, item.cz);
    }
}

template <typename T, int TY>
hipError_t launch_tiled2_ty(const RealDesc *desc, const Coef *coef, int r, int nreal, int nx, int ny,
                            int nz, int zh, int cz, hipStream_t stream) {
    const long blocks = (long)(nx / 64) * ((ny + TY - 1) / TY) * ((nz + cz - 1) / cz);
    if (fits_off32((long)nx * ny * (nz + 2 * zh), sizeof(T)))
        hipLaunchKernelGGL((k_step_tiled2<T, TY, true>), dim3((unsigned)blocks),
                           dim3(64 * Tile2Geom<TY>::NW), 0, stream, desc, coef, r, nreal, cz);
    else
        hipLaunchKernelGGL((k_step_tiled2<T, TY, false>), dim3((unsigned)blocks),
                           dim3(64 * Tile2Geom<TY>::NW), 0, stream, desc, coef, r, nreal, cz);
    return hipGetLastError();
}

// Launch the two-step kernel of element type T for realization r with tile
// height ty and z-chunk cz (both resolved and checked by the caller).
template <typename T>
int launch_step_tiled2_t(const RealDesc *desc, const Coef *coef, int r, int nreal, int nx, int ny,
                         int nz, int zh, int ty, int cz, hipStream_t stream) {
    hipError_t e;
    if constexpr (std::is_same<T, double>::value) {
        if (ty == 5)
            e = launch_tiled2_ty<double, 5>(desc, coef, r, nreal, nx, ny, nz, zh, cz, stream);
        else
            e = launch_tiled2_ty<double, 4>(desc, coef, r, nreal, nx, ny, nz, zh, cz, stream);
    } else {
        if (ty == 4)
            e = launch_tiled2_ty<float, 4>(desc, coef, r, nreal, nx, ny, nz, zh, cz, stream);
        else if (ty == 9)
            e = launch_tiled2_ty<float, 9>(desc, coef, r, nreal, nx, ny, nz, zh, cz, stream);
        else
            e = launch_tiled2_ty<float, 8>(desc, coef, r, nreal, nx, ny, nz, zh, cz, stream);
    }
    return (int)e;
}

} // namespace ah

namespace ah {

template <typename T, int TY, bool OFF32>
hipError_t batch2_ty(const RealDesc *desc, const Coef *coef, const BatchItem *items, int n_items,
                     int nreal, int grid, hipStream_t stream, int *grid_out) {
    if (grid_out) {
        int per_cu = 0, dev = 0, cus = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step_batch2<T, TY, OFF32>,
                                                             64 * Tile2Geom<TY>::NW, 0);
        *grid_out = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
        return e;
    }
    if (grid > n_items)
        grid = n_items;
    if (grid < 1)
        return hipSuccess;
    hipLaunchKernelGGL((k_step_batch2<T, TY, OFF32>), dim3((unsigned)grid),
                       dim3(64 * Tile2Geom<TY>::NW), 0, stream, desc, coef, items, n_items, nreal);
    return hipGetLastError();
}

// The batched two-step kernel of element type T and tile height ty (checked
// by the caller): with grid_out != NULL only its resident-block count
// (occupancy x compute units) is returned; otherwise it is launched on `grid`
// blocks.  off32: every realization's planes are below 4 GiB.
template <typename T>
int batch2_dispatch_t(int ty, bool off32, const RealDesc *desc, const Coef *coef,
                      const BatchItem *items, int n_items, int nreal, int grid, hipStream_t stream,
                      int *grid_out) {
#define AH_B2(TY_)                                                                                 \
    (off32 ? batch2_ty<T, TY_, true>(desc, coef, items, n_items, nreal, grid, stream, grid_out)    \
           : batch2_ty<T, TY_, false>(desc, coef, items, n_items, nreal, grid, stream, grid_out))
    hipError_t e;
    if constexpr (std::is_same<T, double>::value)
        e = ty == 5 ? AH_B2(5) : AH_B2(4);
    else
        e = ty == 4 ? AH_B2(4) : (ty == 9 ? AH_B2(9) : AH_B2(8));
#undef AH_B2
    return (int)e;
}

} // namespace ah
