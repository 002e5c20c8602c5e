// k_measure_tiled.hpp -- the read-only measuring pass for gfx950: the network
// diagnostics of a state S_n (Sec. 2, Eqs. (9)-(12)) without advancing it.
//
// The tile geometry and the per-site arithmetic are those of the tiled step
// kernel's measuring mode (k_step_tiled.hpp: measure_densities, the shared
// wrap counts, the winding formula), so a state gives the same per-site
// values whichever pass measures it; only the order of the FP64 sums differs.
// What this kernel changes is the schedule, for a pass that reads 40 (FP32)
// or 80 (FP64) bytes per site and computes several hundred instructions on
// them:
//  - Only the forward halo is staged (the row above the tile and the column
//    to its right): the diagnostics read no backward neighbour.
//  - The global reads of plane z+2 (and the momenta of plane z+1) are issued
//    one iteration ahead, into registers, and both barriers of an iteration
//    order LDS only (lds_barrier), so the reads stay in flight while plane z
//    is measured.
//  - Planes z and z+1 live in two LDS buffers.  An iteration first forms the
//    wrap counts of plane z+1's in-plane links (each once, by the thread that
//    staged the site; the halo sites' by the halo threads) and of plane z's
//    z links at x, x+x and x+y, then measures plane z, then stages plane z+2
//    into plane z's buffer.
//  - OFF32: every plane is below 4 GiB, so each global address is one 32-bit
//    byte offset from a plane base held in scalar registers.
#pragma once

#include "k_step_tiled.hpp"

namespace ah {

template <typename T, int TY, bool OFF32>
__device__ __forceinline__ void measure_tile(const RealDesc &d, const Coef &c, int tile, int cz,
                                             Slot *slot, int8_t *wind) {
    using G = TileGeom<TY>;
    static_assert(G::HALO_FWD <= 64 * TY, "one forward halo site per thread at most");
    __shared__ T lds[2][Q_COUNT][G::S];
    __shared__ float lth[2][G::S];      // FP32 phase of phi
    __shared__ T laz[2][G::S];          // raw A_z
    __shared__ int lcnt[2][2][G::S];    // wrap counts of the x and y links

    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const int ntx = nx >> 6, nty = (ny + TY - 1) / TY;
    const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
    const int x0 = tx << 6, y0 = ty * TY, z0 = tz * cz;
    const int z1 = min(z0 + cz, nz);

    const int t = threadIdx.x, lx = t & 63, ly = t >> 6;
    const bool owner = (y0 + ly) < ny;       // rows past a ragged tile edge only stage data
    const int q = G::li(lx, ly);
    const int own_xy = x0 + lx + nx * wrap_mod(y0 + ly, ny);
    // this thread's forward halo site, if any
    const bool has_h = t < G::HALO_FWD;
    int hx = 0, hy = 0;
    if (has_h)
        G::halo_fwd(t, hx, hy);
    const int hk = G::li(hx, hy);
    const int h_xy = wrap_mod(x0 + hx, nx) + nx * wrap_mod(y0 + hy, ny);
    const bool h_top = hy == TY && hx < 64;     // its x link is a tile plaquette's
    const bool h_right = hx == 64 && hy < TY;   // its y link is a tile plaquette's

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
    const int plane_sites = nx * ny;

    MeasAcc macc;
    meas_init(macc, d, c);

    struct Raw {
        T pr, pm, ax, ay, az;
    };
    struct Mom {
        T pr, pi, ex, ey, ez;
    };
    // element s of a plane
    auto at = [&](gptr<const T> base, int s) -> gptr<const T> {
        if constexpr (OFF32)
            return (gptr<const T>)((gptr<const char>)base + (uint32_t)s * (uint32_t)sizeof(T));
        else
            return base + s;
    };
    auto fetch = [&](int z, int xy, Raw &w) {
        const int s = xy + plane_sites * zmap(d, z);
        w.pr = *at(phr, s);
        w.pm = *at(phi, s);
        w.ax = *at(A0, s);
        w.ay = *at(A1, s);
        w.az = *at(A2, s);
    };
    auto fetch_mom = [&](int z, Mom &m) {
        // read once, by this thread only: streaming loads
        const int s = own_xy + plane_sites * zmap(d, z);
        m.pr = __builtin_nontemporal_load(at(pir, s));
        m.pi = __builtin_nontemporal_load(at(pii, s));
        m.ex = __builtin_nontemporal_load(at(E0, s));
        m.ey = __builtin_nontemporal_load(at(E1, s));
        m.ez = __builtin_nontemporal_load(at(E2, s));
    };
    // phasors and phase of a site into LDS buffer bf at k
    auto stage = [&](int bf, int k, const Raw &w, SiteV<T> &v) {
        v.pr = w.pr;
        v.pm = w.pm;
        v.ax = w.ax;
        v.ay = w.ay;
        v.az = w.az;
        sincos_t(v.ax, &v.uxs, &v.uxc);
        sincos_t(v.ay, &v.uys, &v.uyc);
        sincos_t(v.az, &v.uzs, &v.uzc);
        v.th = phase_f32((float)v.pm, (float)v.pr);
        lds[bf][Q_PR][k] = v.pr;
        lds[bf][Q_PI][k] = v.pm;
        lds[bf][Q_UXC][k] = v.uxc;
        lds[bf][Q_UXS][k] = v.uxs;
        lds[bf][Q_UYC][k] = v.uyc;
        lds[bf][Q_UYS][k] = v.uys;
        lds[bf][Q_UZC][k] = v.uzc;
        lds[bf][Q_UZS][k] = v.uzs;
        lth[bf][k] = v.th;
        laz[bf][k] = v.az;
    };
    // wrap count of the link from LDS site ka to kb of buffer bf, raw angle a
    auto link_count = [&](int bf, int ka, int kb, T a) {
        int m;
        if (!wrap_count_f32(lth[bf][ka], lth[bf][kb], (float)a, m))
            m = wrap_count(phase64(lds[bf][Q_PR][kb], lds[bf][Q_PI][kb]) -
                           phase64(lds[bf][Q_PR][ka], lds[bf][Q_PI][ka]) + (double)a);
        return m;
    };
    // in-plane counts of buffer bf: this thread's site (angles ax, ay) and its
    // halo site's tile link (angle ha)
    auto plane_counts = [&](int bf, T ax, T ay, T ha, int &mx, int &my) {
        mx = link_count(bf, q, q + 1, ax);
        my = link_count(bf, q, q + G::W, ay);
        lcnt[bf][0][q] = mx;
        lcnt[bf][1][q] = my;
        if (h_top)
            lcnt[bf][0][hk] = link_count(bf, hk, hk + 1, ha);
        else if (h_right)
            lcnt[bf][1][hk] = link_count(bf, hk, hk + G::W, ha);
    };
    auto halo_angle = [&](const SiteV<T> &v) { return h_top ? v.ax : v.ay; };

    // prologue: planes z0 (buffer 0) and z0+1 (buffer 1) staged, plane z0+2
    // and the momenta of z0 in flight
    SiteV<T> cur, nxt, hv;
    Raw rw, hrw;
    Mom mom;
    T ha_c = 0, ha_n = 0;
    fetch(z0, own_xy, rw);
    if (has_h)
        fetch(z0, h_xy, hrw);
    stage(0, q, rw, cur);
    if (has_h) {
        stage(0, hk, hrw, hv);
        ha_c = halo_angle(hv);
    }
    fetch(z0 + 1, own_xy, rw);
    if (has_h)
        fetch(z0 + 1, h_xy, hrw);
    stage(1, q, rw, nxt);
    if (has_h) {
        stage(1, hk, hrw, hv);
        ha_n = halo_angle(hv);
    }
    fetch_mom(z0, mom);
    if (z0 + 1 < z1) {
        fetch(z0 + 2, own_xy, rw);
        if (has_h)
            fetch(z0 + 2, h_xy, hrw);
    }
    lds_barrier();
    int mx_c, my_c;
    plane_counts(0, cur.ax, cur.ay, ha_c, mx_c, my_c);
    lds_barrier();

    for (int z = z0; z < z1; ++z) {
        const int cb = (z - z0) & 1, nb = cb ^ 1;
        const T(*Lc)[G::S] = lds[cb];
        const T(*Ln)[G::S] = lds[nb];
        // wrap counts: the in-plane links of plane z+1, the z links of plane z
        // at x, x+x and x+y
        int mx_n, my_n;
        plane_counts(nb, nxt.ax, nxt.ay, ha_n, mx_n, my_n);
        const int mz = wrap_count_link(cur.th, nxt.th, cur.az, [&]() {
            return phase64(nxt.pr, nxt.pm) - phase64(cur.pr, cur.pm);
        });
        const int mz_xp = wrap_count_link(lth[cb][q + 1], lth[nb][q + 1], laz[cb][q + 1], [&]() {
            return phase64(Ln[Q_PR][q + 1], Ln[Q_PI][q + 1]) - phase64(Lc[Q_PR][q + 1], Lc[Q_PI][q + 1]);
        });
        const int mz_yp = wrap_count_link(lth[cb][q + G::W], lth[nb][q + G::W], laz[cb][q + G::W], [&]() {
            return phase64(Ln[Q_PR][q + G::W], Ln[Q_PI][q + G::W]) -
                   phase64(Lc[Q_PR][q + G::W], Lc[Q_PI][q + G::W]);
        });
        const int my_xp = lcnt[cb][1][q + 1], mx_yp = lcnt[cb][0][q + G::W];
        if (owner) {
            // Eqs. (9)-(12) for site (x, z)
            MeasSite<T> mv;
            mv.pr = cur.pr; mv.pm = cur.pm; mv.pr0 = mom.pr; mv.pi0 = mom.pi;
            mv.ax = cur.ax; mv.ay = cur.ay; mv.az = cur.az;
            mv.ex0 = mom.ex; mv.ey0 = mom.ey; mv.ez0 = mom.ez;
            mv.uxc = cur.uxc; mv.uxs = cur.uxs; mv.uyc = cur.uyc; mv.uys = cur.uys;
            mv.uzc = cur.uzc; mv.uzs = cur.uzs;
            mv.pr_xp = Lc[Q_PR][q + 1]; mv.pi_xp = Lc[Q_PI][q + 1];
            mv.pr_yp = Lc[Q_PR][q + G::W]; mv.pi_yp = Lc[Q_PI][q + G::W];
            mv.pr_zp = nxt.pr; mv.pi_zp = nxt.pm;
            mv.uyc_xp = Lc[Q_UYC][q + 1]; mv.uys_xp = Lc[Q_UYS][q + 1];
            mv.uzc_xp = Lc[Q_UZC][q + 1]; mv.uzs_xp = Lc[Q_UZS][q + 1];
            mv.uxc_yp = Lc[Q_UXC][q + G::W]; mv.uxs_yp = Lc[Q_UXS][q + G::W];
            mv.uzc_yp = Lc[Q_UZC][q + G::W]; mv.uzs_yp = Lc[Q_UZS][q + G::W];
            mv.uxc_zp = nxt.uxc; mv.uxs_zp = nxt.uxs; mv.uyc_zp = nxt.uyc; mv.uys_zp = nxt.uys;
            int w3[3] = { 0, 0, 0 };
            if (measure_densities(macc, mv)) {
                // Eq. (11): W_ij = -(m_i(x) + m_j(x+i) - m_i(x+j) - m_j(x))
                w3[0] = -(mx_c + my_xp - mx_yp - my_c);
                w3[1] = -(my_c + mz_yp - my_n - mz);
                w3[2] = -(mz + mx_n - mz_xp - mx_c);
                count_windings(macc, w3);
            }
            if (wind) {
                const size_t s = (size_t)own_xy + (size_t)plane_sites * (size_t)zmap(d, z);
                for (int k = 0; k < 3; ++k)
                    wind[(size_t)k * (size_t)d.N + s] = (int8_t)w3[k];
            }
        }
        lds_barrier();              // buffer cb is free
        // plane z+2 into buffer cb from the registers fetched last iteration;
        // then plane z+3 and the momenta of z+1 in flight
        SiteV<T> nn = nxt;
        T ha_nn = 0;
        if (z + 1 < z1) {
            stage(cb, q, rw, nn);
            if (has_h) {
                stage(cb, hk, hrw, hv);
                ha_nn = halo_angle(hv);
            }
            fetch_mom(z + 1, mom);
            if (z + 2 < z1) {
                fetch(z + 3, own_xy, rw);
                if (has_h)
                    fetch(z + 3, h_xy, hrw);
            }
        }
        cur = nxt;
        nxt = nn;
        ha_n = ha_nn;
        mx_c = mx_n;
        my_c = my_n;
        lds_barrier();              // plane z+2 and the counts of plane z+1 visible
    }
    meas_commit<TY>(macc, slot, c, tile == 0);
}

// One realization: one block per tile and z-chunk (tiles numbered x-fastest,
// then y, then z-chunk), with the XCD remap of the step kernels.
template <typename T, int TY, bool OFF32>
__global__ void __launch_bounds__(64 * TY)
k_measure_tiled(const RealDesc *descs, const Coef *coefs, int r, int cz, Slot *slot,
                int8_t *wind) {
    const RealDesc d = descs[r];
    const Coef c = coefs[r];
    measure_tile<T, TY, OFF32>(d, c, xcd_remap(blockIdx.x, gridDim.x), cz, slot, wind);
}

// Many realizations in one launch (the ensemble form): a persistent grid walks
// the item list (realization, tile, z-chunk) in rounds of gridDim.x items, as
// the batched step kernels do; a realization whose state is past its n_end is
// skipped, and every other one measures into slots[r].  OFF32: every
// realization's planes are below 4 GiB.  The FP32 form is held to three
// wavefronts per SIMD (at most 168 VGPRs), the occupancy of the single-
// realization pass; the item loop alone would take it one register past.
template <typename T, int TY, bool OFF32>
__global__ void __launch_bounds__(64 * TY) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 1)))
k_measure_batch(const RealDesc *descs, const Coef *coefs, const BatchItem *items, int n_items,
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
        measure_tile<T, TY, OFF32>(d, c, item.tile, item.cz, slots + item.r, nullptr);
    }
}

} // namespace ah
