// k_step_tiled.hpp -- the tiled step kernel for gfx950.
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
#pragma once

#include "ah_device.hpp"

namespace ah {

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

// sin Xi_ij(s) = Im[U_i(s) U_j(s+i) conj(U_i(s+j)) conj(U_j(s))], phasors as (cos, sin)
template <typename T>
__device__ __forceinline__ T plaq_sin(T aic, T ais, T bjc, T bjs, T cic, T cis, T djc, T djs) {
    const T wr = aic * djc + ais * djs, wi = ais * djc - aic * djs;   // U_i(s) conj(U_j(s))
    const T vr = bjc * cic + bjs * cis, vi = bjs * cic - bjc * cis;   // U_j(s+i) conj(U_i(s+j))
    return wr * vi + wi * vr;
}

template <typename T> struct SiteV {
    T pr, pm, ax, ay, az, uxc, uxs, uyc, uys, uzc, uzs;
};

__device__ __forceinline__ int wrap_mod(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

template <typename T, int TY>
__global__ void __launch_bounds__(64 * TY)
k_step_tiled(const RealDesc *descs, const Coef *coefs, int r, int cz) {
    using G = TileGeom<TY>;
    __shared__ T lds[2][Q_COUNT][G::S];

    const RealDesc d = descs[r];
    const Coef c = coefs[r];
    if (!c.active)
        return;
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const int ntx = nx >> 6, nty = (ny + TY - 1) / TY;

    // XCD-aware tile order: block b runs on XCD b % 8; XCD i gets tiles
    // [start_i, start_i + count_i) in x-fastest, then y, then z-chunk order.
    const int nb = gridDim.x, b = blockIdx.x;
    const int xcd = b & 7, per = nb >> 3, rem = nb & 7;
    const int tile = xcd * per + min(xcd, rem) + (b >> 3);
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

    auto load_site = [&](int s, SiteV<T> &v) {
        v.pr = phr[s];
        v.pm = phi[s];
        v.ax = A0[s];
        v.ay = A1[s];
        v.az = A2[s];
        sincos_t(v.ax, &v.uxs, &v.uxc);
        sincos_t(v.ay, &v.uys, &v.uyc);
        sincos_t(v.az, &v.uzs, &v.uzc);
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
        const T pr0 = pir[s], pi0 = pii[s], ex0 = E0[s], ey0 = E1[s], ez0 = E2[s];
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

        // Eq. (4): sum_j [U_j(x) phi(x+j) + conj(U_j(x-j)) phi(x-j)] - 6 phi
        const T pr = cur.pr, pm = cur.pm;
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
            pir[s] = pnr;
            pii[s] = pni;
            E0[s] = enx;
            E1[s] = eny;
            E2[s] = enz;
            ophr[s] = pr + dt * pnr;          // Eq. (6)
            ophi[s] = pm + dt * pni;
            oA0[s] = cur.ax + dt * enx;       // Eq. (7)
            oA1[s] = cur.ay + dt * eny;
            oA2[s] = cur.az + dt * enz;
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

template <typename T, int TY>
hipError_t launch_tiled_ty(const RealDesc *desc, const Coef *coef, int r, int nx, int ny, int nz,
                           int cz, hipStream_t stream) {
    const long blocks = (long)(nx / 64) * ((ny + TY - 1) / TY) * ((nz + cz - 1) / cz);
    hipLaunchKernelGGL((k_step_tiled<T, TY>), dim3((unsigned)blocks), dim3(64 * TY), 0, stream,
                       desc, coef, r, cz);
    return hipGetLastError();
}

// Valid tile heights: FP32 2, 4, 8, 16; FP64 2, 4, 8.
inline bool tiled_ty_valid(bool fp64, int ty) {
    return ty == 2 || ty == 4 || ty == 8 || (!fp64 && ty == 16);
}

inline int launch_step_tiled(bool fp64, const RealDesc *desc, const Coef *coef, int r, int nx,
                             int ny, int nz, int tile_y, int chunk_z, hipStream_t stream) {
    int ty = tile_y, cz = chunk_z;
    tiled_defaults(fp64, nx, ny, nz, ty, cz);
    if (nx % 64 != 0 || !tiled_ty_valid(fp64, ty) || cz < 1)
        return (int)hipErrorInvalidValue;
    hipError_t e;
    if (fp64) {
        switch (ty) {
        case 2: e = launch_tiled_ty<double, 2>(desc, coef, r, nx, ny, nz, cz, stream); break;
        case 4: e = launch_tiled_ty<double, 4>(desc, coef, r, nx, ny, nz, cz, stream); break;
        default: e = launch_tiled_ty<double, 8>(desc, coef, r, nx, ny, nz, cz, stream); break;
        }
    } else {
        switch (ty) {
        case 2: e = launch_tiled_ty<float, 2>(desc, coef, r, nx, ny, nz, cz, stream); break;
        case 4: e = launch_tiled_ty<float, 4>(desc, coef, r, nx, ny, nz, cz, stream); break;
        case 8: e = launch_tiled_ty<float, 8>(desc, coef, r, nx, ny, nz, cz, stream); break;
        default: e = launch_tiled_ty<float, 16>(desc, coef, r, nx, ny, nz, cz, stream); break;
        }
    }
    return (int)e;
}

} // namespace ah
