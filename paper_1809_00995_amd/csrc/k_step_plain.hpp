// k_step_plain.hpp -- the plain step kernel: one thread per site, every
// neighbour value read from memory, every transcendental evaluated where the
// formula has it.  This is the reference GPU variant the tiled kernel is
// measured against; it works for any extents.
#pragma once

#include "ah_device.hpp"

namespace ah {

// Periodic site index of (x, y, z) + (sx, sy, sz), |s| <= 1.
__device__ __forceinline__ int site_shift(int x, int y, int z, int sx, int sy, int sz, int nx,
                                          int ny, int nz) {
    x += sx;
    y += sy;
    z += sz;
    x = x < 0 ? x + nx : (x >= nx ? x - nx : x);
    y = y < 0 ? y + ny : (y >= ny ? y - ny : y);
    z = z < 0 ? z + nz : (z >= nz ? z - nz : z);
    return x + nx * (y + ny * z);
}

// One staggered leapfrog step S_n -> S_{n+1}, Sec. 2, Eqs. (4)-(7):
//   Pi+  = c1 Pi- + c2 sum_j [e^{iA_j^x} phi^{x+j} - 2 phi^x + e^{-iA_j^{x-j}} phi^{x-j}]
//          - c3 (|phi|^2 - sigma^2) phi
//   E_i+ = d1 E_i- + d3 Im[conj(phi^{x+i}) e^{-iA_i^x} phi^x]
//          - d2 sum_{j != i} [sin Xi_ij^x - sin Xi_ij^{x-j}],
//   Xi_ij^y = A_i^y + A_j^{y+i} - A_i^{y+j} - A_j^y                (Eq. (3))
//   phi^{n+1} = phi^n + dt Pi+,  A^{n+1} = A^n + dt E+.
// phi and A are read from one copy and written to the other; Pi and E are
// updated in place in the 15-plane layout (each is read only at its own
// site) and written to the other copy in the 20-plane layout.
template <typename T>
__global__ void __launch_bounds__(256) k_step_plain(const RealDesc *descs, const Coef *coefs, int r) {
    const RealDesc d = descs[r];
    const Coef c = coefs[r];
    if (!c.active)
        return;
    const int64_t gidx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gidx >= d.N)
        return;
    const int o = (int)gidx;
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const int x = o % nx, y = (o / nx) % ny, z = o / (nx * ny);
    const int par = c.parity;

    const int L = d.layout;
    const T *phr = plane<T>(d, field_plane(0, par, L));
    const T *phi = plane<T>(d, field_plane(1, par, L));
    const T *A[3] = { plane<T>(d, field_plane(4, par, L)), plane<T>(d, field_plane(5, par, L)),
                      plane<T>(d, field_plane(6, par, L)) };
    const T *pir = plane<T>(d, field_plane(2, par, L)), *pii = plane<T>(d, field_plane(3, par, L));
    const T *E[3] = { plane<T>(d, field_plane(7, par, L)), plane<T>(d, field_plane(8, par, L)),
                      plane<T>(d, field_plane(9, par, L)) };
    T *pir_o = plane<T>(d, field_plane(2, par ^ 1, L)), *pii_o = plane<T>(d, field_plane(3, par ^ 1, L));
    T *E_o[3] = { plane<T>(d, field_plane(7, par ^ 1, L)), plane<T>(d, field_plane(8, par ^ 1, L)),
                  plane<T>(d, field_plane(9, par ^ 1, L)) };
    T *phr_o = plane<T>(d, field_plane(0, par ^ 1, L));
    T *phi_o = plane<T>(d, field_plane(1, par ^ 1, L));
    T *A_o[3] = { plane<T>(d, field_plane(4, par ^ 1, L)), plane<T>(d, field_plane(5, par ^ 1, L)),
                  plane<T>(d, field_plane(6, par ^ 1, L)) };

    const T c1 = (T)c.c1, c2 = (T)c.c2, c3 = (T)c.c3;
    const T d1 = (T)c.d1, d2 = (T)c.d2, d3 = (T)c.d3;
    const T dt = (T)d.dt, s2 = (T)(d.sigma * d.sigma);

    int fwd[3], bwd[3];
    for (int j = 0; j < 3; ++j) {
        fwd[j] = site_shift(x, y, z, j == 0, j == 1, j == 2, nx, ny, nz);
        bwd[j] = site_shift(x, y, z, -(j == 0), -(j == 1), -(j == 2), nx, ny, nz);
    }

    const T pr = phr[o], pm = phi[o];
    T a[3], ca[3], sa[3];
    for (int j = 0; j < 3; ++j) {
        a[j] = A[j][o];
        sincos_t(a[j], &sa[j], &ca[j]);
    }

    // Eq. (4)
    T lr = (T)-6 * pr, li = (T)-6 * pm;
    for (int j = 0; j < 3; ++j) {
        const T qr = phr[fwd[j]], qi = phi[fwd[j]];
        lr += ca[j] * qr - sa[j] * qi;
        li += ca[j] * qi + sa[j] * qr;
        T sm, cm;
        sincos_t(A[j][bwd[j]], &sm, &cm);
        const T mr = phr[bwd[j]], mi = phi[bwd[j]];
        lr += cm * mr + sm * mi;
        li += cm * mi - sm * mr;
    }
    const T v = pr * pr + pm * pm - s2;
    const T pnr = c1 * pir[o] + c2 * lr - c3 * v * pr;
    const T pni = c1 * pii[o] + c2 * li - c3 * v * pm;
    pir_o[o] = pnr;
    pii_o[o] = pni;
    phr_o[o] = pr + dt * pnr;    // Eq. (6)
    phi_o[o] = pm + dt * pni;

    // Eq. (5)
    for (int i = 0; i < 3; ++i) {
        const T qr = phr[fwd[i]], qi = phi[fwd[i]];
        const T wr = ca[i] * pr + sa[i] * pm;      // e^{-i A_i} phi^x
        const T wi = ca[i] * pm - sa[i] * pr;
        const T cur = qr * wi - qi * wr;
        T curl = 0;
        for (int j = 0; j < 3; ++j) {
            if (j == i)
                continue;
            const int xij = site_shift(x, y, z, (i == 0) - (j == 0), (i == 1) - (j == 1),
                                       (i == 2) - (j == 2), nx, ny, nz);   // x + i - j
            const T xi0 = a[i] + A[j][fwd[i]] - A[i][fwd[j]] - a[j];
            const T xi1 = A[i][bwd[j]] + A[j][xij] - a[i] - A[j][bwd[j]];
            curl += sin_t(xi0) - sin_t(xi1);
        }
        const T en = d1 * E[i][o] + d3 * cur - d2 * curl;
        E_o[i][o] = en;
        A_o[i][o] = a[i] + dt * en;             // Eq. (7)
    }
}

} // namespace ah
