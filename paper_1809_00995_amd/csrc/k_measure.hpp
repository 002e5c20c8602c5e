// k_measure.hpp -- standalone diagnostics of a state S_n (Sec. 2,
// Eqs. (9)-(11)), the Gauss-law residual, and the FP64 finalisation of the
// observables.  Field values of either storage type are widened to FP64 and
// every per-site quantity is formed in FP64; sums are accumulated per thread
// in FP64, reduced over the wavefront and the block, and added to the
// measurement slot with one FP64 (or 64-bit integer) atomic per block and sum.
#pragma once

#include "ah_device.hpp"
#include "k_step_plain.hpp"

namespace ah {

constexpr int kMeasureThreads = 256;
constexpr int kWaves = kMeasureThreads / 64;

__device__ __forceinline__ double wrap_pi(double u) {
    // [u]_pi of Eq. (11): add the multiple of 2 pi that brings u into [-pi, pi).
    return u - kTwoPi * floor((u + kPi) / kTwoPi);
}

// Per-site diagnostics of S_n, summed into acc.  wind (optional) receives W
// of the xy, yz and zx plaquettes at each site (3 int8 planes).
//   K = |Pi|^2, G = dx^-2 sum_i |e^{iA_i^x} phi^{x+i} - phi^x|^2, EE = dx^-2 sum_i E_i^2,
//   BB = 2 dx^-4 sum_{xy,yz,zx} (1 - cos Xi), V = (|phi|^2 - sigma^2)^2 / 4,
//   L = a^2 K - a^2 G + g (EE - BB) - h V, rho = a^2 K + a^2 G + g (EE + BB) + h V,
//   p = a^2 K - a^2 G / 3 + g (EE + BB) / 3 - h V (one third of the stress trace),
//   g = a^(2(1-s))/(2 e0^2), h = lambda0 a^(2+2s), a = a(tau_n);
//   theta = arg phi, Y_i^x = [theta^{x+i} - theta^x + A_i^x]_pi - A_i^x,
//   W_ij^x = rint((Y_i^x + Y_j^{x+i} - Y_i^{x+j} - Y_j^x) / 2 pi).
template <typename T>
__global__ void __launch_bounds__(kMeasureThreads)
k_measure_plain(const RealDesc *descs, const Coef *coefs, int r, Slot *slot, int8_t *wind) {
    const RealDesc d = descs[r];
    const Coef c = coefs[r];
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const int par = c.parity;
    const T *F[10];
    for (int f = 0; f < 10; ++f)
        F[f] = plane<T>(d, field_plane(f, par, d.layout));
    const double a = c.a_0, a2 = a * a;
    const double g = pow(a, 2.0 * (1.0 - c.s_0)) / (2.0 * d.e0 * d.e0);
    const double h = d.lambda0 * pow(a, 2.0 + 2.0 * c.s_0);
    const double idx2 = 1.0 / (d.dx * d.dx), s2 = d.sigma * d.sigma;

    double v[A_COUNT];
    unsigned long long cnt[C_COUNT];
    for (int k = 0; k < A_COUNT; ++k)
        v[k] = 0.0;
    for (int k = 0; k < C_COUNT; ++k)
        cnt[k] = 0ull;

    for (int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gi < d.N;
         gi += (int64_t)gridDim.x * blockDim.x) {
        const int o = (int)gi;
        const int x = o % nx, y = (o / nx) % ny, z = o / (nx * ny);
        bool finite = true;
        double val[10];
        for (int f = 0; f < 10; ++f) {
            val[f] = (double)F[f][o];
            finite = finite && isfinite(val[f]);
        }
        if (!finite) {
            cnt[C_NONFIN] += 1ull;
            if (wind)
                for (int k = 0; k < 3; ++k)
                    wind[(size_t)k * d.N + o] = 0;
            continue;
        }
        const double pr = val[0], pm = val[1];
        const double K = val[2] * val[2] + val[3] * val[3];
        // neighbours x + i, and the corners x + i + j of the three plaquettes
        int fw[3];
        for (int j = 0; j < 3; ++j)
            fw[j] = site_shift(x, y, z, j == 0, j == 1, j == 2, nx, ny, nz);
        const int cxy = site_shift(x, y, z, 1, 1, 0, nx, ny, nz);
        const int cyz = site_shift(x, y, z, 0, 1, 1, nx, ny, nz);
        const int czx = site_shift(x, y, z, 1, 0, 1, nx, ny, nz);

        double G = 0.0, EE = 0.0;
        for (int i = 0; i < 3; ++i) {
            double s, co;
            sincos(val[4 + i], &s, &co);
            const double qr = (double)F[0][fw[i]], qi = (double)F[1][fw[i]];
            const double dr = co * qr - s * qi - pr, di = co * qi + s * qr - pm;
            G += dr * dr + di * di;
            EE += val[7 + i] * val[7 + i];
        }
        G *= idx2;
        EE *= idx2;

        // A at the plaquette corners: A_j(x+i), A_i(x+j)
        const double ax = val[4], ay = val[5], az = val[6];
        const double ay_px = (double)F[5][fw[0]], ax_py = (double)F[4][fw[1]];
        const double az_py = (double)F[6][fw[1]], ay_pz = (double)F[5][fw[2]];
        const double ax_pz = (double)F[4][fw[2]], az_px = (double)F[6][fw[0]];
        const double xi_xy = ax + ay_px - ax_py - ay;
        const double xi_yz = ay + az_py - ay_pz - az;
        const double xi_zx = az + ax_pz - az_px - ax;
        const double BB = 2.0 * idx2 * idx2 *
                          ((1.0 - cos(xi_xy)) + (1.0 - cos(xi_yz)) + (1.0 - cos(xi_zx)));
        const double vv = pr * pr + pm * pm - s2;
        const double V = 0.25 * vv * vv;
        const double lag = a2 * K - a2 * G + g * (EE - BB) - h * V;
        const double rho = a2 * K + a2 * G + g * (EE + BB) + h * V;
        const double pres = a2 * K - a2 * G / 3.0 + g * (EE + BB) / 3.0 - h * V;

        v[A_KIN] += a2 * K;
        v[A_GRAD] += a2 * G;
        v[A_ELEC] += g * EE;
        v[A_MAG] += g * BB;
        v[A_POT] += h * V;
        v[A_LAG] += lag;
        v[A_NUM_L] += K * lag;
        v[A_NUM_V] += K * V;
        v[A_NUM_R] += K * rho;
        v[A_DEN_L] += G * lag;
        v[A_DEN_V] += G * V;
        v[A_DEN_R] += G * rho;
        v[A_PRES_L] += pres * lag;
        v[A_RHO_L] += rho * lag;

        // winding, Eq. (11)
        auto arg = [&](int s) { return atan2((double)F[1][s], (double)F[0][s]); };
        const double t0 = atan2(pm, pr);
        const double tx = arg(fw[0]), ty = arg(fw[1]), tz = arg(fw[2]);
        const double txy = arg(cxy), tyz = arg(cyz), tzx = arg(czx);
        // Y_i at the four corners used by each plaquette
        const double yx0 = wrap_pi(tx - t0 + ax) - ax;       // Y_x^x
        const double yy0 = wrap_pi(ty - t0 + ay) - ay;       // Y_y^x
        const double yz0 = wrap_pi(tz - t0 + az) - az;       // Y_z^x
        const double yy_px = wrap_pi(txy - tx + ay_px) - ay_px;   // Y_y^{x+x}
        const double yx_py = wrap_pi(txy - ty + ax_py) - ax_py;   // Y_x^{x+y}
        const double yz_py = wrap_pi(tyz - ty + az_py) - az_py;   // Y_z^{x+y}
        const double yy_pz = wrap_pi(tyz - tz + ay_pz) - ay_pz;   // Y_y^{x+z}
        const double yx_pz = wrap_pi(tzx - tz + ax_pz) - ax_pz;   // Y_x^{x+z}
        const double yz_px = wrap_pi(tzx - tx + az_px) - az_px;   // Y_z^{x+x}
        const double loops[3] = { yx0 + yy_px - yx_py - yy0,
                                  yy0 + yz_py - yy_pz - yz0,
                                  yz0 + yx_pz - yz_px - yx0 };
        for (int k = 0; k < 3; ++k) {
            const long long w = (long long)rint(loops[k] / kTwoPi);
            cnt[C_W0 + k] += (unsigned long long)w;
            cnt[C_N0 + k] += (unsigned long long)(w < 0 ? -w : w);
            cnt[C_PIERCED] += w != 0 ? 1ull : 0ull;
            if (wind)
                wind[(size_t)k * d.N + o] = (int8_t)w;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        slot->c = c;
        slot->measured = 1;
    }
    block_accumulate<A_COUNT, C_COUNT, kWaves>(v, cnt, slot->acc.s, slot->acc.c);
}

// Gauss-law residual of S_n:
//   G_x = sum_i (E_i^x - E_i^{x-i}) a_-^(2(1-s))/e0^2 + 2 dx^2 a_-^2 Im(conj(phi^x) Pi^x),
// a_- = a(tau_{n-1/2}).  out[0] receives max |G| (as the bit pattern of a
// non-negative double, which orders like the value), out[1] the sum of G^2.
template <typename T>
__global__ void __launch_bounds__(kMeasureThreads)
k_gauss(const RealDesc *descs, const Coef *coefs, int r, unsigned long long *out) {
    const RealDesc d = descs[r];
    const Coef c = coefs[r];
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const int par = c.parity;
    const int L = d.layout;
    const T *phr = plane<T>(d, field_plane(0, par, L)), *phi = plane<T>(d, field_plane(1, par, L));
    const T *pir = plane<T>(d, field_plane(2, par, L)), *pii = plane<T>(d, field_plane(3, par, L));
    const T *E[3] = { plane<T>(d, field_plane(7, par, L)), plane<T>(d, field_plane(8, par, L)),
                      plane<T>(d, field_plane(9, par, L)) };
    const double fe = pow(c.a_m, 2.0 * (1.0 - c.s_m)) / (d.e0 * d.e0);
    const double fp = 2.0 * d.dx * d.dx * c.a_m * c.a_m;
    double mx = 0.0, sq = 0.0;
    for (int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gi < d.N;
         gi += (int64_t)gridDim.x * blockDim.x) {
        const int o = (int)gi;
        const int x = o % nx, y = (o / nx) % ny, z = o / (nx * ny);
        double div = 0.0;
        for (int i = 0; i < 3; ++i) {
            const int b = site_shift(x, y, z, -(i == 0), -(i == 1), -(i == 2), nx, ny, nz);
            div += (double)E[i][o] - (double)E[i][b];
        }
        const double charge = (double)phr[o] * (double)pii[o] - (double)phi[o] * (double)pir[o];
        const double G = fe * div + fp * charge;
        const double ag = fabs(G);
        mx = ag > mx ? ag : mx;
        sq += G * G;
    }
    __shared__ double smx[kWaves], ssq[kWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    mx = wave_max(mx);
    sq = wave_sum(sq);
    if (lane == 0) {
        smx[wave] = mx;
        ssq[wave] = sq;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0, s = 0.0;
        for (int w = 0; w < kWaves; ++w) {
            m = smx[w] > m ? smx[w] : m;
            s += ssq[w];
        }
        atomicMax(out, (unsigned long long)__double_as_longlong(m));
        unsafeAtomicAdd(reinterpret_cast<double *>(out + 1), s);
    }
}

// Observables of slot k (realization k % nreal) from the raw sums, in FP64
// (Eqs. (9)-(12)): xi_L = a sqrt(-mu V_box / (dx^3 sum L)), mu = 2 pi sigma^2;
// <v^2>_X = 2R/(1+R), R = sum K X / sum G X; length = (pi/6) dx sum |W|;
// xi_W = sqrt(V_box / length).  Slots nobody measured get step = -1.
__global__ void k_finalize(const RealDesc *descs, const Slot *slots, ah_obs *out, int nslots,
                           int nreal) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nslots)
        return;
    const RealDesc d = descs[k % nreal];
    const Slot &sl = slots[k];
    ah_obs o;
    const double dv = d.dx * d.dx * d.dx;
    const double vbox = (double)d.nx * (double)d.ny * (double)d.nz * dv;   // the slab only
    o.step = sl.measured ? sl.c.n : -1;
    o.tau = sl.c.tau;
    o.a = sl.c.a_0;
    o.n_wind = 0;
    for (int i = 0; i < 3; ++i) {
        o.net_wind_dir[i] = (int64_t)sl.acc.c[C_W0 + i];
        o.n_wind_dir[i] = (int64_t)sl.acc.c[C_N0 + i];
        o.n_wind += o.n_wind_dir[i];
    }
    o.n_pierced = (int64_t)sl.acc.c[C_PIERCED];
    o.nonfinite = (int64_t)sl.acc.c[C_NONFIN];
    o.length = (kPi / 6.0) * d.dx * (double)o.n_wind;
    o.xi_w = sqrt(vbox / o.length);
    o.kin = dv * sl.acc.s[A_KIN];
    o.grad = dv * sl.acc.s[A_GRAD];
    o.elec = dv * sl.acc.s[A_ELEC];
    o.mag = dv * sl.acc.s[A_MAG];
    o.pot = dv * sl.acc.s[A_POT];
    o.energy = o.kin + o.grad + o.elec + o.mag + o.pot;
    // p = a^2 K - a^2 G/3 + g (EE + BB)/3 - h V
    o.sum_lag = dv * sl.acc.s[A_LAG];
    o.xi_l = o.sum_lag < 0.0 ? o.a * sqrt(-(kTwoPi * d.sigma * d.sigma) * vbox / o.sum_lag)
                             : __builtin_nan("");
    o.pres = o.kin - o.grad / 3.0 + (o.elec + o.mag) / 3.0 - o.pot;
    o.pres_lag = dv * sl.acc.s[A_PRES_L];
    o.rho_lag = dv * sl.acc.s[A_RHO_L];
    o.v2_eos = 0.5 * (1.0 + 3.0 * o.pres_lag / o.rho_lag);   // Eq. (12)
    for (int i = 0; i < 3; ++i) {
        o.num[i] = dv * sl.acc.s[A_NUM_L + i];
        o.den[i] = dv * sl.acc.s[A_DEN_L + i];
        const double R = o.num[i] / o.den[i];
        o.v2[i] = 2.0 * R / (1.0 + R);
    }
    out[k] = o;
}

} // namespace ah
