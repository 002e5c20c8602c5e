// k_common.hpp -- small kernels shared by all step variants: FP64 time
// bookkeeping, the seeded initial condition, scratch clearing.
#pragma once

#include "ah_device.hpp"

namespace ah {

__device__ __forceinline__ double scale_factor(const RealDesc &d, double tau) {
    // a(tau) = (max(tau,0)/tau_ref)^p; p = 1 radiation, 2 matter (Sec. 4), 0 flat.
    double t = tau > 0.0 ? tau : 0.0;
    return pow(t / d.tau_ref, d.era_p);
}

// s(tau) of Eq. (8): a core-growth value s until tau_s, then s_late (when tau_s > 0).
__device__ __forceinline__ double s_at(const RealDesc &d, double tau) {
    return (d.tau_s > 0.0 && tau >= d.tau_s) ? d.s_late : d.s;
}

// FP64 bookkeeping of Eqs. (4), (5) and (8) for advancing S_n, read from
// copy `copy`.  Substituting e = e0 a^(s-1) and lambda = lambda0 a^(2(s-1))
// into the coefficients of Eqs. (4)-(5) and cancelling powers of a gives
// forms that stay finite at a(tau0) = 0:
//   c1 = (a_-/a_+)^2, c2 = dt/dx^2 (a_0/a_+)^2, c3 = dt lambda0/2 (a_0/a_+)^2 a_0^(2s),
//   d1 = (a_-/a_+)^(2(1-s)), d2 = dt/dx^2 (a_0/a_+)^(2(1-s)), d3 = 2 dt e0^2 (a_0/a_+)^2 a_+^(2s).
// When s changes between the three times of a step (core growth ending),
// each coupling takes s at its own time: d1 = (e_+/e_-)^2 =
// a_-^(2(1-s_-)) a_+^(2(s_+-1)), d2 = dt/dx^2 a_0^(2(1-s_0)) a_+^(2(s_+-1)).
__device__ __forceinline__ Coef coef_at(const RealDesc &d, int64_t n, int copy) {
    Coef c;
    c.n = n;
    c.active = (d.n_end <= 0 || n < d.n_end) ? 1 : 0;
    c.parity = copy;
    c.tau = d.tau0 + (double)n * d.dt;
    c.a_m = scale_factor(d, c.tau - 0.5 * d.dt);
    c.a_0 = scale_factor(d, c.tau);
    c.a_p = scale_factor(d, c.tau + 0.5 * d.dt);
    const double q = c.a_m / c.a_p, rr = c.a_0 / c.a_p;
    const double h = d.dt / (d.dx * d.dx);
    c.s_m = s_at(d, c.tau - 0.5 * d.dt);
    c.s_0 = s_at(d, c.tau);
    const double s_p = s_at(d, c.tau + 0.5 * d.dt);
    c.c1 = q * q;
    c.c2 = h * rr * rr;
    c.c3 = d.dt * 0.5 * d.lambda0 * rr * rr * pow(c.a_0, 2.0 * c.s_0);
    c.d1 = c.s_m == s_p ? pow(q, 2.0 * (1.0 - s_p))
                        : pow(c.a_m, 2.0 * (1.0 - c.s_m)) * pow(c.a_p, 2.0 * (s_p - 1.0));
    c.d2 = h * (c.s_0 == s_p ? pow(rr, 2.0 * (1.0 - s_p))
                             : pow(c.a_0, 2.0 * (1.0 - c.s_0)) * pow(c.a_p, 2.0 * (s_p - 1.0)));
    c.d3 = 2.0 * d.dt * d.e0 * d.e0 * rr * rr * pow(c.a_p, 2.0 * s_p);
    return c;
}

// One thread per realization: the coefficients of the next pass over
// memory.  steps = 0: coef[r] describes the current state (measurement
// only).  steps = 1: coef[r] is step n; the counter moves to n+1 and the
// current copy flips.  steps = 2: coef[r] is step n and coef[nreal + r] step
// n+1, both read from the current copy; the counter moves on by the number of
// active steps and the copy flips once.  Realizations that reached n_end
// stay (their passes are skipped by the kernels).
__global__ void k_bookkeep(const RealDesc *desc, int64_t *step, int32_t *copy, Coef *coef,
                           int nreal, int steps) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nreal)
        return;
    const RealDesc d = desc[r];
    const int64_t n = step[r];
    const int cp = copy[r];
    const Coef c = coef_at(d, n, cp);
    coef[r] = c;
    if (steps <= 0 || !c.active)
        return;
    int64_t adv = 1;
    if (steps == 2) {
        const Coef c2 = coef_at(d, n + 1, cp);
        coef[nreal + r] = c2;
        adv += c2.active;
    }
    step[r] = n + adv;
    copy[r] = cp ^ 1;
}

// SplitMix64 (Steele, Lea & Flood 2014): output number k of the generator
// seeded with `seed` is the fixed 64-bit mix of seed + k * 0x9e3779b97f4a7c15.
__device__ __forceinline__ uint64_t splitmix64_output(uint64_t seed, uint64_t k) {
    uint64_t v = seed + k * 0x9e3779b97f4a7c15ull;
    v = (v ^ (v >> 30)) * 0xbf58476d1ce4e5b9ull;
    v = (v ^ (v >> 27)) * 0x94d049bb133111ebull;
    return v ^ (v >> 31);
}

// Initial state (Sec. 2, after Eq. (8)): phi = sigma e^{i theta} with
// theta = 2 pi u - pi, u = (output idx+1 >> 11) 2^-53, computed in FP64 and
// rounded once to the storage type; Pi = A = E = 0 (Gauss's law holds).  The
// second copy is cleared too.  kind: AH_INIT_RANDOM_PHASE or VACUUM.
template <typename T>
__global__ void __launch_bounds__(256) k_init(const RealDesc *desc, int r, int kind, uint64_t seed) {
    const RealDesc d = desc[r];
    const T zero = 0;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < d.N;
         idx += (int64_t)gridDim.x * blockDim.x) {
        double pr = d.sigma, pi = 0.0;
        if (kind == AH_INIT_RANDOM_PHASE) {
            uint64_t bits = splitmix64_output(seed, (uint64_t)idx + 1u) >> 11;
            double theta = kTwoPi * ((double)bits * 0x1.0p-53) - kPi;
            double s, c;
            sincos(theta, &s, &c);
            pr = d.sigma * c;
            pi = d.sigma * s;
        }
        plane<T>(d, P_PHR)[idx] = (T)pr;
        plane<T>(d, P_PHI)[idx] = (T)pi;
        for (int k = 2; k < plane_count(d.layout); ++k)
            plane<T>(d, k)[idx] = zero;
    }
}

// Clear n 64-bit words (used instead of a memset so the step sequence can be
// graph-captured).
__global__ void k_zero_u64(unsigned long long *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

} // namespace ah
