// ah_device.hpp -- device-side types and helpers of the gfx950 Abelian-Higgs library.
//
// Every kernel reads its realization's description (RealDesc) and the FP64
// step bookkeeping (Coef) from device memory, so kernel arguments are the same
// on every step and a sequence of steps can be replayed from a captured graph.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ah.h"

namespace ah {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kTwoPi = 6.28318530717958647692528676655900577;

// Field numbers (planes of the first copy) and the second-copy planes of
// phi and A in the 15-plane layout.
enum : int { P_PHR = 0, P_PHI = 1, P_PIR = 2, P_PII = 3, P_AX = 4, P_EX = 7,
             P_PHR2 = 10, P_AX2 = 12 };

// Static description of one realization (written once by ah_init).
struct RealDesc {
    char *base;            // 15 or 20 planes of N elements
    int32_t nx, ny, nz;
    int32_t elem;          // bytes per element (4 or 8)
    int32_t layout;        // AH_LAYOUT_15 or AH_LAYOUT_20
    int32_t zh;            // 0: periodic in z; > 0: a slab with zh halo planes a side
    int64_t N;             // elements per plane: nx * ny * (nz + 2 zh)
    double dx, dt, tau0, tau_ref, era_p, s, lambda0, e0, sigma;
    int64_t step0, n_end;
    double s_late, tau_s;  // s(tau) = s_late from tau_s on when tau_s > 0
};

// A work item of the batched kernels: tile `tile` of realization r, with that
// realization's z-chunk cz.
struct BatchItem {
    int32_t r, tile, cz, pad;
};

// FP64 bookkeeping for advancing realization r from S_n (written on the
// device by k_bookkeep before each step or measurement).
struct Coef {
    int64_t n;             // step index of the state being read
    int32_t active;        // 0 once the realization has reached n_end
    int32_t parity;        // copy holding the state read (see field_plane)
    double tau, a_m, a_0, a_p;
    double s_m, s_0;       // comoving-width parameter at tau_{n-1/2}, tau_n
    double c1, c2, c3;     // Pi update, Eq. (4)
    double d1, d2, d3;     // E update, Eq. (5)
};

// Raw per-measurement accumulators (sums over sites, before the dx^3 factor).
// The sum of the pressure is linear in the five parts of the energy density
// and is formed from their sums; the Lagrangian, a difference of those parts
// that can be much smaller than each, is summed site by site.
enum : int { A_KIN, A_GRAD, A_ELEC, A_MAG, A_POT, A_LAG,
             A_NUM_L, A_NUM_V, A_NUM_R, A_DEN_L, A_DEN_V, A_DEN_R,
             A_PRES_L, A_RHO_L, A_COUNT };
enum : int { C_W0, C_W1, C_W2, C_N0, C_N1, C_N2, C_PIERCED, C_NONFIN, C_COUNT };

struct Acc {
    double s[A_COUNT];
    unsigned long long c[C_COUNT];   // two's complement for signed sums
};

// One measurement slot: the sums, the bookkeeping of the measured state, and
// whether a measurement kernel wrote it.  Cleared to zero before use.
struct Slot {
    Acc acc;
    Coef c;
    int32_t measured;
    int32_t pad;
};

template <typename T> __device__ __forceinline__ T* plane(const RealDesc &d, int k) {
    return reinterpret_cast<T*>(d.base + (size_t)k * (size_t)d.N * sizeof(T));
}

// The same plane as a pointer into the global address space.  The planes'
// addresses come from a descriptor in memory, so the compiler cannot infer
// their address space and would emit flat accesses, which also count against
// the LDS wait counter; global accesses leave a barrier free to wait for LDS
// only while prefetched loads are in flight.
template <typename T> using gptr = __attribute__((address_space(1))) T *;

template <typename T> __device__ __forceinline__ gptr<T> gplane(const RealDesc &d, int k) {
    return (gptr<T>)(d.base + (size_t)k * (size_t)d.N * sizeof(T));
}

// Plane of field f (0..9) in copy `parity` (0 or 1).  AH_LAYOUT_15: copy 1
// of phi and A is planes 10-14 and Pi, E have one plane each (updated in
// place); AH_LAYOUT_20: copy 1 of every field is plane f + 10.
__host__ __device__ __forceinline__ int field_plane(int f, int parity, int layout) {
    if (!parity)
        return f;
    if (layout == AH_LAYOUT_20)
        return f + 10;
    if (f < 2)
        return P_PHR2 + f;
    if (f >= 4 && f < 7)
        return P_AX2 + (f - 4);
    return f;
}

// Stored z-plane of slab-relative plane z (-zh <= z < nz + zh for a slab,
// any z within one period of [0, nz) for a periodic lattice, zh = 0).  One
// expression for both, so that the compiler emits selects, not branches: a
// slab's planes never leave [0, nz + 2 zh).
__device__ __forceinline__ int zmap(const RealDesc &d, int z) {
    const int w = z + d.zh, top = d.nz + 2 * d.zh;
    return w < 0 ? w + d.nz : (w >= top ? w - d.nz : w);
}

__host__ __device__ __forceinline__ int plane_count(int layout) {
    return layout == AH_LAYOUT_20 ? 20 : 15;
}

// sin and cos of a link angle.
// Float: x = 2 pi k + r with k = rint(x / 2 pi), r from 2 pi split in a high
// and a low part (one fused multiply-add each), then the hardware sine and
// cosine of t = r / 2 pi in revolutions (|t| <= 1/2 up to the rounding of
// x / 2 pi).  The reduction's roundings (of r twice, of the float 1/(2 pi), of
// t) are bounded by 4.6e-7; measured on the GPU over 2^24 angles in [-40, 40]
// the whole error is at most 4.3e-7.  Half an ulp of an FP32 angle is 1.9e-6 at
// |x| = 40, so the stored angle itself is uncertain by more wherever |x| > 4.
// The minimax polynomial scheme used for double below gives 1.5e-7 in float
// but costs about 14 more instructions per link, 3 % of a pair of steps.
// Double: x = k pi + r with k = rint(x / pi), r = x - k pi from pi split in a
// high and a low part, so |r| <= pi/2; then
//   sin r = r + r^3 P(r^2),   cos r = 1 + r^2 Q(r^2),
// with P and Q the minimax polynomials printed by fit_polys.py (Remez
// exchange on 0 <= r <= pi/2: relative error of sin r, absolute error of
// cos r) of degrees 17 and 16, and both signs flip for odd k; error a few
// 2^-53.  The angles held by the links are far inside the range of either.
__device__ __forceinline__ void sincos_t(float x, float *s, float *c) {
    const float k = __builtin_rintf(x * 1.5915494e-01f);        // 1/(2 pi)
    float r = __builtin_fmaf(-k, 6.2831855e+00f, x);           // 2 pi, high part
    r = __builtin_fmaf(-k, -1.7484555e-07f, r);                 // 2 pi, low part
    const float t = r * 1.5915494e-01f;                         // revolutions
    *s = __builtin_amdgcn_sinf(t);
    *c = __builtin_amdgcn_cosf(t);
}

__device__ __forceinline__ void sincos_t(double x, double *s, double *c) {
    const double k = __builtin_rint(x * 0.3183098861837907);
    double r = __builtin_fma(-k, 3.141592653589793, x);
    r = __builtin_fma(-k, 1.2246467991473532e-16, r);
    const double u = r * r;
    double p = __builtin_fma(u, 2.721174976425455e-15, -7.642991490758669e-13);
    p = __builtin_fma(u, p, 1.605893970595926e-10);
    p = __builtin_fma(u, p, -2.5052106872803682e-08);
    p = __builtin_fma(u, p, 2.755731921113729e-06);
    p = __builtin_fma(u, p, -0.00019841269841209218);
    p = __builtin_fma(u, p, 0.008333333333333194);
    p = __builtin_fma(u, p, -0.16666666666666666);
    const double sr = __builtin_fma(r * u, p, r);
    double q = __builtin_fma(u, 4.61029416776206e-14, -1.1463039370063416e-11);
    q = __builtin_fma(u, q, 2.087656774105309e-09);
    q = __builtin_fma(u, q, -2.755731652522837e-07);
    q = __builtin_fma(u, q, 2.480158727914903e-05);
    q = __builtin_fma(u, q, -0.0013888888888785652);
    q = __builtin_fma(u, q, 0.04166666666666437);
    q = __builtin_fma(u, q, -0.49999999999999983);
    const double cr = __builtin_fma(u, q, 1.0);
    const unsigned long long sign = (unsigned long long)(long long)k << 63;
    *s = __longlong_as_double((long long)((unsigned long long)__double_as_longlong(sr) ^ sign));
    *c = __longlong_as_double((long long)((unsigned long long)__double_as_longlong(cr) ^ sign));
}

// FP32 phase arg(x + iy) in [-pi, pi], the quadrant and signs taken as atan2
// takes them (signed zeros included): a = min(|x|,|y|) / max(|x|,|y|) from a
// hardware reciprocal, atan a = a + a^3 T(a^2) with the minimax T printed by
// fit_polys.py, then pi/2 - . for |y| > |x|, pi - . for negative x, and the
// sign of y.  Absolute error below 5e-7 (4.3e-7 measured over all octants and
// 40 decades of magnitude).  Returns NaN when max(|x|,|y|) is below 1e-30 or
// not finite, so that callers take the FP64 phase instead.
__device__ __forceinline__ float phase_f32(float y, float x) {
    const float ax = __builtin_fabsf(x), ay = __builtin_fabsf(y);
    const float mx = __builtin_fmaxf(ax, ay), mn = __builtin_fminf(ax, ay);
    const float a = mn * __builtin_amdgcn_rcpf(mx);
    const float u = a * a;
    float t = __builtin_fmaf(u, -4.822534e-03f, 2.4734063e-02f);
    t = __builtin_fmaf(u, t, -6.0203128e-02f);
    t = __builtin_fmaf(u, t, 9.968473e-02f);
    t = __builtin_fmaf(u, t, -1.4041328e-01f);
    t = __builtin_fmaf(u, t, 1.9974214e-01f);
    t = __builtin_fmaf(u, t, -3.3332393e-01f);
    float r = __builtin_fmaf(a * u, t, a);
    r = ay > ax ? 1.5707964e+00f - r : r;
    r = __builtin_signbit(x) ? 3.1415927e+00f - r : r;
    r = __builtin_copysignf(r, y);
    return (mx >= 1e-30f && mx <= 3.0e38f) ? r : __builtin_nanf("");
}

template <typename T> __device__ __forceinline__ T sin_t(T x) {
    T s, c;
    sincos_t(x, &s, &c);
    return s;
}

// Workgroup barrier that orders LDS only: each wave waits for its own LDS
// accesses, not for its global loads, so loads issued ahead of the barrier
// (prefetches of the next plane) stay in flight across it.  For kernels that
// share data between waves through LDS alone.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------- reductions
// Sum over a 64-lane wavefront; lane 0 ends with the total.
template <typename V> __device__ __forceinline__ V wave_sum(V v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

template <typename V> __device__ __forceinline__ V wave_max(V v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        V o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Block-wide sum of NV doubles and NC 64-bit integers over a block of NW
// wavefronts, then one atomic per value into acc_s / acc_c.  Every thread of
// the block must call it.
template <int NV, int NC, int NW>
__device__ __forceinline__ void block_accumulate(double (&v)[NV], unsigned long long (&cnt)[NC],
                                                 double *acc_s, unsigned long long *acc_c) {
    static_assert(NV + NC <= 64 * NW, "block too small for the reduction");
    __shared__ double sv[NW][NV];
    __shared__ unsigned long long sc[NW][NC];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double t = wave_sum(v[k]);
        if (lane == 0)
            sv[wave][k] = t;
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        unsigned long long t = wave_sum(cnt[k]);
        if (lane == 0)
            sc[wave][k] = t;
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < NV) {
        double s = 0.0;
        for (int w = 0; w < NW; ++w)
            s += sv[w][t];
        unsafeAtomicAdd(acc_s + t, s);
    } else if (t < NV + NC) {
        unsigned long long s = 0;
        for (int w = 0; w < NW; ++w)
            s += sc[w][t - NV];
        atomicAdd(acc_c + (t - NV), s);
    }
}

} // namespace ah
