/*
 * ah_oracle.h -- plain FP64 CPU oracle for the Abelian-Higgs lattice leapfrog
 * (Correia & Martins, "Abelian-Higgs Cosmic String Evolution with CUDA",
 * arXiv:1809.00995, Sec. 2).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link or
 * call this code: only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no header, helper or constant with the
 * HIP library; the two are compared only through their outputs.
 *
 * State layout: one array of 10 planes of nx*ny*nz doubles, plane order
 *   0 phi_re, 1 phi_im, 2 Pi_re, 3 Pi_im, 4 A_x, 5 A_y, 6 A_z, 7 E_x, 8 E_y, 9 E_z
 * with site index idx = x + nx*(y + ny*z) and periodic boundaries.  A state
 * S_n holds phi^n, A^n (integer time level) and Pi^{n-1/2}, E^{n-1/2}
 * (half-step momenta), as in the staggered scheme of Sec. 2, Eqs. (4)-(7).
 */
#ifndef AH_ORACLE_H
#define AH_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny, nz;
    double dx, dt;          /* lattice spacing and conformal time step          */
    double tau0, tau_ref;   /* tau_n = tau0 + n*dt; a = (max(tau,0)/tau_ref)^p  */
    double era_p;           /* 0 flat, 1 radiation (a ~ tau), 2 matter (tau^2)  */
    double s;               /* comoving-width parameter, Eq. (8)                */
    double lambda0, e0, sigma;
    uint64_t seed;
    double s_late, tau_s;   /* s(tau) = s_late for tau >= tau_s when tau_s > 0 */
} or_params;

typedef struct {
    double tau, a_m, a_0, a_p;      /* a at tau_{n-1/2}, tau_n, tau_{n+1/2} */
    double c1, c2, c3;              /* Pi update coefficients, Eq. (4)      */
    double d1, d2, d3;              /* E update coefficients, Eq. (5)       */
} or_coeffs;

typedef struct {
    int64_t step;
    double tau, a;
    int64_t n_wind;            /* sum over plaquettes of |W|                  */
    int64_t n_wind_dir[3];     /* same, per orientation xy, yz, zx           */
    int64_t net_wind_dir[3];   /* signed sum of W per orientation (always 0) */
    int64_t n_pierced;         /* number of plaquettes with W != 0           */
    double length, xi_w;       /* (pi/6) dx n_wind ; sqrt(V_box / length)    */
    double sum_lag, xi_l;      /* dx^3 sum L ; a sqrt(-mu V_box / sum_lag)   */
    double num[3], den[3], v2[3];  /* weights X = L, V, rho                  */
    double kin, grad, elec, mag, pot, energy; /* dx^3-weighted parts of rho  */
    double pres;               /* dx^3 sum p                                 */
    double pres_lag, rho_lag;  /* dx^3 sum p L, dx^3 sum rho L               */
    double v2_eos;             /* (1 + 3 pres_lag / rho_lag) / 2, Eq. (12)   */
    int64_t nonfinite;         /* sites with a non-finite field value        */
} or_obs;

double or_scale_factor(const or_params *p, double tau);
double or_s_of(const or_params *p, double tau);
void or_coefficients(const or_params *p, int64_t n, or_coeffs *c);

/* k-th output (k >= 1) of the SplitMix64 generator seeded with `seed`. */
uint64_t or_splitmix64(uint64_t seed, uint64_t k);

/* Random-phase initial condition (Sec. 2, text after Eq. (8)). */
void or_init_random_phase(const or_params *p, double *state);

/* S_n -> S_{n+1}; `in` and `out` must not overlap. */
void or_step(const or_params *p, int64_t n, const double *in, double *out);

/* S_{n+1} at the listed sites only: out[k*10 + f] = field f at site idx[k]. */
void or_step_sites(const or_params *p, int64_t n, const double *in, int64_t nsites,
                   const int64_t *idx, double *out);

/* Diagnostics of S_n.  wmap (optional) receives W for the xy, yz, zx
 * plaquettes at each site, as 3 planes of int8. */
void or_measure(const or_params *p, int64_t n, const double *state,
                or_obs *obs, int8_t *wmap);

/* Gauss-law residual of S_n; gmap (optional) receives G_x per site. */
void or_gauss(const or_params *p, int64_t n, const double *state,
              double *max_abs, double *rms, double *gmap);

/* Number of threads the parallel loops use (OpenMP), 1 without OpenMP. */
int or_threads(void);

#ifdef __cplusplus
}
#endif
#endif
