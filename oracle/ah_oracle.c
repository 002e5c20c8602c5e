/*
 * ah_oracle.c -- plain FP64 CPU oracle for the Abelian-Higgs lattice leapfrog
 * of Correia & Martins, arXiv:1809.00995, Sec. 2.
 *
 * TEST INFRASTRUCTURE ONLY (see ah_oracle.h).  Written for clarity, not speed:
 * every update reads the whole old state S_n and writes a separate S_{n+1}
 * (Jacobi order), every transcendental is evaluated where the formula has it,
 * and every sum is taken per z-plane and then over planes in a fixed order, so
 * results do not depend on the OpenMP thread count.
 *
 * Readings of the paper that this file follows (the paper is silent,
 * ambiguous or internally inconsistent on these points):
 *  - link sign: the covariant difference is exp(+iA_i^x) phi^{x+i} - phi^x,
 *    the sign used by the equations of motion, Eqs. (4)-(5), and the winding,
 *    Eq. (11); the opposite sign printed in Eq. (2) and the text after Eq. (3)
 *    would break the discrete Gauss law;
 *  - couplings e = e0 a^(s-1), lambda = lambda0 a^(2(s-1)), Eq. (8), are
 *    substituted into Eqs. (4)-(5) and the ratios simplified so that no 0/0
 *    appears at a = 0 (pow(0,0) = 1); s may change once, at tau_s (core
 *    growth, then physical width), each coupling taking s at its own time;
 *  - scale factor a(tau) = (max(tau,0)/tau_ref)^p, p = 1 radiation, 2 matter,
 *    0 flat (the normalisation is not stated in Sec. 4);
 *  - magnetic energy (1/(e^2 dx^4)) sum_{i<j} (1 - cos Xi_ij), twice the
 *    coefficient printed in Eq. (2), as required by the curl term of Eq. (5)
 *    and by the continuum limit;
 *  - densities are the conformal (action) densities of S_n as stored, with
 *    a = a(tau_n) and the momenta at tau_{n-1/2};
 *  - string tension mu = 2 pi sigma^2 (BPS value at lambda0 = 2 e0^2);
 *    xi_W = sqrt(V_box / length); length = (pi/6) dx sum |W| (Sec. 2, after
 *    Eq. (11)); [.]_pi maps to [-pi, pi) by adding multiples of 2 pi;
 *  - Gauss law: the discrete Noether charge of the lattice action under
 *    time-independent gauge transformations (not written in the paper).
 */
#include "ah_oracle.h"

#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846264338327950288
#define OR_TWO_PI 6.28318530717958647692528676655900577

enum { PHR = 0, PHI = 1, PIR = 2, PII = 3, AX = 4, EX = 7 };

static size_t sites(const or_params *p)
{
    return (size_t)p->nx * (size_t)p->ny * (size_t)p->nz;
}

/* Neighbour index of site (x,y,z) shifted by (sx,sy,sz), periodic. */
static size_t nb(const or_params *p, int x, int y, int z, int sx, int sy, int sz)
{
    int xx = (x + sx + p->nx) % p->nx;
    int yy = (y + sy + p->ny) % p->ny;
    int zz = (z + sz + p->nz) % p->nz;
    return (size_t)xx + (size_t)p->nx * ((size_t)yy + (size_t)p->ny * (size_t)zz);
}

/* unit vectors k_i */
static const int UNIT[3][3] = { { 1, 0, 0 }, { 0, 1, 0 }, { 0, 0, 1 } };

double or_scale_factor(const or_params *p, double tau)
{
    double t = tau > 0.0 ? tau : 0.0;
    return pow(t / p->tau_ref, p->era_p);
}

/* The comoving-width parameter at time tau (Sec. 2, after Eq. (8)): s before
 * tau_s and s_late from tau_s on when tau_s > 0 (a core-growth period
 * followed by the true equations of motion); s throughout otherwise. */
double or_s_of(const or_params *p, double tau)
{
    return (p->tau_s > 0.0 && tau >= p->tau_s) ? p->s_late : p->s;
}

/*
 * Coefficients of the staggered leapfrog, Sec. 2, Eqs. (4) and (5), with the
 * s-scaled couplings of Eq. (8):
 *   Pi+ = c1 Pi- + c2 [covariant Laplacian] - c3 (|phi|^2 - sigma^2) phi
 *     c1 = (a_-/a_+)^2, c2 = (dt/dx^2)(a_0/a_+)^2,
 *     c3 = dt (a_0^2/a_+)^2 lambda_0/2 = dt (lambda0/2) (a_0/a_+)^2 a_0^(2s)
 *   E+ = d1 E- + d3 Im[...] - d2 [curl]
 *     d1 = (e_+/e_-)^2 = (a_-/a_+)^(2(1-s)),
 *     d2 = (dt/dx^2)(e_+/e_0)^2 = (dt/dx^2)(a_0/a_+)^(2(1-s)),
 *     d3 = 2 dt a_0^2 e_+^2 = 2 dt e0^2 (a_0/a_+)^2 a_+^(2s).
 */
void or_coefficients(const or_params *p, int64_t n, or_coeffs *c)
{
    double tau = p->tau0 + (double)n * p->dt;
    double am = or_scale_factor(p, tau - 0.5 * p->dt);
    double a0 = or_scale_factor(p, tau);
    double ap = or_scale_factor(p, tau + 0.5 * p->dt);
    double q = am / ap;
    double r = a0 / ap;
    double h = p->dt / (p->dx * p->dx);
    double sm = or_s_of(p, tau - 0.5 * p->dt);
    double s0 = or_s_of(p, tau);
    double sp = or_s_of(p, tau + 0.5 * p->dt);

    c->tau = tau;
    c->a_m = am;
    c->a_0 = a0;
    c->a_p = ap;
    c->c1 = q * q;
    c->c2 = h * r * r;
    c->c3 = p->dt * 0.5 * p->lambda0 * r * r * pow(a0, 2.0 * s0);
    /* (e_+/e_-)^2 and (e_+/e_0)^2; with s the same at both times they reduce
     * to powers of the ratios q and r */
    c->d1 = sm == sp ? pow(q, 2.0 * (1.0 - sp))
                     : pow(am, 2.0 * (1.0 - sm)) * pow(ap, 2.0 * (sp - 1.0));
    c->d2 = h * (s0 == sp ? pow(r, 2.0 * (1.0 - sp))
                          : pow(a0, 2.0 * (1.0 - s0)) * pow(ap, 2.0 * (sp - 1.0)));
    c->d3 = 2.0 * p->dt * p->e0 * p->e0 * r * r * pow(ap, 2.0 * sp);
}

/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the state advances by the
 * golden-ratio increment and each output is a fixed bijective mix of it, so
 * the k-th output is mix(seed + k * gamma). */
uint64_t or_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + k * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/*
 * Initial conditions of Sec. 2 (text after Eq. (8)): |phi| = sigma with a
 * uniformly random phase, every other field zero (this satisfies the discrete
 * Gauss law).  The phase of site idx is theta = 2 pi u - pi with u the top 53
 * bits of SplitMix64 output number idx+1, scaled to [0,1).
 */
void or_init_random_phase(const or_params *p, double *st)
{
    size_t n = sites(p);
    memset(st, 0, 10 * n * sizeof(double));
    for (size_t idx = 0; idx < n; ++idx) {
        uint64_t bits = or_splitmix64(p->seed, (uint64_t)idx + 1u) >> 11;
        double u = (double)bits * 0x1.0p-53;
        double theta = OR_TWO_PI * u - OR_PI;
        st[PHR * n + idx] = p->sigma * cos(theta);
        st[PHI * n + idx] = p->sigma * sin(theta);
    }
}

/* Xi_ij at site y: A_i^y + A_j^{y+i} - A_i^{y+j} - A_j^y, Eq. (3). */
static double plaquette(const or_params *p, const double *st, int x, int y, int z,
                        int i, int j)
{
    size_t n = sites(p);
    const double *Ai = st + (AX + i) * n;
    const double *Aj = st + (AX + j) * n;
    size_t o = nb(p, x, y, z, 0, 0, 0);
    size_t pi = nb(p, x, y, z, UNIT[i][0], UNIT[i][1], UNIT[i][2]);
    size_t pj = nb(p, x, y, z, UNIT[j][0], UNIT[j][1], UNIT[j][2]);
    return Ai[o] + Aj[pi] - Ai[pj] - Aj[o];
}

/*
 * The update of one site, Sec. 2, Eqs. (4)-(7): S_{n+1} at site (x,y,z) from
 * S_n = (phi^n, A^n, Pi^{n-1/2}, E^{n-1/2}).  The ten new values (plane order)
 * go to out10.
 */
static void update_site(const or_params *p, const or_coeffs *c, const double *in, int x, int y,
                        int z, double out10[10])
{
    size_t N = sites(p);
    size_t o = nb(p, x, y, z, 0, 0, 0);
    double pr = in[PHR * N + o], pim = in[PHI * N + o];

    /* Eq. (4): covariant Laplacian
     * sum_j [ e^{iA_j^x} phi^{x+j} - 2 phi^x + e^{-iA_j^{x-j}} phi^{x-j} ] */
    double lr = 0.0, li = 0.0;
    for (int j = 0; j < 3; ++j) {
        const int *u = UNIT[j];
        size_t fp = nb(p, x, y, z, u[0], u[1], u[2]);
        size_t fm = nb(p, x, y, z, -u[0], -u[1], -u[2]);
        double ajp = in[(AX + j) * N + o];
        double ajm = in[(AX + j) * N + fm];
        double qr = in[PHR * N + fp], qi = in[PHI * N + fp];
        double mr = in[PHR * N + fm], mi = in[PHI * N + fm];
        /* e^{i a} (qr + i qi) */
        lr += cos(ajp) * qr - sin(ajp) * qi;
        li += cos(ajp) * qi + sin(ajp) * qr;
        /* e^{-i a} (mr + i mi) */
        lr += cos(ajm) * mr + sin(ajm) * mi;
        li += cos(ajm) * mi - sin(ajm) * mr;
        lr -= 2.0 * pr;
        li -= 2.0 * pim;
    }
    double v = pr * pr + pim * pim - p->sigma * p->sigma;
    double pinr = c->c1 * in[PIR * N + o] + c->c2 * lr - c->c3 * v * pr;
    double pini = c->c1 * in[PII * N + o] + c->c2 * li - c->c3 * v * pim;
    out10[PIR] = pinr;
    out10[PII] = pini;

    /* Eq. (6) */
    out10[PHR] = pr + p->dt * pinr;
    out10[PHI] = pim + p->dt * pini;

    /* Eq. (5), for each link direction i */
    for (int i = 0; i < 3; ++i) {
        const int *u = UNIT[i];
        size_t fp = nb(p, x, y, z, u[0], u[1], u[2]);
        double ai = in[(AX + i) * N + o];
        /* Im[ conj(phi^{x+i}) e^{-i A_i^x} phi^x ] */
        double qr = in[PHR * N + fp], qi = in[PHI * N + fp];
        double wr = cos(ai) * pr + sin(ai) * pim;  /* e^{-ia} phi^x */
        double wi = cos(ai) * pim - sin(ai) * pr;
        double cur = qr * wi - qi * wr;
        /* sum_{j != i} [ sin Xi_ij^x - sin Xi_ij^{x-j} ] */
        double curl = 0.0;
        for (int j = 0; j < 3; ++j) {
            if (j == i)
                continue;
            const int *w = UNIT[j];
            curl += sin(plaquette(p, in, x, y, z, i, j));
            curl -= sin(plaquette(p, in, (x - w[0] + p->nx) % p->nx,
                                  (y - w[1] + p->ny) % p->ny,
                                  (z - w[2] + p->nz) % p->nz, i, j));
        }
        double en = c->d1 * in[(EX + i) * N + o] + c->d3 * cur - c->d2 * curl;
        out10[EX + i] = en;
        /* Eq. (7) */
        out10[AX + i] = ai + p->dt * en;
    }
}

/*
 * One staggered leapfrog step, Sec. 2, Eqs. (4)-(7): from
 * S_n = (phi^n, A^n, Pi^{n-1/2}, E^{n-1/2}) to S_{n+1}.  All right-hand sides
 * read S_n only.
 */
void or_step(const or_params *p, int64_t n, const double *in, double *out)
{
    or_coeffs c;
    size_t N = sites(p);
    or_coefficients(p, n, &c);

#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                double v[10];
                update_site(p, &c, in, x, y, z, v);
                size_t o = nb(p, x, y, z, 0, 0, 0);
                for (int f = 0; f < 10; ++f)
                    out[f * N + o] = v[f];
            }
}

/* S_{n+1} at the listed sites only: out[k*10 + f] is field f at site idx[k]. */
void or_step_sites(const or_params *p, int64_t n, const double *in, int64_t nsites,
                   const int64_t *idx, double *out)
{
    or_coeffs c;
    or_coefficients(p, n, &c);
    for (int64_t k = 0; k < nsites; ++k) {
        int64_t s = idx[k];
        int x = (int)(s % p->nx);
        int y = (int)((s / p->nx) % p->ny);
        int z = (int)(s / ((int64_t)p->nx * p->ny));
        update_site(p, &c, in, x, y, z, out + k * 10);
    }
}

static double wrap_pi(double u)
{
    return u - OR_TWO_PI * floor((u + OR_PI) / OR_TWO_PI);
}

/* accumulators of one z-plane */
enum { S_KIN, S_GRAD, S_ELEC, S_MAG, S_POT, S_LAG,
       S_NUM_L, S_NUM_V, S_NUM_R, S_DEN_L, S_DEN_V, S_DEN_R,
       S_PRES, S_PRES_L, S_RHO_L, S_COUNT };
enum { I_W0, I_W1, I_W2, I_N0, I_N1, I_N2, I_PIERCED, I_NONFIN, I_COUNT };

/*
 * Network diagnostics of S_n, Sec. 2, Eqs. (9)-(11).
 * Per site: K = |Pi|^2, G = dx^-2 sum_i |e^{iA_i} phi^{x+i} - phi^x|^2,
 * EE = dx^-2 sum_i E_i^2, BB = 2 dx^-4 sum_{xy,yz,zx} (1 - cos Xi),
 * V = (|phi|^2 - sigma^2)^2 / 4, and with a = a(tau_n),
 * g = a^(2(1-s)) / (2 e0^2), h = lambda0 a^(2+2s):
 *   L   = a^2 K - a^2 G + g (EE - BB) - h V
 *   rho = a^2 K + a^2 G + g (EE + BB) + h V.
 * <v^2>_X = 2R/(1+R), R = sum K X / sum G X, for X = L, V, rho.
 * Pressure (one third of the trace of the stress tensor, the gauge part
 * radiating with p = rho/3):  p = a^2 K - a^2 G / 3 + g (EE + BB) / 3 - h V;
 * <v^2>_w = (1 + 3 p_L / rho_L) / 2 with p_L / rho_L = sum p L / sum rho L
 * (Eq. (12), Lagrangian-weighted pressure and density).
 * Winding (Eq. (11)): theta = arg phi, Y_i = [theta^{x+i} - theta^x + A_i]_pi
 * - A_i, W_ij = rint((Y_i^x + Y_j^{x+i} - Y_i^{x+j} - Y_j^x) / 2pi).
 */
void or_measure(const or_params *p, int64_t n, const double *st, or_obs *obs,
                int8_t *wmap)
{
    size_t N = sites(p);
    int nz = p->nz;
    double tau = p->tau0 + (double)n * p->dt;
    double a = or_scale_factor(p, tau);
    double a2 = a * a;
    double sn = or_s_of(p, tau);
    double g = pow(a, 2.0 * (1.0 - sn)) / (2.0 * p->e0 * p->e0);
    double h = p->lambda0 * pow(a, 2.0 + 2.0 * sn);
    double idx2 = 1.0 / (p->dx * p->dx);
    double dv = p->dx * p->dx * p->dx;
    double s2 = p->sigma * p->sigma;

    double *theta = malloc(N * sizeof(double));
    double *Y = malloc(3 * N * sizeof(double));
    double *ps = calloc((size_t)nz * S_COUNT, sizeof(double));
    int64_t *pc = calloc((size_t)nz * I_COUNT, sizeof(int64_t));

    for (size_t o = 0; o < N; ++o)
        theta[o] = atan2(st[PHI * N + o], st[PHR * N + o]);

#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                size_t o = nb(p, x, y, z, 0, 0, 0);
                for (int i = 0; i < 3; ++i) {
                    const int *u = UNIT[i];
                    size_t fp = nb(p, x, y, z, u[0], u[1], u[2]);
                    double ai = st[(AX + i) * N + o];
                    Y[i * N + o] = wrap_pi(theta[fp] - theta[o] + ai) - ai;
                }
            }

    /* plaquette orientations (i,j): xy, yz, zx */
    static const int PL[3][2] = { { 0, 1 }, { 1, 2 }, { 2, 0 } };

#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z) {
        double *acc = ps + (size_t)z * S_COUNT;
        int64_t *cnt = pc + (size_t)z * I_COUNT;
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                size_t o = nb(p, x, y, z, 0, 0, 0);
                double pr = st[PHR * N + o], pim = st[PHI * N + o];

                int finite = 1;
                for (int f = 0; f < 10; ++f)
                    if (!isfinite(st[f * N + o]))
                        finite = 0;
                if (!finite)
                    cnt[I_NONFIN] += 1;

                double K = st[PIR * N + o] * st[PIR * N + o]
                         + st[PII * N + o] * st[PII * N + o];
                double G = 0.0, EE = 0.0, BB = 0.0;
                for (int i = 0; i < 3; ++i) {
                    const int *u = UNIT[i];
                    size_t fp = nb(p, x, y, z, u[0], u[1], u[2]);
                    double ai = st[(AX + i) * N + o];
                    double qr = st[PHR * N + fp], qi = st[PHI * N + fp];
                    double dr = cos(ai) * qr - sin(ai) * qi - pr;
                    double di = cos(ai) * qi + sin(ai) * qr - pim;
                    G += dr * dr + di * di;
                    double e = st[(EX + i) * N + o];
                    EE += e * e;
                }
                G *= idx2;
                EE *= idx2;
                for (int k = 0; k < 3; ++k) {
                    int i = PL[k][0], j = PL[k][1];
                    BB += 1.0 - cos(plaquette(p, st, x, y, z, i, j));

                    size_t fi = nb(p, x, y, z, UNIT[i][0], UNIT[i][1], UNIT[i][2]);
                    size_t fj = nb(p, x, y, z, UNIT[j][0], UNIT[j][1], UNIT[j][2]);
                    double loop = Y[i * N + o] + Y[j * N + fi] - Y[i * N + fj]
                                - Y[j * N + o];
                    double w = rint(loop / OR_TWO_PI);
                    int64_t iw = (int64_t)w;
                    cnt[I_W0 + k] += iw;
                    cnt[I_N0 + k] += iw < 0 ? -iw : iw;
                    if (iw != 0)
                        cnt[I_PIERCED] += 1;
                    if (wmap)
                        wmap[(size_t)k * N + o] = (int8_t)iw;
                }
                BB *= 2.0 * idx2 * idx2;
                double vv = pr * pr + pim * pim - s2;
                double V = 0.25 * vv * vv;

                double lag = a2 * K - a2 * G + g * (EE - BB) - h * V;
                double rho = a2 * K + a2 * G + g * (EE + BB) + h * V;
                double pres = a2 * K - a2 * G / 3.0 + g * (EE + BB) / 3.0 - h * V;

                acc[S_KIN] += a2 * K;
                acc[S_GRAD] += a2 * G;
                acc[S_ELEC] += g * EE;
                acc[S_MAG] += g * BB;
                acc[S_POT] += h * V;
                acc[S_LAG] += lag;
                acc[S_NUM_L] += K * lag;
                acc[S_NUM_V] += K * V;
                acc[S_NUM_R] += K * rho;
                acc[S_DEN_L] += G * lag;
                acc[S_DEN_V] += G * V;
                acc[S_DEN_R] += G * rho;
                acc[S_PRES] += pres;
                acc[S_PRES_L] += pres * lag;
                acc[S_RHO_L] += rho * lag;
            }
    }

    double tot[S_COUNT] = { 0 };
    int64_t itot[I_COUNT] = { 0 };
    for (int z = 0; z < nz; ++z) {
        for (int k = 0; k < S_COUNT; ++k)
            tot[k] += ps[(size_t)z * S_COUNT + k];
        for (int k = 0; k < I_COUNT; ++k)
            itot[k] += pc[(size_t)z * I_COUNT + k];
    }

    memset(obs, 0, sizeof(*obs));
    obs->step = n;
    obs->tau = tau;
    obs->a = a;
    for (int k = 0; k < 3; ++k) {
        obs->net_wind_dir[k] = itot[I_W0 + k];
        obs->n_wind_dir[k] = itot[I_N0 + k];
        obs->n_wind += itot[I_N0 + k];
    }
    obs->n_pierced = itot[I_PIERCED];
    obs->nonfinite = itot[I_NONFIN];

    double vbox = (double)N * dv;
    obs->length = (OR_PI / 6.0) * p->dx * (double)obs->n_wind;
    obs->xi_w = sqrt(vbox / obs->length);
    obs->sum_lag = dv * tot[S_LAG];
    obs->xi_l = obs->sum_lag < 0.0
        ? a * sqrt(-(OR_TWO_PI * s2) * vbox / obs->sum_lag) : NAN;
    obs->kin = dv * tot[S_KIN];
    obs->grad = dv * tot[S_GRAD];
    obs->elec = dv * tot[S_ELEC];
    obs->mag = dv * tot[S_MAG];
    obs->pot = dv * tot[S_POT];
    obs->energy = obs->kin + obs->grad + obs->elec + obs->mag + obs->pot;
    obs->pres = dv * tot[S_PRES];
    obs->pres_lag = dv * tot[S_PRES_L];
    obs->rho_lag = dv * tot[S_RHO_L];
    obs->v2_eos = 0.5 * (1.0 + 3.0 * obs->pres_lag / obs->rho_lag);
    for (int k = 0; k < 3; ++k) {
        obs->num[k] = dv * tot[S_NUM_L + k];
        obs->den[k] = dv * tot[S_DEN_L + k];
        double R = obs->num[k] / obs->den[k];
        obs->v2[k] = 2.0 * R / (1.0 + R);
    }

    free(theta);
    free(Y);
    free(ps);
    free(pc);
}

/*
 * Discrete Gauss law of S_n (checked in Sec. 4, not written out there):
 *   G_x = sum_i (E_i^x - E_i^{x-i}) a_-^(2(1-s)) / e0^2
 *       + 2 dx^2 a_-^2 Im(conj(phi^x) Pi^x),
 * a_- = a(tau_{n-1/2}), the time level of the stored momenta.  It is the
 * charge conserved by Eqs. (4)-(7) at every site.
 */
void or_gauss(const or_params *p, int64_t n, const double *st, double *max_abs,
              double *rms, double *gmap)
{
    size_t N = sites(p);
    int nz = p->nz;
    double tau = p->tau0 + (double)n * p->dt;
    double am = or_scale_factor(p, tau - 0.5 * p->dt);
    double fe = pow(am, 2.0 * (1.0 - or_s_of(p, tau - 0.5 * p->dt))) / (p->e0 * p->e0);
    double fp = 2.0 * p->dx * p->dx * am * am;
    double *pmax = calloc((size_t)nz, sizeof(double));
    double *psq = calloc((size_t)nz, sizeof(double));

#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                size_t o = nb(p, x, y, z, 0, 0, 0);
                double div = 0.0;
                for (int i = 0; i < 3; ++i) {
                    const int *u = UNIT[i];
                    size_t fm = nb(p, x, y, z, -u[0], -u[1], -u[2]);
                    div += st[(EX + i) * N + o] - st[(EX + i) * N + fm];
                }
                double charge = st[PHR * N + o] * st[PII * N + o]
                              - st[PHI * N + o] * st[PIR * N + o];
                double G = fe * div + fp * charge;
                if (gmap)
                    gmap[o] = G;
                if (fabs(G) > pmax[z])
                    pmax[z] = fabs(G);
                psq[z] += G * G;
            }

    double m = 0.0, sq = 0.0;
    for (int z = 0; z < nz; ++z) {
        if (pmax[z] > m)
            m = pmax[z];
        sq += psq[z];
    }
    *max_abs = m;
    *rms = sqrt(sq / (double)N);
    free(pmax);
    free(psq);
}

int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
