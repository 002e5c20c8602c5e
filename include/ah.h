/*
 * ah.h -- C ABI of the MI355X (gfx950) Abelian-Higgs lattice library.
 *
 * The library advances a local U(1) Abelian-Higgs field -- complex scalar phi
 * with momentum Pi, link angles A_i with electric fields E_i -- on a periodic
 * comoving 3D lattice in an FRW background with the staggered leapfrog of
 * Correia & Martins, arXiv:1809.00995, Sec. 2, Eqs. (4)-(8), and measures the
 * network diagnostics of Sec. 2, Eqs. (9)-(11): the plaquette winding string
 * length and the weighted mean square velocity.
 *
 * Conventions shared by every entry point
 *  - Return value: AH_OK (0) or a negative ah_status.  ah_error_string()
 *    names a code; ah_last_error() gives the message of the last failure on
 *    a context.  A context is not thread safe: calls on one context must not
 *    overlap.
 *  - Device memory: all field storage is owned by the caller (for instance
 *    one torch tensor per realization) and must outlive the context.  The
 *    library owns only its small scratch (step counters, coefficients,
 *    reduction accumulators), allocated in ah_init and released in ah_free.
 *    The accumulators hold 64 measured states per realization; an ah_step
 *    call that measures more states at once grows them (at least doubling),
 *    the only allocation a step call makes apart from the one-time work
 *    lists and graphs of the batched form (ah_set_launch).
 *  - Streams: every GPU operation of a context is issued on the hipStream_t
 *    given to ah_init (NULL = the default stream).  ah_step is asynchronous
 *    unless it returns observations; ah_measure and ah_gauss_residual
 *    synchronise that stream before returning host values.
 *  - Field layout (struct ah_buffers): 15 planes of nx*ny*nz elements
 *    (nx*ny*(nz + 2 z_halo) for a slab, see "Slabs" below; float for
 *    AH_FP32, double for AH_FP64), contiguous, site index
 *    idx = x + nx*(y + ny*z), in the order
 *      0 phi_re  1 phi_im  2 Pi_re  3 Pi_im  4 A_x  5 A_y  6 A_z
 *      7 E_x     8 E_y     9 E_z   10 phi_re' 11 phi_im' 12 A_x' 13 A_y' 14 A_z'
 *    Planes 10-14 are the second copy of phi and A: each step reads phi, A
 *    from one copy and writes the other, and updates Pi, E in place.  With
 *    layout AH_LAYOUT_20 there are 20 planes: planes 10-19 are a second copy
 *    of all ten fields 0-9, and each pass over memory reads one copy and
 *    writes the other (this is what lets one pass advance two steps, see
 *    AH_KERNEL_TILED2).  ah_current_planes() says which planes hold the
 *    current state.  A state S_n stores phi^n, A^n and the half-step momenta
 *    Pi^{n-1/2}, E^{n-1/2}.  A_i is the raw link angle (never reduced modulo
 *    2 pi).
 */
#ifndef AH_H
#define AH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ah_status {
    AH_OK = 0,
    AH_E_INVALID = -1,    /* bad argument, NULL pointer, bad extents, misaligned buffer */
    AH_E_NOMEM = -2,      /* host or device allocation of library scratch failed       */
    AH_E_HIP = -3,        /* a HIP runtime call failed (message names it)               */
    AH_E_DOMAIN = -4,     /* parameters outside the method's domain (CFL, s, era, a)    */
    AH_E_STATE = -5,      /* call not valid in the context's current state              */
    AH_E_NONFINITE = -6   /* a measurement found non-finite field values                */
} ah_status;

enum { AH_FP64 = 0, AH_FP32 = 1 };

enum {
    AH_INIT_RANDOM_PHASE = 0, /* |phi| = sigma, uniform random phase, all else 0 (Sec. 2) */
    AH_INIT_VACUUM = 1,       /* phi = sigma, all else 0                                   */
    AH_INIT_NONE = 2          /* keep the caller's planes 0-9 as S_{step0} (resume)        */
};

enum {
    AH_KERNEL_AUTO = 0,       /* the library's fastest variant for the shape, precision and
                                 layout (AH_KERNEL_TILED2 with AH_LAYOUT_20)                */
    AH_KERNEL_PLAIN = 1,      /* one thread per site, every neighbour read from memory     */
    AH_KERNEL_TILED = 2,      /* z-streaming tiles with LDS-staged phasors and plaquettes  */
    AH_KERNEL_TILED2 = 3      /* two steps per pass over memory: each block advances its
                                 tile S_n -> S_{n+2}, recomputing S_{n+1} on a one-site
                                 ring around it; needs AH_LAYOUT_20.  A measured state
                                 takes the AH_KERNEL_TILED pass with the fused measurement,
                                 or in FP32, when the next stop is an even number of steps
                                 away, a read-only measuring pass and then pairs; an odd
                                 step left over takes the AH_KERNEL_TILED pass.            */
};

enum {
    AH_LAYOUT_15 = 0,         /* 15 planes: phi, A double-buffered, Pi, E updated in place */
    AH_LAYOUT_20 = 1          /* 20 planes: all ten fields double-buffered                 */
};

/* Problem statement of one realization (Sec. 2 and Sec. 4 of the paper). */
typedef struct ah_params {
    int32_t nx, ny, nz;   /* periodic extents, each >= 4, nx*ny*nz < 2^31; the tiled
                             kernel needs nx a multiple of 64                          */
    int32_t precision;    /* AH_FP64 or AH_FP32: field storage and stencil arithmetic;
                             time bookkeeping and reductions are FP64 in both            */
    double dx, dt;        /* lattice spacing, conformal time step; dt/dx < 1/sqrt(3)     */
    double tau0, tau_ref; /* tau_n = tau0 + n dt; a(tau) = (max(tau,0)/tau_ref)^era_p    */
    double era_p;         /* 0 flat (a = 1), 1 radiation (a ~ tau), 2 matter (a ~ tau^2) */
    double s;             /* -4 <= s <= 1: couplings e0 a^(s-1), lambda0 a^(2(s-1)), Eq. (8);
                             s < 0 grows the comoving core; needs a(tau_step0) > 0     */
    double lambda0, e0, sigma; /* scalar coupling, gauge coupling, vacuum expectation   */
    uint64_t seed;        /* random-phase seed (AH_INIT_RANDOM_PHASE)                   */
    int32_t init;         /* AH_INIT_*                                                  */
    int32_t layout;       /* AH_LAYOUT_15 or AH_LAYOUT_20 (one for all realizations)    */
    int64_t step0;        /* step index n of the initial state (resume from step0)      */
    int64_t n_end;        /* 0: no limit; else the realization stops at S_{n_end} (its
                             tau_end): further steps leave it unchanged                 */
    double s_late, tau_s; /* tau_s > 0: s(tau) = s before tau_s and s_late from tau_s on,
                             e.g. a core-growth period (s < 0) followed by the true
                             equations of motion (s_late = 1), Sec. 2 after Eq. (8);
                             tau_s <= 0: s throughout                                   */
    int32_t z_halo;       /* 0: periodic in z.  1 or 2: the realization is a z-slab of
                             a larger lattice (one GPU's share of a z-decomposed run):
                             see "Slabs" below                                          */
    int32_t reserved;     /* must be 0                                                  */
} ah_params;

/*
 * Slabs (z_halo = H > 0).  Every field plane holds nz + 2H z-planes: planes
 * [0, H) are the halo below the slab, [H, H + nz) the slab, [H + nz, nz + 2H)
 * the halo above (site index x + nx*(y + ny*z) over the stored planes).  Only
 * the slab's planes are advanced and measured (box volume nx*ny*nz dx^3); the
 * halo planes are read, never written.  Before every ah_step and ah_measure
 * call the caller fills all ten fields of the current copy
 * (ah_current_planes) on every halo plane with the neighbouring slabs' planes
 * of the same state: on several GPUs that is the exchange with the z
 * neighbours; a slab closed on itself (halo below = its top planes, halo
 * above = its bottom planes) is a periodic lattice.  ah_step then advances one
 * pass per call: nsteps = 1, or nsteps = 2 when H = 2, the two-step kernel is
 * in use and no measurement is due at the first step.  Requirements: the
 * tiled kernels (nx % 64 == 0), unbatched launches without graphs,
 * AH_INIT_NONE or AH_INIT_VACUUM; ah_gauss_residual and ah_autotune are not
 * available (AH_E_INVALID / AH_E_STATE otherwise).
 */

/* Caller-owned device memory of one realization: 15 or 20 planes (per
 * layout), see above.  Alignment: 256 bytes. */
typedef struct ah_buffers {
    void *planes;
} ah_buffers;

/* Diagnostics of one state S_n (Sec. 2, Eqs. (9)-(11)).  Densities are the
 * conformal densities of S_n as stored, with a = a(tau_n):
 *   L = a^2 K - a^2 G + g (EE - BB) - h V,  rho = a^2 K + a^2 G + g (EE + BB) + h V,
 *   K = |Pi|^2, G = dx^-2 sum_i |e^{iA_i} phi^{x+i} - phi^x|^2, EE = dx^-2 sum_i E_i^2,
 *   BB = 2 dx^-4 sum_{xy,yz,zx} (1 - cos Xi), V = (|phi|^2 - sigma^2)^2 / 4,
 *   g = a^(2(1-s)) / (2 e0^2), h = lambda0 a^(2+2s). */
typedef struct ah_obs {
    int64_t step;
    double tau, a;
    int64_t n_wind;          /* sum over plaquettes of |W|, Eq. (11)                  */
    int64_t n_wind_dir[3];   /* per orientation xy, yz, zx                             */
    int64_t net_wind_dir[3]; /* signed sums per orientation (zero on a periodic box)  */
    int64_t n_pierced;       /* plaquettes with W != 0                                */
    double length, xi_w;     /* (pi/6) dx n_wind ; sqrt(V_box / length)               */
    double sum_lag, xi_l;    /* dx^3 sum L ; a sqrt(-2 pi sigma^2 V_box / sum_lag), Eq. (9) */
    double num[3], den[3];   /* dx^3 sum K X, dx^3 sum G X for X = L, V, rho          */
    double v2[3];            /* <v^2>_X = 2R/(1+R), R = num/den, Eqs. (9)-(10)        */
    double kin, grad, elec, mag, pot, energy; /* dx^3 sums of the parts of rho      */
    double pres;             /* dx^3 sum p, p = a^2 K - a^2 G/3 + g (EE + BB)/3 - h V */
    double pres_lag, rho_lag;/* dx^3 sum p L, dx^3 sum rho L                          */
    double v2_eos;           /* <v^2>_w = (1 + 3 pres_lag / rho_lag) / 2, Eq. (12)   */
    int64_t nonfinite;       /* sites holding a non-finite field value               */
} ah_obs;

typedef struct ah_ctx ah_ctx;

/* Text for a status code (static storage). */
const char *ah_error_string(int code);

/* Message of the last failed call on ctx (valid until the next call). */
const char *ah_last_error(const ah_ctx *ctx);

/*
 * Create a context for n_real >= 1 independent realizations.  p[r] and buf[r]
 * describe realization r; all realizations share one precision.  Validates
 * the parameters (extents, alignment, CFL dt/dx < 1/sqrt(3), -4 <= s, s_late
 * <= 1, era_p >= 0, tau_ref > 0, a(tau_{step0 + 1/2}) > 0, and a(tau_step0)
 * > 0 when some s < 0), allocates the scratch,
 * then writes the initial state on the stream: the random-phase initial
 * condition of Sec. 2 (theta = 2 pi u - pi, u from SplitMix64 output number
 * idx+1 of generator p[r].seed), the vacuum, or nothing (AH_INIT_NONE: the
 * caller's planes 0-9 hold S_{step0}).  On failure *ctx is NULL and nothing
 * is allocated.  hip_stream is a hipStream_t or NULL.
 */
int ah_init(ah_ctx **ctx, int32_t n_real, const ah_params *p, const ah_buffers *buf,
            void *hip_stream);

/*
 * Advance every realization by nsteps (>= 0) leapfrog steps, Eqs. (4)-(7):
 * S_n -> S_{n+1} (a realization that has reached its n_end stays there).
 * With measure_every = k > 0, every state S_n with n % k == 0 met before its
 * update is measured (as ah_measure would), and the observations are written
 * to out[j * n_real + r] for the j-th step of the call that measured; slots
 * of realizations that did not measure at that step have step = -1.
 * *n_out receives the number of slots written per realization.
 * out_cap is the capacity of out in states per realization; the call fails
 * with AH_E_INVALID, before any work, if it is too small.  With out == NULL
 * (and measure_every = 0) the call only enqueues work and returns at once.
 * Returns AH_E_NONFINITE if a measurement saw non-finite values.  A context
 * holding slabs (z_halo > 0) advances one pass per call, see "Slabs".
 */
int ah_step(ah_ctx *ctx, int64_t nsteps, int32_t measure_every, ah_obs *out,
            int64_t out_cap, int64_t *n_out);

/*
 * Measure the current state S_n of every realization into out[r] (host
 * array of n_real).  wind_dev, if not NULL, is a device array that receives,
 * per realization, 3 int8 planes (xy, yz, zx plaquette at site x) of W,
 * realizations back to back.  Synchronises the stream.
 */
int ah_measure(ah_ctx *ctx, ah_obs *out, int8_t *wind_dev);

/* Most states one ah_measure_noalloc call measures: the capacity of the
 * library's static device scratch (a descriptor, the coefficients and one
 * slot of sums per state: 36 KB per GPU). */
#define AH_NOALLOC_MAX_REAL 64

/*
 * ah_measure without a context and without allocating anything, for callers
 * that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Measures, with the kernels
 * ah_measure uses and the diagnostics it returns (Sec. 2, Eqs. (9)-(12)), the
 * state S_n with n = p[r].step0 held in planes 0-9 of buf[r] (the first copy;
 * ah_current_planes says whether a context's current state is there), for
 * 1 <= n_real <= AH_NOALLOC_MAX_REAL realizations described as for ah_init
 * and validated the same way (init, seed and n_end are not used).
 *  - out_dev: device array of n_real ah_obs, written on the stream;
 *    wind_dev: NULL or a device array as for ah_measure.
 *  - Every operation is issued on hip_stream (a hipStream_t or NULL) and the
 *    call returns without waiting: out_dev holds the results once the stream
 *    has passed this point.  Non-finite sites are counted in
 *    out_dev[r].nonfinite (the call cannot see them, so it does not return
 *    AH_E_NONFINITE).
 *  - Scratch: the library's static device array (one per GPU, held until the
 *    process ends).  Its address is looked up, with the device current, by
 *    the first ah_init or ah_measure_noalloc call on that device: make one such
 *    call before capturing a graph.  Each call clears the part it uses, and
 *    the array keeps the last call's contents, so calls that overlap on one GPU
 *    (other streams, other host threads) race and must be ordered by the
 *    caller.
 *  - Errors (AH_E_INVALID for n_real outside [1, AH_NOALLOC_MAX_REAL] or a
 *    bad realization, AH_E_DOMAIN, AH_E_HIP) are returned before any device
 *    work except a failed launch; ah_last_error(NULL) gives the message.
 */
int ah_measure_noalloc(int32_t n_real, const ah_params *p, const ah_buffers *buf,
                       ah_obs *out_dev, int8_t *wind_dev, void *hip_stream);

/*
 * Gauss-law residual of the current state (discrete Noether charge of the
 * lattice action under time-independent gauge transformations, conserved by
 * Eqs. (4)-(7); checked in Sec. 4):
 *   G_x = sum_i (E_i^x - E_i^{x-i}) a_-^(2(1-s)) / e0^2 + 2 dx^2 a_-^2 Im(conj(phi^x) Pi^x),
 * a_- = a(tau_{n-1/2}).  max_abs[r], rms[r]: host arrays of n_real.
 * Synchronises the stream.
 */
int ah_gauss_residual(ah_ctx *ctx, double *max_abs, double *rms);

/* Plane index (0-14, or 0-19 with AH_LAYOUT_20) of each of the 10 fields
 * phi_re, phi_im, Pi_re, Pi_im, A_x, A_y, A_z, E_x, E_y, E_z of realization r
 * in the current state. */
int ah_current_planes(const ah_ctx *ctx, int32_t r, int32_t plane_of_field[10]);

/* Step index n of the current state of realization r. */
int ah_current_step(const ah_ctx *ctx, int32_t r, int64_t *n);

/*
 * Select the step-kernel variant (AH_KERNEL_*) and, for the tiled kernels, the
 * tile: tile_y rows of 64 sites per block and chunk_z planes per block along
 * z (>= 1); 0 picks the library default.  tile_y: AH_KERNEL_TILED 2, 4, 8, or
 * 16 for FP32; AH_KERNEL_TILED2 4, 8 or 9 for FP32, 4 or 5 for FP64 (its
 * measuring and odd steps keep the AH_KERNEL_TILED defaults, except that in the
 * batched form they walk the two-step kernel's z-chunks).  The tiled kernels need
 * nx % 64 == 0 in every realization, AH_KERNEL_TILED2 also AH_LAYOUT_20
 * (AH_E_INVALID otherwise).  Results do not depend on the choice beyond
 * floating-point rounding of the same formulas; the tiled variants of one
 * precision, AH_KERNEL_TILED2 included, agree bit for bit.
 */
int ah_set_kernel(ah_ctx *ctx, int32_t kernel, int32_t tile_y, int32_t chunk_z);

/*
 * Launch strategy.  batched = 1: every step of all realizations is one
 * launch of a persistent kernel that walks a work list of (realization,
 * tile, z-chunk) items -- the ensemble form for many independent
 * realizations of uneven size (Sec. 1 and Sec. 5 of the paper motivate
 * thousands of runs); it needs nx % 64 == 0 and one common step0, and falls
 * back to one launch per realization otherwise.  Where the two-step kernel is
 * in use, unmeasured pairs are likewise one persistent launch per pair.  graph_steps = g > 0: runs
 * of g unmeasured steps are captured once into a hipGraph (on a stream of
 * the context, ordered after and before the caller's stream with events) and
 * replayed; measuring steps are launched directly.  0, 0 is the default.
 * Results are bit-identical to the default launch.
 */
int ah_set_launch(ah_ctx *ctx, int32_t batched, int32_t graph_steps);

/*
 * Autotuner: times the tiled step kernel (AH_KERNEL_TILED2 when that is the
 * selected or automatic choice, else AH_KERNEL_TILED) for candidate tile
 * heights and z-chunks on a scratch lattice of each distinct shape of the
 * context (the caller's fields are not touched), installs the tile height with
 * the least estimated total time per step and the best z-chunk for each
 * realization, and returns them in *tile_y and chunk_z[n_real] (either may be
 * NULL).  It tunes for the launch form in force, so call ah_set_launch first:
 * with one launch per realization the scratch lattice is the shape itself
 * (nx*ny*min(nz,128), up to 20 planes); in the batched form it is a lattice of
 * the same nx, ny, tall enough that every candidate chunk fills the chip (up
 * to about 2^26 sites, 20 planes; the shape itself if that allocation fails).
 * The scratch is freed before returning.  Needs the tiled kernel (AH_E_STATE
 * otherwise).  Synchronises the stream.
 */
int ah_autotune(ah_ctx *ctx, int32_t *tile_y, int32_t *chunk_z);

/* Release the context's scratch (not the caller's planes).  NULL is a no-op. */
int ah_free(ah_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* AH_H */
