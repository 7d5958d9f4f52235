/*
 * libire: immediate re-emission (IRE) Monte Carlo dust radiative transfer in
 * spherically symmetric clouds, on AMD Instinct MI355X (gfx950).
 *
 * The problem follows Juvela (2024), "DIES: Parallel dust radiative transfer
 * program with the immediate re-emission method", Sect. 2: a cloud of
 * concentric shells with given densities (Sect. 2.1), dust with absorption
 * and scattering opacities and a Henyey-Greenstein phase function (Eq. 4 and
 * Sect. 2.2.1), an external isotropic radiation field and/or a central point
 * source whose power is split over N photon packages per source (Sect. 2.1);
 * the result is the absorbed power and the equilibrium temperature of every
 * shell (Sect. 2.1).  Weighting options: centre-weighted background
 * directions (Eq. 5), forced first interaction (Eqs. 9-12), weight floor
 * (Sect. 2.2.1).
 *
 * Units (cgs): cm, g cm^-3, Hz, cm^2 g^-1, erg s^-1 cm^-2 Hz^-1 sr^-1 for the
 * external mean intensity J_nu, erg s^-1 for luminosities, K.
 *
 * Conventions for every entry point:
 *  - return 0 (IRE_OK) or a negative IRE_E_* code; no exception crosses the ABI;
 *    ire_last_error() describes the last failure of a handle;
 *  - arguments are validated before any device work is queued;
 *  - host input arrays are copied during the call; the caller keeps ownership;
 *  - output arrays are allocated by the caller;
 *  - a handle is used by one host thread at a time; separate handles are
 *    independent; `hip_stream` arguments may be NULL (the null stream).
 */
#ifndef IRE_H
#define IRE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IRE_OK 0
#define IRE_E_INVALID (-1)   /* bad argument (NaN, non-monotone radii, albedo >= 1, ...) */
#define IRE_E_STATE (-2)     /* call out of order (run before shells/dust/source are set) */
#define IRE_E_NOMEM (-3)     /* host or device allocation failed */
#define IRE_E_DEVICE (-4)    /* HIP runtime error */
#define IRE_E_LIMIT (-5)     /* some package reached max_events (counted in ire_stats.n_limit) */

#define IRE_FP32 0           /* FP32 path stepping, tables in LDS, FP64 accumulators */
#define IRE_FP64 1           /* FP64 everywhere, tables in global memory */

typedef struct ire_model ire_model;

typedef struct ire_options {
    double k_bg;          /* Eq. 5: background directions mu = u^k_bg with weight 2 k mu^(2-1/k); 0.5 = off */
    int32_t ffi;          /* Eqs. 9-12: force the first flight from the source to interact (0/1) */
    double w_floor;       /* Sect. 2.2.1: stop a package whose weight fell below w_floor * launch weight (1e-10) */
    uint64_t max_events;  /* stop a package that would start event max_events+1 (scatterings + absorptions) */
    int32_t stepping;     /* IRE_FP32 or IRE_FP64 */
    int32_t max_lanes;    /* 0: fill the device; n > 0: at most n packages in flight (1 = serial order) */
    int32_t reemit_uniform; /* Sect. 4: re-emit at a uniformly random point of the shell volume (0/1) */
    int32_t aggregate;    /* 1: wave-level reduction of absorbed energy before the global atomic; 0: one atomic per lane */
    int32_t batch;        /* lanes of a wave parked at an event before their events are processed together
                             (1..64; 0 = default 24); changes speed, not the distribution of results */
} ire_options;

typedef struct ire_stats {
    double L_ext, L_ps;        /* source luminosities of the run (erg/s) */
    double escaped[2];         /* escaped power per source: [external, point] */
    double ffi_escaped;        /* unforced fraction exp(-tau0) of FFI packages */
    double terminated;         /* power of packages stopped by the weight floor or max_events */
    uint64_t n_launch, n_cross, n_scat, n_abs, n_escape, n_direct, n_limit, n_floor;
    uint64_t n_below, n_above; /* final temperatures clamped to [t_min, t_max] */
    uint64_t n_reemit_above;   /* re-emission draws above the last temperature table point */
    float ms_tables, ms_trace, ms_finalize; /* host table build, tracing kernel, finalize kernel */
} ire_stats;

/* Fill *o with the defaults: k_bg 0.5, ffi 0, w_floor 1e-10, max_events 1e6,
 * stepping IRE_FP32, max_lanes 0, reemit_uniform 0, aggregate 1, batch 0. */
int ire_default_options(ire_options *o);

/* Create a handle bound to HIP device `hip_device`; *out is owned by the caller
 * and released with ire_destroy (NULL-safe). */
int ire_create(int hip_device, ire_model **out);
void ire_destroy(ire_model *m);

/* Sect. 2.1 (cells are concentric shells): n shells, r_edges[n+1] strictly
 * increasing with r_edges[0] >= 0 (r_edges[0] > 0 is an empty central cavity),
 * rho[n] >= 0 densities. */
int ire_set_shells(ire_model *m, int32_t n, const double *r_edges, const double *rho);

/* Eq. 4: K frequencies nu[K] strictly increasing; kappa_abs[K] > 0 absorption
 * opacity per mass; albedo[K] in [0,1) (kappa_sca = kappa_abs a / (1-a));
 * g[K] in (-1,1) Henyey-Greenstein asymmetry parameter. */
int ire_set_dust(ire_model *m, int32_t K, const double *nu, const double *kappa_abs,
                 const double *albedo, const double *g);

/* Sect. 2.1 (temperature lookup table): n_t log-spaced points over
 * [t_min, t_max]; defaults 3 K, 1600 K, 512. */
int ire_set_temperature_grid(ire_model *m, double t_min, double t_max, int32_t n_t);

/* Sect. 2.1: external isotropic field, J_nu[K] >= 0 mean intensity on the dust
 * grid; NULL clears it.  Luminosity entering the cloud: 4 pi R^2 * pi * sum J w. */
int ire_set_external_field(ire_model *m, const double *J_nu);

/* Sect. 2.1: central point source of luminosity L > 0 with spectrum shape
 * spectrum[K] >= 0 (any normalisation); L = 0 clears it. */
int ire_set_point_source(ire_model *m, double L, const double *spectrum);

int ire_set_options(ire_model *m, const ire_options *o);

/* Sect. 2.1: trace n_ext external and n_ps point-source packages from seed
 * `seed`, starting from zero absorbed energy.  Asynchronous on hip_stream.
 * Equivalent to ire_begin + ire_advance(n_ext, n_ps). */
int ire_run(ire_model *m, uint64_t n_ext, uint64_t n_ps, uint64_t seed, void *hip_stream);

/* Chunked runs: ire_begin zeroes the accumulators and fixes the package
 * energy L/N_total per source; each ire_advance traces the next packages of
 * each source (package ids continue, so the random streams of a chunked run
 * equal those of one run).  Asynchronous on hip_stream. */
int ire_begin(ire_model *m, uint64_t n_ext_total, uint64_t n_ps_total, uint64_t seed);
int ire_advance(ire_model *m, uint64_t n_ext, uint64_t n_ps, void *hip_stream);

/* Zero the accumulators and counters of the current run. */
int ire_reset(ire_model *m);

/* Wait for queued work of this handle. */
int ire_sync(ire_model *m);

/* Synchronise and copy results: absorbed[n] (erg/s) and T[n] (K) host arrays
 * (either may be NULL); stats may be NULL.  Returns IRE_E_LIMIT if any package
 * reached max_events (results are still written). */
int ire_get_results(ire_model *m, double *absorbed, double *T, ire_stats *stats);

/* Synchronise and return the statistics of the current run (event counts,
 * tallies, kernel times) without finalizing or copying shell results; the
 * clamp counters n_below/n_above are those of the last finalize. */
int ire_get_stats(ire_model *m, ire_stats *stats);

/* Device-pointer variant: writes absorbed[n] and T[n] into caller device
 * memory on hip_stream (kept alive by the caller until the work completes). */
int ire_get_results_dev(ire_model *m, double *absorbed_dev, double *T_dev, void *hip_stream);

/* Human-readable description of the last failure on m (owned by m). */
const char *ire_last_error(const ire_model *m);

/* Planck function B_nu(T) on nu[K] into out[K] (host helper). */
int ire_planck(int32_t K, const double *nu, double T, double *out);

#ifdef __cplusplus
}
#endif
#endif
