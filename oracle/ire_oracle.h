/*
 * Serial FP64 reference ("the oracle") of the immediate re-emission (IRE)
 * Monte Carlo dust radiative-transfer method for spherically symmetric clouds,
 * as described in Juvela (2024), "DIES: Parallel dust radiative transfer
 * program with the immediate re-emission method", Sect. 2.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the GPU path.
 *
 * Units are cgs throughout: cm, g cm^-3, Hz, cm^2 g^-1, erg s^-1 cm^-2 Hz^-1
 * sr^-1 for the external mean intensity J_nu, erg s^-1 for luminosities, K.
 *
 * Parity status: every function here is pinned by tests that do not reuse
 * its own formulas (closed forms, importance-sampling identities, brute-force
 * deterministic solutions, published Philox known-answer vectors); the
 * paper's own printed temperature profiles cannot be used (their input
 * datasets are not available), so that particular comparison is
 * "parity unpinned".
 */
#ifndef IRE_ORACLE_H
#define IRE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct or_model {
    int32_t n;              /* number of shells */
    const double *r_edges;  /* n+1 radii, strictly increasing, r_edges[0] >= 0 (empty cavity if > 0) */
    const double *rho;      /* n densities */
    int32_t K;              /* number of frequencies */
    const double *nu;       /* K, strictly increasing */
    const double *kabs;     /* K absorption opacity per mass */
    const double *albedo;   /* K, in [0,1) */
    const double *g;        /* K, Henyey-Greenstein asymmetry parameter */
    double t_min, t_max;    /* temperature table range */
    int32_t n_t;            /* temperature table points (log spaced) */
    const double *J;        /* K external isotropic mean intensity, or NULL */
    double L_ps;            /* central point-source luminosity (0 = none) */
    const double *S;        /* K point-source spectrum shape (any normalisation), or NULL */
} or_model;

typedef struct or_options {
    double k_bg;            /* centre weighting of background directions, Eq. 5; 0.5 = unweighted */
    int32_t ffi;            /* forced first interaction, Eqs. 9-12: 0 off, 1 in extinction optical depth,
                               2 in absorption optical depth (the stronger variant named after Eq. 12) */
    double w_floor;         /* terminate when W < w_floor * (launch weight) */
    uint64_t max_events;    /* terminate a package that would start event max_events+1 */
    int32_t table_mode;     /* 0: exact T inversion + exact difference spectra; 1: lookup tables */
    int32_t acc_bits;       /* 0: FP64 accumulators; >0: emulate a float with this many significand bits */
    int32_t n_batches;      /* with acc_bits: the two-counter batch scheme of Sect. 2.3 (1 = one counter) */
    int32_t reemit_uniform; /* re-emit at a uniformly random position in the shell volume (Sect. 4) */
    /* Sect. 2.2, Table 1: weighted sampling of directions and free paths */
    int32_t use_g_E;        /* re-emission directions from HG(g_E) about the reference direction (Eq. 6) */
    double g_E;
    int32_t use_g_S;        /* scattering directions from HG(g_S) about the reference direction (Eq. 7) */
    double g_S;
    double k_A, k_S;        /* free paths from k e^{-k tau} (Eq. 8); 1 = unweighted */
    int32_t k_A_rho;        /* absorption scaling linear in log rho (Sect. 3.2): k_A_lowest at the
                               lowest density of the model, k_A_highest at the highest (k_A must be 1) */
    double k_A_lowest, k_A_highest;
} or_options;

typedef struct or_stats {
    double L_ext, L_ps;     /* source luminosities */
    double escaped[2];      /* escaped power per source (external, point) */
    double ffi_escaped;     /* power of the unforced fraction exp(-tau0) under FFI */
    double terminated;      /* power of packages stopped by the weight floor or max_events */
    uint64_t n_launch, n_cross, n_scat, n_abs, n_escape, n_direct, n_limit, n_floor;
    uint64_t n_below, n_above;      /* final temperatures clamped to the table range */
    uint64_t n_reemit_above;        /* table mode: re-emission draws above the last table point */
    double terminated_floor;        /* the part of `terminated` stopped by the weight floor */
} or_stats;

void or_default_options(or_options *o);

/* Run n_ext external and n_ps point-source packages with the given seed.
 * A, T: n outputs (absorbed power, temperature).  reemit (n*K), first_abs (n),
 * sed (2*K: escaped power per source and frequency, the unforced FFI fraction
 * included) and sed_direct (2*K: the part that escaped without any event) are
 * optional tallies (NULL to skip).  Returns 0 or a negative error code for
 * invalid input. */
int or_run(const or_model *m, const or_options *o, uint64_t n_ext, uint64_t n_ps,
           uint64_t seed, double *A, double *T, or_stats *st, double *reemit,
           double *first_abs, double *sed, double *sed_direct);

/* Philox4x32-10 (Salmon et al. 2011): out = bijection(ctr) under key. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Planck function B_nu(T) in erg s^-1 cm^-2 Hz^-1 sr^-1. */
double or_planck(double nu, double T);

/* Tables as the oracle builds them (for tests).  Any pointer may be NULL.
 * w: K quadrature weights; G: n_t emitted power per mass on the T grid;
 * D: n_t*K re-emission CDF rows; cdf_ext, cdf_ps: K; mass: n; L: [L_ext, L_ps]. */
int or_tables(const or_model *m, double *w, double *G, double *D, double *cdf_ext,
              double *cdf_ps, double *mass, double *L);

/* Temperature for an absorbed power per mass a: exact inversion (table_mode 0)
 * or log-log table interpolation (table_mode 1); no clamping. */
double or_temperature(const or_model *m, double a, int32_t table_mode);

/* Evaluate one of the oracle's samplers on arrays of uniforms (for tests).
 * which: 0 external launch cosine (param k_bg) -> out mu, w weight;
 *        1 Henyey-Greenstein cos(theta) (param g);  2 free path -ln u;
 *        3 forced first interaction (param tau0) -> out tau, w weight;
 *        4 isotropic direction cosine. */
int or_eval_sampler(int32_t which, double param, int64_t n, const double *u, double *out,
                    double *w);

/* The oracle's scattering rotation (for tests): d is rotated in place by the
 * angle acos(ct) at azimuth ph measured from the plane of d and x. */
int or_scatter_direction(const double x[3], double d[3], double ct, double ph);

/* Weighted samplers (for tests).  Reference direction: towards the centre
 * for packages of the external field (src 0), away from it for the point
 * source (src 1).
 * or_reemit_weighted: new direction cosine mu' about the reference drawn from
 *   HG(g_E) with uniform u; returns the radial direction cosine, *W the weight.
 * or_scatter_weighted: d (unit, at position x) is replaced by a direction whose
 *   cosine about the reference is drawn from HG(g_S) (u0) at azimuth 2 pi u1
 *   from the plane of d and x; *cos_theta = cosine between the old and new
 *   directions, *W = HG(cos_theta; g) / HG(mu'; g_S).
 * or_ffi_absorption: interaction point of the forced first flight in units of
 *   absorption depth (tau0 = extinction depth of the ray, albedo a): returns
 *   the extinction depth of the point, *W its weight. */
double or_reemit_weighted(double g_E, int32_t src, double u, double *W);
int or_scatter_weighted(const double x[3], double d[3], double g, double g_S, int32_t src, double u0,
                        double u1, double *cos_theta, double *W);
double or_ffi_absorption(double tau0, double albedo, double u, double *W);

#ifdef __cplusplus
}
#endif
#endif
