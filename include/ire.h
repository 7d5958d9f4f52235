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
    int32_t ffi;          /* Eqs. 9-12: force the first flight from the source to interact: 0 off,
                             1 in extinction optical depth, 2 in absorption optical depth */
    double w_floor;       /* Sect. 2.2.1: stop a package whose weight fell below w_floor * launch weight (1e-10) */
    uint64_t max_events;  /* stop a package that would start event max_events+1 (scatterings + absorptions) */
    int32_t stepping;     /* IRE_FP32 or IRE_FP64 */
    int32_t max_lanes;    /* 0: fill the device; n > 0: at most n packages in flight (1 = serial order) */
    int32_t reemit_uniform; /* Sect. 4: re-emit at a uniformly random point of the shell volume (0/1) */
    int32_t aggregate;    /* how the absorptions of a pass are folded before the returning global atomics:
                             0: one atomic per lane; 1: per wave, by shell; 2: per workgroup, by shell (the
                             workgroup's waves then run their event passes together; fewer than 2^22 shells);
                             -1 (default): 2 with replicas = 1, 1 otherwise */
    int32_t batch;        /* lanes of a wave parked at an event before their events are processed together
                             (1..64, at most the wave's lanes with packages; 0 = default: 48 with aggregate 2
                             (56 with ffi), else 64 with replicas = 1 and 40 otherwise); changes speed, not
                             the distribution of results */
    /* Sect. 2.2, Table 1: weighted sampling.  Reference direction: towards the
     * centre for packages of the external field, outwards for the point source. */
    int32_t use_g_E;      /* Eq. 6: re-emission cosine about the reference direction from HG(g_E), g_E in (-1,1) */
    double g_E;
    int32_t use_g_S;      /* Eq. 7: scattering cosine about the reference direction from HG(g_S), weight =
                             dust HG density at the scattering angle / HG(g_S) density */
    double g_S;
    double k_A, k_S;      /* Eq. 8: free paths from k e^{-k tau} (> 0; 1 = unweighted); the weight of a flight
                             is the fired clock's (1/k) e^{(k-1) tau} times the other's e^{(k'-1) tau'} */
    int32_t k_A_rho;      /* Sect. 3.2: absorption scaling linear in log rho, k_A_lowest at the model's lowest
                             density, k_A_highest at its highest (k_A must be 1); the weight is the fired
                             clock's 1/k times e^{modified - true absorption depth} */
    double k_A_lowest, k_A_highest;
    int32_t replicas;     /* 1 (default): one running total of absorbed energy per shell for the whole device,
                             as the single set of absorption counters of Sect. 2.3.  R = 2..8: the workgroups
                             form R groups, each an independent IRE run over its share of the packages with
                             its own accumulators (temperatures and re-emission slices from R times its own
                             running total); the results are the sum over the groups.  This spreads the
                             returning atomics over R addresses per shell (R = 8: about one group per XCD);
                             it estimates the temperatures as the mean of R runs of N/R packages does, with
                             the low-N bias of runs of N/R packages in the innermost cells (Sect. 3.1 finds
                             ~1e8 packages per run enough for ~1 % in every cell).  Needs max_lanes = 0. */
    int32_t quorum;       /* aggregate = 2 only: once this many of a workgroup's waves have ended their
                             crossing sweeps at `batch` parked lanes, the others end theirs early and the
                             workgroup runs its event pass; with `quorum` or fewer waves left with packages
                             each wave sweeps to its own batch (1..16; 16: every wave always does; 0 = default:
                             2, 3 with ffi); changes speed, not the distribution of results */
} ire_options;

typedef struct ire_stats {
    double L_ext, L_ps;        /* source luminosities of the run (erg/s) */
    double escaped[2];         /* escaped power per source: [external, point] */
    double ffi_escaped;        /* unforced fraction exp(-tau0) of FFI packages */
    double terminated;         /* power of packages stopped by the weight floor or max_events */
    uint64_t n_launch, n_cross, n_scat, n_abs, n_escape, n_direct, n_limit, n_floor;
    uint64_t n_below, n_above; /* final temperatures clamped to [t_min, t_max] */
    uint64_t n_reemit_above;   /* re-emission draws above the last temperature table point */
    uint64_t n_pass;           /* event passes of the tracer's waves (each handles the interactions,
                                  escapes and launches of the wave's parked lanes together) */
    uint64_t n_step_slots;     /* lane slots of the crossing sweeps (64 per wave-level step); n_cross /
                                  n_step_slots is the share of them that moved a package */
    float ms_tables, ms_trace, ms_finalize; /* host table build, tracing kernel, finalize kernel */
} ire_stats;

/* Fill *o with the defaults: k_bg 0.5, ffi 0, w_floor 1e-10, max_events 1e6,
 * stepping IRE_FP32, max_lanes 0, reemit_uniform 0, aggregate -1, batch 0,
 * use_g_E 0, g_E 0, use_g_S 0, g_S 0, k_A 1, k_S 1, k_A_rho 0, k_A_lowest 3, k_A_highest 1, replicas 1,
 * quorum 0. */
int ire_default_options(ire_options *o);

/* Create a handle bound to HIP device `hip_device`; *out is owned by the caller
 * and released with ire_destroy (NULL-safe). */
int ire_create(int hip_device, ire_model **out);
void ire_destroy(ire_model *m);

/* Sect. 2.1 (cells are concentric shells): n shells, r_edges[n+1] strictly
 * increasing with r_edges[0] >= 0 (r_edges[0] > 0 is an empty central cavity),
 * rho[n] >= 0 densities. */
int ire_set_shells(ire_model *m, int32_t n, const double *r_edges, const double *rho);

/* Eq. 4: K (1..255) frequencies nu[K] strictly increasing; kappa_abs[K] > 0 absorption
 * opacity per mass; albedo[K] in [0,1) (kappa_sca = kappa_abs a / (1-a));
 * g[K] in (-1,1) Henyey-Greenstein asymmetry parameter. */
int ire_set_dust(ire_model *m, int32_t K, const double *nu, const double *kappa_abs,
                 const double *albedo, const double *g);

/* Sect. 2.1 (temperature lookup table): n_t (2..65535) log-spaced points over
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

/* Pick the event-pass schedule for this model: time one launch of a sample of
 * the run (at most 2e7 packages in all, split as n_ext : n_ps) for every candidate
 * (with workgroup grouping in FP32: quorum 2, 3, 4, 6 x parked lanes 36, 40,
 * 44, 48, 52; otherwise parked lanes 24, 32, 40, 48, 64), after one untimed launch, and
 * set the fastest in the handle's options (the other options are kept).
 * Schedules change speed, not the distribution of results.  *quorum and *batch
 * (either may be NULL) receive the choice; the tuning runs synchronously on
 * the null stream and leaves no run begun (call ire_run next).  IRE_E_INVALID
 * for n_ext + n_ps = 0 or max_lanes > 0. */
int ire_tune_schedule(ire_model *m, uint64_t n_ext, uint64_t n_ps, int32_t *quorum, int32_t *batch);

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

/* Escaping spectrum of the current run (synchronises): escaped power per
 * source and frequency, sed[2][K] (external, then point source; the unforced
 * fraction of FFI packages included at their launch frequency), and the part
 * that left without any scattering or absorption, sed_direct[2][K].  Either
 * pointer may be NULL.  With both sources, which source's packages carry the
 * re-emitted light depends on the order of the absorptions (packages of both
 * sources run at once); the sum over sources and the unscattered parts do not. */
int ire_get_sed(ire_model *m, double *sed, double *sed_direct);

/* Device-pointer variant: writes absorbed[n] and T[n] into caller device
 * memory on hip_stream (kept alive by the caller until the work completes). */
int ire_get_results_dev(ire_model *m, double *absorbed_dev, double *T_dev, void *hip_stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc.  Equivalent to
 * ire_run(m, n_ext, n_ps, seed) followed by ire_get_results_dev(absorbed_dev,
 * T_dev): a complete run of the handle's current model and options from zero
 * absorbed energy, asynchronous on hip_stream, writing absorbed[n] (erg/s) and
 * T[n] (K) into caller device memory (kept alive by the caller until the work
 * completes).  It calls no hipMalloc, hipFree or other allocating routine: the
 * run's accumulators, event counters, tallies, package cursor and escaping
 * spectrum live in a fixed array inside the library, one per GPU (about 520 KB,
 * held until the process ends), cleared by a fill kernel at the start of every
 * call.  Limits: shells x accumulator groups (options.replicas) <= 4096 and
 * K <= 255 (IRE_E_INVALID beyond).  The model's tables must already be on the
 * device: call ire_run or ire_begin once after the last setter (IRE_E_STATE
 * otherwise).  The handle's own run, statistics and results are not touched;
 * event counts of this call are not returned.  Every call on one GPU shares
 * that GPU's array, so calls that overlap on one GPU (on different streams,
 * from different threads, or with different handles) race and must be
 * serialised by the caller. */
int ire_run_noalloc(ire_model *m, uint64_t n_ext, uint64_t n_ps, uint64_t seed, double *absorbed_dev,
                    double *T_dev, void *hip_stream);

/* Human-readable description of the last failure on m (owned by m). */
const char *ire_last_error(const ire_model *m);

/* Planck function B_nu(T) on nu[K] into out[K] (host helper). */
int ire_planck(int32_t K, const double *nu, double T, double *out);

/* ------------------------------------------------------------------------
 * Batched parameter studies: many cloud models in one persistent launch.
 * The models share the dust, the temperature grid and the source spectral
 * shapes; each has its own shells, source type and strength, package budget
 * and seed.  The method per model is the one above (Sect. 2.1-2.2); batching
 * is a scheduling device for the parameter studies the paper has in view
 * (Abstract, Sect. 5).  FP32 path stepping, FP64 accumulators.
 */

#define IRE_SRC_EXTERNAL 0
#define IRE_SRC_POINT 1

typedef struct ire_batch ire_batch;

typedef struct ire_model_desc {
    int32_t n_shells;     /* shells of this model; its r_edges hold n_shells + 1 values */
    int32_t source;       /* IRE_SRC_EXTERNAL or IRE_SRC_POINT */
    double scale;         /* external: multiplier of the batch's J_nu shape; point: luminosity L (erg/s) */
    uint64_t n_packages;  /* packages of this model (>= 1) */
    uint64_t seed;        /* random stream of this model */
} ire_model_desc;

typedef struct ire_batch_options {
    double k_bg;              /* as ire_options */
    int32_t ffi;
    double w_floor;
    uint64_t max_events;
    int32_t reemit_uniform;
    int32_t aggregate;        /* 0 or 1 as in ire_options (the workgroup grouping is single-model only) */
    int32_t batch;            /* lanes parked at an event before the wave processes events (0 = 32) */
    uint64_t item_packages;   /* packages per work item; a model is split into items (0 = 524288) */
    int32_t use_graph;        /* 1: replay zero/trace/finalize as a captured HIP graph (default) */
    int32_t use_g_E;          /* weighted sampling, as ire_options */
    double g_E;
    int32_t use_g_S;
    double g_S;
    double k_A, k_S;
    int32_t k_A_rho;          /* Sect. 3.2: absorption scaling by density per model, as ire_options
                                 (each model's scale runs over its own shells' densities) */
    double k_A_lowest, k_A_highest;
} ire_batch_options;

typedef struct ire_batch_stats {
    double L_total;            /* sum of the models' source luminosities (erg/s) */
    double escaped, ffi_escaped, terminated;
    uint64_t n_launch, n_cross, n_scat, n_abs, n_escape, n_limit, n_floor, n_below, n_above;
    uint64_t n_models, n_items, n_shells;
    uint64_t n_pass;           /* event passes of the tracer's waves */
    uint64_t n_step_slots;     /* lane slots of the crossing sweeps (64 per wave-level step) */
    float ms_run;              /* zero + trace + finalize on the device (HIP events) */
} ire_batch_stats;

/* Defaults: as ire_default_options, item_packages 524288, use_graph 1. */
int ire_batch_default_options(ire_batch_options *o);
int ire_batch_create(int hip_device, ire_batch **out);
void ire_batch_destroy(ire_batch *b);
/* As ire_set_dust / ire_set_temperature_grid, shared by every model of the batch. */
int ire_batch_set_dust(ire_batch *b, int32_t K, const double *nu, const double *kappa_abs,
                       const double *albedo, const double *g);
int ire_batch_set_temperature_grid(ire_batch *b, double t_min, double t_max, int32_t n_t);
/* Spectral shapes on the dust grid: J_shape[K] for external models (NULL if
 * none), S_shape[K] for point-source models (NULL if none); copied. */
int ire_batch_set_sources(ire_batch *b, const double *J_shape, const double *S_shape);
/* M models; r_edges_flat holds sum(n_shells + 1) radii and rho_flat sum(n_shells)
 * densities, model after model, with the constraints of ire_set_shells. */
int ire_batch_set_models(ire_batch *b, int32_t M, const ire_model_desc *models,
                         const double *r_edges_flat, const double *rho_flat);
int ire_batch_set_options(ire_batch *b, const ire_batch_options *o);
/* Run every model from zero absorbed energy (asynchronous on hip_stream). */
int ire_batch_run(ire_batch *b, void *hip_stream);
/* Synchronise and copy A_flat[sum n_shells] (erg/s) and T_flat (K); either may be NULL. */
int ire_batch_get(ire_batch *b, double *A_flat, double *T_flat, ire_batch_stats *stats);
/* Time candidate schedules (parking threshold 24/32/48 x item size 65536 ..
 * 1048576) on every model with package budgets and item sizes scaled by
 * `fraction` (0 < fraction <= 1), keep the fastest in the batch options and
 * in *chosen (may be NULL).  With a
 * cache_path, a previous choice for the same device and model class is reused
 * and new choices are stored (JSON). */
int ire_batch_autotune(ire_batch *b, double fraction, const char *cache_path, ire_batch_options *chosen);
const char *ire_batch_last_error(const ire_batch *b);

/* ------------------------------------------------------------------------
 * Learned surrogate of the IRE temperature profile: an ensemble of MLPs
 * mapping 6 inputs (log10 tau_V, density exponent, log10 L/L_sun or 0,
 * log10 external-field scale or 0, source type 0/1, r_mid/R_out), plus the
 * derived input log10(max(r_mid/R_out, 1e-4)) + 1.5, through `depth` hidden
 * layers of width 256 (SiLU) to log10 T of a shell.  BF16
 * weights and matrix-core (MFMA) products with FP32 accumulation; FP32 master
 * weights and Adam.  Trained on temperatures from the IRE tracer, which also
 * serves as the fallback wherever the ensemble's spread is too large.
 */

typedef struct sur_net sur_net;

typedef struct sur_train_opts {
    int64_t batch;       /* rows per member and step (default 4096, multiple of 128) */
    int64_t steps;       /* optimizer steps (default 2000) */
    double lr, lr_min;   /* cosine learning-rate schedule from lr to lr_min (1e-3, 1e-5) */
    double beta1, beta2, eps;  /* Adam (0.9, 0.999, 1e-8) */
    uint64_t seed;       /* mini-batch sampling (rows drawn with replacement) */
    int32_t use_graph;   /* 1: capture one step as a HIP graph and replay it (default) */
} sur_train_opts;

int sur_default_train_opts(sur_train_opts *o);
/* members >= 1 ensemble members, width must be 256, depth >= 1 hidden layers;
 * weights initialised from `seed` (He-uniform, zero biases). */
int sur_create(int hip_device, int32_t members, int32_t width, int32_t depth, uint64_t seed, sur_net **out);
void sur_destroy(sur_net *s);
/* Input standardisation x' = (x - mean) / std (6 values each) and target
 * log10 T = y_mean + y_std * output.  sur_train sets them from its data when
 * they were never set. */
int sur_set_normalization(sur_net *s, const float *x_mean, const float *x_std, float y_mean, float y_std);
/* Parameters per member (FP32, the flat layout of the weights, biases, output weights). */
int64_t sur_param_count(const sur_net *s);
int sur_get_params(sur_net *s, float *params /* members * sur_param_count */);
/* The first layer's weights on the padding inputs (columns 7..31 of W_0) are set to zero. */
int sur_set_params(sur_net *s, const float *params);
/* Train every member on rows X[n][6] (host), targets log10 T y[n] (host). */
int sur_train(sur_net *s, const float *X, const float *y, int64_t n, const sur_train_opts *o, void *hip_stream,
              float *final_loss /* members, may be NULL */);
/* Loss (mean squared error of the standardised target) and its gradient with
 * respect to every parameter for exactly these rows (1 <= n <= 65536), every
 * member, without an update (gradient checks). */
int sur_gradients(sur_net *s, const float *X, const float *y, int64_t n, float *grads /* members * count */,
                  float *loss /* members */);
/* Ensemble prediction: mean over members of log10 T and the relative spread
 * std(T)/mean(T) per row (host arrays). */
int sur_predict(sur_net *s, const float *X, int64_t n, float *mean_logT, float *spread);
/* Same on device pointers, asynchronous on hip_stream. */
int sur_predict_dev(sur_net *s, const float *X_dev, int64_t n, float *mean_logT_dev, float *spread_dev,
                    void *hip_stream);
/* Ensemble prediction for whole cloud models.  Model m owns output rows
 * [row_off[m], row_off[m+1]) (row_off[0] = 0, non-decreasing); its cloud
 * parameters are model_x[5m .. 5m+4] (the first five surrogate inputs: log10
 * tau_V, density exponent, log10 L/L_sun, log10 field scale, source type) and
 * its shells' relative mid-radii r_mid/R_out are radius[radius_off[m] + j],
 * j < row_off[m+1] - row_off[m] (models with the same shell grid may share
 * radius values; radius[n_radius]).  Writes mean log10 T and the spread
 * std(T)/mean(T) per row, and, when model_spread is not NULL, the largest row
 * spread of every model (model_spread[n_models]) for the choice of models to
 * re-run with the tracer.  Host arrays; offsets are validated (IRE_E_INVALID). */
int sur_predict_models(sur_net *s, int64_t n_models, const float *model_x, const int64_t *row_off,
                       const int64_t *radius_off, const float *radius, int64_t n_radius, float *mean_logT,
                       float *spread, float *model_spread);
/* Same on device pointers, asynchronous on hip_stream; n_rows = row_off[n_models]
 * is passed by the caller.  Offsets are not validated on the host; the kernels
 * keep every access inside the given arrays (a radius index outside
 * [0, n_radius) reads 0). */
int sur_predict_models_dev(sur_net *s, int64_t n_models, int64_t n_rows, const float *model_x_dev,
                           const int64_t *row_off_dev, const int64_t *radius_off_dev, const float *radius_dev,
                           int64_t n_radius, float *mean_logT_dev, float *spread_dev, float *model_spread_dev,
                           void *hip_stream);
int sur_save(sur_net *s, const char *path);
int sur_load(sur_net *s, const char *path);
const char *sur_last_error(const sur_net *s);

#ifdef __cplusplus
}
#endif
#endif
