/*
 * Serial FP64 reference of the immediate re-emission (IRE) tracer.
 * TEST INFRASTRUCTURE ONLY (see ire_oracle.h): called by tests, the smoke
 * check and the CPU-baseline leg of the benchmark, never by the product.
 *
 * The method (Juvela 2024, Sect. 2.1, after Bjorkman & Wood 2001):
 *   - each source's power is split over N equal packages;
 *   - a package carries two free paths in optical depth, tau_S and tau_A,
 *     each drawn as -ln u (Eq. 1);
 *   - external packages enter at (0,0,-R0) with cos(theta) = sqrt(u) about the
 *     inward normal (Eqs. 2-3); central packages start at the centre;
 *   - the package is followed one cell at a time, both free paths decreasing
 *     by kappa rho l (Eq. 4);
 *   - whichever free path reaches zero first ends the step: scattering by the
 *     Henyey-Greenstein phase function, or absorption, which raises the cell
 *     temperature and immediately re-emits the same energy isotropically at a
 *     frequency drawn from the difference of the cell emission spectra at the
 *     new and old temperatures; both free paths are redrawn after either event;
 *   - the run ends when every package has left the cloud.
 * Weighting options: centre-weighted background directions (Sect. 2.2, Eq. 5),
 * forced first interaction (Eqs. 9-12), the weight floor (Sect. 2.2.1).
 *
 * The geometry is the paper's own 3-D Cartesian frame.  Everything is FP64.
 *
 * Readings of points the paper leaves open (each is also listed with the
 * design notes of the project):
 *   - frequency integrals are sums over the discrete grid with trapezoid
 *     weights in linear nu; a package carries a frequency index;
 *   - emitted power per unit mass G(T) = 4 pi sum_k kappa_abs,k B_k(T) w_k,
 *     and a cell's temperature solves A/M = G(T); A = 0 means T = 0;
 *   - the external luminosity is the inward flux pi J through the surface:
 *     L_ext = 4 pi R0^2 * pi * sum_k J_k w_k;
 *   - the difference emission spectrum is kappa_abs,k [B_k(T_new) - B_k(T_old)] w_k;
 *   - in lookup-table mode the cumulative emission is taken as linear in G
 *     inside each temperature bin: a point a* is drawn uniformly in the slice
 *     [A_before, A_after]/M, its bin is found in the G table and the frequency
 *     is drawn from that bin's difference-spectrum CDF;
 *   - uniforms are u = (x + 0.5) 2^-32 from one 32-bit Philox word, so u is in
 *     the open interval (0,1);
 *   - with FFI the first flight is forced to end inside the cloud at an
 *     extinction depth tau = -ln[1 - u (1 - e^-tau0)]; the event is an
 *     absorption with probability 1 - albedo; the unforced fraction e^-tau0
 *     of the package power is tallied as escaped;
 *   - the weight floor is relative to the package weight after launch.
 *
 * Random-number layout (a specification the GPU path implements separately):
 * package p of source s (0 external, 1 point) uses Philox4x32-10 with key
 * (seed_lo, seed_hi) and counter (b, p_lo, p_hi, s), b = 0,1,2,... the block
 * index within the package's history.  Launch takes one block (frequency,
 * direction, tau_A or FFI depth, tau_S or FFI event type); a scattering one
 * block (cos theta, azimuth, tau_A, tau_S); an absorption two blocks, (slice
 * point a*, frequency, direction, tau_A) and (tau_S, re-emission radius).
 * The scattering azimuth is measured from the plane that holds the propagation
 * direction and the radius vector.
 */
#include "ire_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_H 6.62607015e-27   /* Planck constant, erg s */
#define OR_KB 1.380649e-16    /* Boltzmann constant, erg/K */
#define OR_C 2.99792458e10    /* speed of light, cm/s */
#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, written from Salmon, Moraes, Dror & Shaw (2011), "Parallel
 * random numbers: as easy as 1, 2, 3": a 10-round Feistel-like bijection on a
 * 128-bit counter; each round multiplies two counter words by fixed odd
 * constants, keeps the 64-bit products' halves and mixes them with the other
 * two words and the round key; the 64-bit key is advanced by the Weyl
 * constants between rounds. */
#define PH_M0 0xD2511F53u
#define PH_M1 0xCD9E8D57u
#define PH_W0 0x9E3779B9u
#define PH_W1 0xBB67AE85u

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)PH_M0 * c0;
        uint64_t p1 = (uint64_t)PH_M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += PH_W0; k1 += PH_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

typedef struct {
    uint32_t key[2];
    uint32_t pid_lo, pid_hi, src;
    uint32_t blk;
} stream_t;

static void next_block(stream_t *s, double u[4]) {
    uint32_t ctr[4] = {s->blk, s->pid_lo, s->pid_hi, s->src};
    uint32_t x[4];
    or_philox4x32_10(ctr, s->key, x);
    s->blk++;
    for (int j = 0; j < 4; ++j) u[j] = ((double)x[j] + 0.5) * 0x1p-32;
}

/* ------------------------------------------------------------------------ */
/* Physics helpers */

double or_planck(double nu, double T) {
    if (!(T > 0.0)) return 0.0;
    double x = OR_H * nu / (OR_KB * T);
    if (x > 700.0) return 0.0;
    return 2.0 * OR_H * nu * nu * nu / (OR_C * OR_C) / expm1(x);
}

/* dB/dT */
static double planck_dT(double nu, double T) {
    if (!(T > 0.0)) return 0.0;
    double x = OR_H * nu / (OR_KB * T);
    if (x > 700.0) return 0.0;
    double B = 2.0 * OR_H * nu * nu * nu / (OR_C * OR_C) / expm1(x);
    return B * x / (T * (-expm1(-x)));
}

static void trapezoid_weights(int K, const double *nu, double *w) {
    if (K == 1) { w[0] = 1.0; return; }
    for (int k = 0; k < K; ++k) {
        double hi = (k + 1 < K) ? nu[k + 1] : nu[k];
        double lo = (k > 0) ? nu[k - 1] : nu[k];
        w[k] = 0.5 * (hi - lo);
    }
}

/* ------------------------------------------------------------------------ */
/* Model state */

typedef struct {
    const or_model *m;
    or_options o;
    int K, nsh, cav;          /* nsh internal shells; cav = 1 if a virtual cavity shell leads */
    double *R;                /* nsh+1 radii */
    double *rho;              /* nsh */
    double *M;                /* nsh masses */
    double *w, *kA, *kS, *g, *alb;
    double *kAsh;             /* nsh: absorption free-path scaling per shell (Eq. 8, constant or k_A(rho)) */
    int kscale;               /* any free-path scaling */
    double *cdf[2];
    double L[2], eps[2];
    double *Tg, *lnT, *G, *lnG, *D;   /* tables (n_t and n_t*K) */
    double *q;                        /* K scratch */
} ostate;

static double G_exact(const ostate *s, double T) {
    double acc = 0.0;
    for (int k = 0; k < s->K; ++k) acc += s->kA[k] * or_planck(s->m->nu[k], T) * s->w[k];
    return 4.0 * OR_PI * acc;
}

static double dG_exact(const ostate *s, double T) {
    double acc = 0.0;
    for (int k = 0; k < s->K; ++k) acc += s->kA[k] * planck_dT(s->m->nu[k], T) * s->w[k];
    return 4.0 * OR_PI * acc;
}

/* Solve G(T) = a by bracketed Newton iteration. */
static double T_exact(const ostate *s, double a) {
    if (!(a > 0.0)) return 0.0;
    double lo = 1.0, hi = 1.0;
    int guard = 0;
    while (G_exact(s, lo) > a && guard++ < 2000) lo *= 0.5;
    guard = 0;
    while (G_exact(s, hi) < a && guard++ < 2000) hi *= 2.0;
    double T = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        double f = G_exact(s, T) - a;
        if (f == 0.0) return T;
        if (f > 0.0) hi = T; else lo = T;
        double d = dG_exact(s, T);
        double Tn = (d > 0.0) ? T - f / d : 0.5 * (lo + hi);
        if (!(Tn > lo && Tn < hi)) Tn = 0.5 * (lo + hi);
        if (fabs(Tn - T) <= 1e-15 * T || hi - lo <= 4e-16 * hi) return Tn;
        T = Tn;
    }
    return T;
}

/* Largest j in [0, n-1] with tab[j] <= x, or -1 if x < tab[0]. */
static int bin_below(const double *tab, int n, double x) {
    if (x < tab[0]) return -1;
    int lo = 0, hi = n - 1;
    if (x >= tab[hi]) return hi;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (tab[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

static double T_table(const ostate *s, double a) {
    int nt = s->m->n_t;
    if (!(a > 0.0)) return 0.0;
    int j = bin_below(s->G, nt, a);
    if (j < 0) j = 0;
    if (j > nt - 2) j = nt - 2;
    double f = (log(a) - s->lnG[j]) / (s->lnG[j + 1] - s->lnG[j]);
    return exp(s->lnT[j] + f * (s->lnT[j + 1] - s->lnT[j]));
}

/* Smallest k with u < cdf[k]; the last entry is 1 so the search always ends. */
static int sample_cdf(const double *cdf, int K, double u) {
    int lo = 0, hi = K - 1;
    while (lo < hi) {
        int mid = (lo + hi) / 2;
        if (u < cdf[mid]) hi = mid; else lo = mid + 1;
    }
    return lo;
}

static void make_cdf(const double *q, int K, double *cdf) {
    double tot = 0.0;
    for (int k = 0; k < K; ++k) tot += q[k];
    double run = 0.0;
    for (int k = 0; k < K; ++k) {
        run += q[k];
        cdf[k] = (tot > 0.0) ? run / tot : 1.0;
    }
    cdf[K - 1] = 1.0;
}

static int validate(const or_model *m) {
    if (!m || m->n < 1 || m->K < 1 || !m->r_edges || !m->rho || !m->nu || !m->kabs ||
        !m->albedo || !m->g)
        return -1;
    if (!(m->r_edges[0] >= 0.0)) return -1;
    for (int i = 0; i < m->n; ++i) {
        if (!(m->r_edges[i + 1] > m->r_edges[i])) return -1;
        if (!(m->rho[i] >= 0.0)) return -1;
    }
    for (int k = 0; k < m->K; ++k) {
        if (k > 0 && !(m->nu[k] > m->nu[k - 1])) return -1;
        if (!(m->kabs[k] > 0.0) || !(m->albedo[k] >= 0.0 && m->albedo[k] < 1.0)) return -1;
        if (!(m->g[k] > -1.0 && m->g[k] < 1.0)) return -1;
        if (m->J && !(m->J[k] >= 0.0)) return -1;
        if (m->S && !(m->S[k] >= 0.0)) return -1;
    }
    if (!(m->t_min > 0.0 && m->t_max > m->t_min) || m->n_t < 2) return -1;
    if (!(m->L_ps >= 0.0)) return -1;
    return 0;
}

static void state_free(ostate *s) {
    free(s->R); free(s->rho); free(s->M); free(s->w); free(s->kA); free(s->kS); free(s->kAsh);
    free(s->g); free(s->alb); free(s->cdf[0]); free(s->cdf[1]); free(s->Tg); free(s->lnT);
    free(s->G); free(s->lnG); free(s->D); free(s->q);
}

static int state_init(ostate *s, const or_model *m, const or_options *o) {
    memset(s, 0, sizeof(*s));
    if (validate(m)) return -1;
    s->m = m;
    if (o) s->o = *o; else or_default_options(&s->o);
    if ((s->o.k_A_rho != 0 && s->o.k_A_rho != 1) ||
        (s->o.k_A_rho && (s->o.k_A != 1.0 || !(s->o.k_A_lowest > 0.0) || !(s->o.k_A_highest > 0.0) ||
                          !isfinite(s->o.k_A_lowest) || !isfinite(s->o.k_A_highest))))
        return -1;
    if (!(s->o.k_A > 0.0) || !(s->o.k_S > 0.0) || !isfinite(s->o.k_A) || !isfinite(s->o.k_S) ||
        !(fabs(s->o.g_E) < 1.0) || !(fabs(s->o.g_S) < 1.0) || s->o.ffi < 0 || s->o.ffi > 2)
        return -1;
    int K = m->K, n = m->n, nt = m->n_t;
    s->K = K;
    s->cav = (m->r_edges[0] > 0.0) ? 1 : 0;
    s->nsh = n + s->cav;
    s->R = calloc(s->nsh + 1, sizeof(double));
    s->rho = calloc(s->nsh, sizeof(double));
    s->M = calloc(s->nsh, sizeof(double));
    s->w = calloc(K, sizeof(double));
    s->kA = calloc(K, sizeof(double));
    s->kS = calloc(K, sizeof(double));
    s->g = calloc(K, sizeof(double));
    s->alb = calloc(K, sizeof(double));
    s->cdf[0] = calloc(K, sizeof(double));
    s->cdf[1] = calloc(K, sizeof(double));
    s->Tg = calloc(nt, sizeof(double));
    s->lnT = calloc(nt, sizeof(double));
    s->G = calloc(nt, sizeof(double));
    s->lnG = calloc(nt, sizeof(double));
    s->D = calloc((size_t)nt * K, sizeof(double));
    s->q = calloc(K, sizeof(double));
    s->kAsh = calloc(s->nsh, sizeof(double));
    if (!s->kAsh || !s->R || !s->rho || !s->M || !s->w || !s->kA || !s->kS || !s->g || !s->alb ||
        !s->cdf[0] || !s->cdf[1] || !s->Tg || !s->lnT || !s->G || !s->lnG || !s->D || !s->q) {
        state_free(s);
        return -3;
    }
    /* shells; a central cavity becomes a leading shell of zero density */
    s->R[0] = 0.0;
    for (int i = 0; i <= n; ++i) s->R[i + s->cav] = m->r_edges[i];
    for (int i = 0; i < n; ++i) {
        double r0 = m->r_edges[i], r1 = m->r_edges[i + 1];
        s->rho[i + s->cav] = m->rho[i];
        s->M[i + s->cav] = m->rho[i] * 4.0 / 3.0 * OR_PI * (r1 * r1 * r1 - r0 * r0 * r0);
    }
    /* absorption free-path scaling per shell (Eq. 8): constant k_A, or k_A(rho)
     * linear in log rho from k_A_lowest at the lowest density of the model to
     * k_A_highest at the highest (k_A_highest everywhere when all densities
     * are equal; the empty cavity carries no absorption) */
    {
        double lo = INFINITY, hi = -INFINITY;
        for (int i = 0; i < s->nsh; ++i)
            if (s->rho[i] > 0.0) { lo = fmin(lo, log(s->rho[i])); hi = fmax(hi, log(s->rho[i])); }
        s->kscale = s->o.k_S != 1.0;
        for (int i = 0; i < s->nsh; ++i) {
            double k = s->o.k_A;
            if (s->o.k_A_rho) {
                k = s->o.k_A_highest;
                if (s->rho[i] > 0.0 && hi > lo)
                    k = s->o.k_A_lowest + (s->o.k_A_highest - s->o.k_A_lowest) * (log(s->rho[i]) - lo) / (hi - lo);
            }
            s->kAsh[i] = k;
            if (k != 1.0) s->kscale = 1;
        }
    }
    /* dust: kappa_S = kappa_A a / (1 - a) so that a = kappa_S / (kappa_A + kappa_S) */
    trapezoid_weights(K, m->nu, s->w);
    for (int k = 0; k < K; ++k) {
        s->kA[k] = m->kabs[k];
        s->alb[k] = m->albedo[k];
        s->kS[k] = m->kabs[k] * m->albedo[k] / (1.0 - m->albedo[k]);
        s->g[k] = m->g[k];
    }
    /* sources */
    double Rout = m->r_edges[n];
    double sJ = 0.0;
    for (int k = 0; k < K; ++k) {
        s->q[k] = m->J ? m->J[k] * s->w[k] : 0.0;
        sJ += s->q[k];
    }
    make_cdf(s->q, K, s->cdf[0]);
    s->L[0] = 4.0 * OR_PI * Rout * Rout * OR_PI * sJ;
    for (int k = 0; k < K; ++k) s->q[k] = m->S ? m->S[k] * s->w[k] : 0.0;
    make_cdf(s->q, K, s->cdf[1]);
    s->L[1] = m->S ? m->L_ps : 0.0;
    /* temperature table and re-emission CDF rows */
    for (int j = 0; j < nt; ++j) {
        s->Tg[j] = m->t_min * pow(m->t_max / m->t_min, (double)j / (double)(nt - 1));
        s->lnT[j] = log(s->Tg[j]);
        s->G[j] = G_exact(s, s->Tg[j]);
        s->lnG[j] = log(s->G[j]);
    }
    for (int j = 0; j < nt; ++j) {
        for (int k = 0; k < K; ++k) {
            double nu = m->nu[k];
            double b = (j == 0) ? or_planck(nu, s->Tg[0])
                                : or_planck(nu, s->Tg[j]) - or_planck(nu, s->Tg[j - 1]);
            s->q[k] = s->kA[k] * b * s->w[k];
        }
        make_cdf(s->q, K, s->D + (size_t)j * K);
    }
    return 0;
}

void or_default_options(or_options *o) {
    o->k_bg = 0.5;
    o->ffi = 0;
    o->w_floor = 1e-10;
    o->max_events = 1000000;
    o->table_mode = 1;
    o->acc_bits = 0;
    o->n_batches = 1;
    o->reemit_uniform = 0;
    o->use_g_E = 0;
    o->g_E = 0.0;
    o->use_g_S = 0;
    o->g_S = 0.0;
    o->k_A = 1.0;
    o->k_S = 1.0;
    o->k_A_rho = 0;
    o->k_A_lowest = 3.0;
    o->k_A_highest = 1.0;
}

/* ------------------------------------------------------------------------ */
/* Samplers (the formulas of Sect. 2.1-2.2) */

/* Eq. 2 and Eq. 5: cosine about the inward normal; weight 2 k mu^(2 - 1/k). */
static double launch_mu(double k_bg, double u, double *W) {
    if (k_bg == 0.5) { *W = 1.0; return sqrt(u); }
    double mu = pow(u, k_bg);
    *W = 2.0 * k_bg * pow(mu, 2.0 - 1.0 / k_bg);
    return mu;
}

/* Henyey-Greenstein scattering angle by inversion of its cumulative distribution. */
static double hg_cos(double g, double u) {
    if (fabs(g) < 1e-6) return 2.0 * u - 1.0;
    double f = (1.0 - g * g) / (1.0 - g + 2.0 * g * u);
    double c = (1.0 + g * g - f * f) / (2.0 * g);
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    return c;
}

/* Eq. 10 and Eq. 12 */
static double ffi_depth(double tau0, double u, double *W) {
    double p = -expm1(-tau0);
    *W = p;
    return -log1p(-u * p);
}

/* Eqs. 10 and 12 with the optical depth counted in absorption only.  The
 * interaction point is drawn from the truncated exponential in absorption
 * depth tA in [0, tau0_A); its extinction depth is tA / (1 - a).  The weight
 * is the ratio of the densities of the interaction point in extinction depth,
 * e^{-tau} against the drawn (1 - a) e^{-tA} / (1 - e^{-tau0_A}). */
double or_ffi_absorption(double tau0, double a, double u, double *W) {
    const double tau0A = tau0 * (1.0 - a);
    const double pA = -expm1(-tau0A);
    const double tA = -log1p(-u * pA);
    const double tau = tA / (1.0 - a);
    *W = pA / (1.0 - a) * exp(tA - tau);
    return tau;
}

/* Henyey-Greenstein probability density of mu = cos(theta), Eq. 6 */
static double hg_pdf(double g, double mu) {
    const double q = 1.0 + g * g - 2.0 * g * mu;
    return 0.5 * (1.0 - g * g) / (q * sqrt(q));
}

int or_eval_sampler(int32_t which, double param, int64_t n, const double *u, double *out,
                    double *w) {
    for (int64_t i = 0; i < n; ++i) {
        double W = 1.0;
        switch (which) {
        case 0: out[i] = launch_mu(param, u[i], &W); break;
        case 1: out[i] = hg_cos(param, u[i]); break;
        case 2: out[i] = -log(u[i]); break;
        case 3: out[i] = ffi_depth(param, u[i], &W); break;
        case 4: out[i] = 2.0 * u[i] - 1.0; break;
        default: return -1;
        }
        if (w) w[i] = W;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 3-D geometry */

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Any unit vector perpendicular to unit vector a. */
static void perp_unit(const double *a, double *e) {
    double ax = fabs(a[0]), ay = fabs(a[1]), az = fabs(a[2]);
    double t[3] = {0, 0, 0};
    if (ax <= ay && ax <= az) t[0] = 1; else if (ay <= az) t[1] = 1; else t[2] = 1;
    double c = dot3(t, a);
    for (int j = 0; j < 3; ++j) e[j] = t[j] - c * a[j];
    double nrm = sqrt(dot3(e, e));
    for (int j = 0; j < 3; ++j) e[j] /= nrm;
}

/* Rotate unit direction d by the scattering angle acos(ct) at azimuth ph,
 * the azimuth measured from the plane that holds d and the radius vector x
 * (any reference plane when the flight is radial or x = 0). */
static void scatter_direction(const double *x, double *d, double ct, double ph) {
    double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    double r = sqrt(dot3(x, x));
    double e2[3], e3[3];
    double nv = 0.0;
    if (r > 0.0) {
        double mu = dot3(x, d) / r;
        for (int j = 0; j < 3; ++j) e2[j] = x[j] / r - mu * d[j];
        nv = sqrt(dot3(e2, e2));
    }
    if (nv > 1e-12) {
        for (int j = 0; j < 3; ++j) e2[j] /= nv;
    } else {
        perp_unit(d, e2);
    }
    e3[0] = d[1] * e2[2] - d[2] * e2[1];
    e3[1] = d[2] * e2[0] - d[0] * e2[2];
    e3[2] = d[0] * e2[1] - d[1] * e2[0];
    double cp = cos(ph), sph = sin(ph);
    for (int j = 0; j < 3; ++j) d[j] = ct * d[j] + st * (cp * e2[j] + sph * e3[j]);
    double nrm = sqrt(dot3(d, d));
    for (int j = 0; j < 3; ++j) d[j] /= nrm;
}

int or_scatter_direction(const double x[3], double d[3], double ct, double ph) {
    scatter_direction(x, d, ct, ph);
    return 0;
}

/* Eq. 6: re-emission cosine mu' about the reference direction from HG(g_E);
 * the weight is the isotropic density over the HG density at mu'. */
double or_reemit_weighted(double g_E, int32_t src, double u, double *W) {
    const double mup = hg_cos(g_E, u);
    *W = 0.5 / hg_pdf(g_E, mup);
    return src == 0 ? -mup : mup;
}

/* Eq. 7 (as the ratio of the two densities): the new direction's cosine mu'
 * about the reference direction is drawn from HG(g_S), its azimuth about the
 * radius vector uniformly from the plane of d and x; the weight is the dust's
 * HG density at the actual scattering angle over HG(g_S) at mu'. */
int or_scatter_weighted(const double x[3], double d[3], double g, double g_S, int32_t src, double u0,
                        double u1, double *cos_theta, double *W) {
    double xh[3], e1[3], e2[3], dn[3];
    const double r = sqrt(dot3(x, x));
    if (r > 0.0) { for (int j = 0; j < 3; ++j) xh[j] = x[j] / r; }
    else { for (int j = 0; j < 3; ++j) xh[j] = d[j]; }
    const double mu_old = dot3(xh, d);
    for (int j = 0; j < 3; ++j) e1[j] = d[j] - mu_old * xh[j];
    const double ne = sqrt(dot3(e1, e1));
    if (ne > 1e-12) { for (int j = 0; j < 3; ++j) e1[j] /= ne; }
    else perp_unit(xh, e1);
    e2[0] = xh[1] * e1[2] - xh[2] * e1[1];
    e2[1] = xh[2] * e1[0] - xh[0] * e1[2];
    e2[2] = xh[0] * e1[1] - xh[1] * e1[0];
    const double mup = hg_cos(g_S, u0);
    const double mun = src == 0 ? -mup : mup;
    const double sn = sqrt(fmax(0.0, 1.0 - mun * mun));
    const double ph = 2.0 * OR_PI * u1;
    for (int j = 0; j < 3; ++j) dn[j] = mun * xh[j] + sn * (cos(ph) * e1[j] + sin(ph) * e2[j]);
    double ct = dot3(d, dn);
    if (ct > 1.0) ct = 1.0;
    if (ct < -1.0) ct = -1.0;
    *cos_theta = ct;
    *W = hg_pdf(g, ct) / hg_pdf(g_S, mup);
    const double nrm = sqrt(dot3(dn, dn));
    for (int j = 0; j < 3; ++j) d[j] = dn[j] / nrm;
    return 0;
}

/* Distance along d from x to the boundary that ends the straight flight in
 * internal shell i; *dir = -1 for the inner sphere, +1 for the outer one. */
static double boundary_distance(const ostate *s, const double *x, const double *d, int i, int *dir) {
    double p = dot3(x, d), q = dot3(x, x);
    double Rlo = s->R[i], Rhi = s->R[i + 1];
    if (Rlo > 0.0 && p < 0.0) {
        double disc = p * p - (q - Rlo * Rlo);
        if (disc > 0.0) {
            double sd = (q - Rlo * Rlo) / (-p + sqrt(disc));
            *dir = -1;
            return sd > 0.0 ? sd : 0.0;
        }
    }
    double c = Rhi * Rhi - q;
    double disc = p * p + c;
    if (disc < 0.0) disc = 0.0;
    double sd = (p >= 0.0) ? c / (p + sqrt(disc)) : -p + sqrt(disc);
    if (!(sd > 0.0)) sd = 0.0;
    *dir = +1;
    return sd;
}

/* Extinction optical depth along the ray from x in shell i to the outer surface. */
static double ray_depth(const ostate *s, const double *x0, const double *d, int i, int k) {
    double x[3] = {x0[0], x0[1], x0[2]};
    double tau = 0.0, kext = s->kA[k] + s->kS[k];
    for (;;) {
        int dir;
        double l = boundary_distance(s, x, d, i, &dir);
        tau += kext * s->rho[i] * l;
        for (int j = 0; j < 3; ++j) x[j] += l * d[j];
        i += dir;
        if (i >= s->nsh) return tau;
    }
}

/* Emulated reduced-precision accumulator: round to `bits` significand bits. */
static double round_bits(double v, int bits) {
    if (bits <= 0 || v == 0.0) return v;
    int e;
    double f = frexp(v, &e);
    double sc = ldexp(1.0, bits);
    return ldexp(nearbyint(f * sc) / sc, e);
}

/* ------------------------------------------------------------------------ */
/* The tracer */

typedef struct {
    double *A;          /* nsh accumulators (FP64 or emulated) */
    double *Acur;       /* current-batch counters in the two-counter emulation */
    double *reemit;     /* nsh*K or NULL */
    double *first_abs;  /* nsh or NULL */
    double *sed;        /* 2*K escaped power per source and frequency, or NULL */
    double *sed_direct; /* 2*K the part that escaped without any event, or NULL */
    or_stats st;
} tally_t;

/* escaping power of a package of source src at frequency k */
static void tally_escape(tally_t *t, int K, int src, int k, double e, int direct) {
    t->st.escaped[src] += e;
    if (t->sed) t->sed[src * K + k] += e;
    if (direct && t->sed_direct) t->sed_direct[src * K + k] += e;
}

static double acc_read(const ostate *s, const tally_t *t, int i) {
    if (s->o.acc_bits > 0 && s->o.n_batches > 1) return round_bits(t->A[i] + t->Acur[i], s->o.acc_bits);
    return t->A[i];
}

static void acc_add(const ostate *s, tally_t *t, int i, double E) {
    if (s->o.acc_bits <= 0) { t->A[i] += E; return; }
    if (s->o.n_batches > 1) t->Acur[i] = round_bits(t->Acur[i] + E, s->o.acc_bits);
    else t->A[i] = round_bits(t->A[i] + E, s->o.acc_bits);
}

static void trace_package(const ostate *s, tally_t *t, int src, uint64_t pid, uint64_t seed) {
    const or_model *m = s->m;
    const int K = s->K;
    stream_t rs;
    rs.key[0] = (uint32_t)seed; rs.key[1] = (uint32_t)(seed >> 32);
    rs.pid_lo = (uint32_t)pid; rs.pid_hi = (uint32_t)(pid >> 32);
    rs.src = (uint32_t)src; rs.blk = 0;
    const double eps = s->eps[src];

    double u[4], u2[4];
    double x[3], d[3];
    int i, k;
    double W = 1.0, tauA, tauS;

    /* launch */
    next_block(&rs, u);
    t->st.n_launch++;
    k = sample_cdf(s->cdf[src], K, u[0]);
    if (src == 0) {
        double mu = launch_mu(s->o.k_bg, u[1], &W);
        x[0] = 0.0; x[1] = 0.0; x[2] = -s->R[s->nsh];
        d[0] = sqrt(fmax(0.0, 1.0 - mu * mu)); d[1] = 0.0; d[2] = mu;
        i = s->nsh - 1;
    } else {
        double mu = 2.0 * u[1] - 1.0;
        x[0] = x[1] = x[2] = 0.0;
        d[0] = sqrt(fmax(0.0, 1.0 - mu * mu)); d[1] = 0.0; d[2] = mu;
        i = 0;
    }
    /* Free paths drawn from k e^{-k tau} (Eq. 8), with k the same everywhere
     * or, for absorption, a function of the local density: the absorption
     * clock runs down a standard exponential depth at k_i times the true rate
     * in shell i, the scattering clock at k_S times it.  The realised outcome
     * carries, when the flight ends, the weight true / modified probability:
     * the fired clock's 1/k times e^{modified - true depth} of both clocks. */
    const double kS = s->o.k_S;
    int kw;                      /* this flight's free paths are k-scaled */
    double tA0, tS0;             /* the depths drawn for this flight (absorption: modified depth) */
    double trA = 0.0;            /* true absorption depth traversed in this flight */
    if (s->o.ffi) {
        double tau0 = ray_depth(s, x, d, i, k);
        if (!(tau0 > 0.0)) {
            tally_escape(t, K, src, k, eps * W, 1);
            t->st.n_escape++;
            t->st.n_direct++;
            return;
        }
        double p;
        double tau = s->o.ffi == 2 ? or_ffi_absorption(tau0, s->alb[k], u[2], &p) : ffi_depth(tau0, u[2], &p);
        t->st.ffi_escaped += eps * W * exp(-tau0);
        /* the unforced fraction leaves unscattered at the launch frequency */
        if (t->sed) t->sed[src * K + k] += eps * W * exp(-tau0);
        if (t->sed_direct) t->sed_direct[src * K + k] += eps * W * exp(-tau0);
        W *= p;
        if (u[3] < s->alb[k]) { tauS = tau * s->alb[k]; tauA = INFINITY; }
        else { tauA = tau * (1.0 - s->alb[k]); tauS = INFINITY; }
        kw = 0;
    } else {
        tauA = -log(u[2]);
        tauS = -log(u[3]) / kS;
        kw = s->kscale;
    }
    tA0 = tauA;
    tS0 = tauS;
    const double W0 = W;
    uint64_t events = 0;

    for (;;) {
        int dir;
        double lb = boundary_distance(s, x, d, i, &dir);
        double chiA = s->kA[k] * s->rho[i], chiS = s->kS[k] * s->rho[i];
        const double kAi = kw ? s->kAsh[i] : 1.0;
        const double chiAm = kAi * chiA;          /* rate of the (modified) absorption clock */
        double lA = chiAm > 0.0 ? tauA / chiAm : INFINITY;
        double lS = chiS > 0.0 ? tauS / chiS : INFINITY;
        if (lb < fmin(lA, lS)) {
            for (int j = 0; j < 3; ++j) x[j] += lb * d[j];
            tauA -= chiAm * lb;
            tauS -= chiS * lb;
            trA += chiA * lb;
            i += dir;
            if (i >= s->nsh) {
                if (kw) W *= exp((tA0 - tauA) - trA + (kS - 1.0) * (tS0 - tauS));
                tally_escape(t, K, src, k, eps * W, events == 0);
                t->st.n_escape++;
                if (events == 0) t->st.n_direct++;
                return;
            }
            t->st.n_cross++;
            continue;
        }
        if (kw) {
            if (lA <= lS) {
                trA += chiA * lA;
                W *= exp(tA0 - trA + (kS - 1.0) * (tS0 - (tauS - chiS * lA))) / kAi;
            } else {
                trA += chiA * lS;
                W *= exp((tA0 - (tauA - chiAm * lS)) - trA + (kS - 1.0) * tS0) / kS;
            }
        }
        if (events >= s->o.max_events) {
            t->st.terminated += eps * W;
            t->st.n_limit++;
            return;
        }
        events++;
        if (lA <= lS) {
            /* absorption and immediate re-emission (Sect. 2.1) */
            for (int j = 0; j < 3; ++j) x[j] += lA * d[j];
            t->st.n_abs++;
            const double E = eps * W;
            if (events == 1 && t->first_abs) t->first_abs[i] += E;
            double A_before = acc_read(s, t, i);
            acc_add(s, t, i, E);
            /* Random numbers: two blocks, (slice point, frequency, direction,
             * tau_A) and (tau_S, position in the shell). */
            next_block(&rs, u);
            next_block(&rs, u2);
            if (s->o.table_mode) {
                /* reading R8: a* uniform in the slice [A_before, A_before + E] / M_i
                 * selects the temperature bin of the G table whose difference
                 * spectrum the frequency is drawn from; a* above the last table
                 * point takes the last bin (counted) */
                const double astar = (A_before + u[0] * E) / s->M[i];
                int row = bin_below(s->G, m->n_t, astar) + 1;
                if (row > m->n_t - 1) { row = m->n_t - 1; t->st.n_reemit_above++; }
                k = sample_cdf(s->D + (size_t)row * K, K, u[1]);
            } else {
                double Told = T_exact(s, A_before / s->M[i]);
                double Tnew = T_exact(s, (A_before + E) / s->M[i]);
                double tot = 0.0;
                for (int kk = 0; kk < K; ++kk) {
                    double nu = m->nu[kk];
                    s->q[kk] = s->kA[kk] * (or_planck(nu, Tnew) - or_planck(nu, Told)) * s->w[kk];
                    if (s->q[kk] < 0.0) s->q[kk] = 0.0;
                    tot += s->q[kk];
                }
                if (!(tot > 0.0)) {
                    /* the slice is below the resolution of FP64: its limit is dB/dT */
                    for (int kk = 0; kk < K; ++kk)
                        s->q[kk] = s->kA[kk] * planck_dT(m->nu[kk], Tnew) * s->w[kk];
                }
                double cdf_run = 0.0, tot2 = 0.0;
                for (int kk = 0; kk < K; ++kk) tot2 += s->q[kk];
                k = K - 1;
                for (int kk = 0; kk < K; ++kk) {
                    cdf_run += s->q[kk];
                    if (u[1] * tot2 < cdf_run) { k = kk; break; }
                }
            }
            if (t->reemit) t->reemit[(size_t)i * K + k] += E;
            /* isotropic direction about the local radius vector */
            double r = sqrt(dot3(x, x));
            double xh[3];
            if (r > 0.0) { for (int j = 0; j < 3; ++j) xh[j] = x[j] / r; }
            else { xh[0] = 0; xh[1] = 0; xh[2] = 1; }
            if (s->o.reemit_uniform) {
                double r0 = s->R[i], r1 = s->R[i + 1];
                double rn = cbrt(r0 * r0 * r0 + u2[1] * (r1 * r1 * r1 - r0 * r0 * r0));
                for (int j = 0; j < 3; ++j) x[j] = rn * xh[j];
            }
            double mu, e[3];
            if (s->o.use_g_E) {
                double wE;
                mu = or_reemit_weighted(s->o.g_E, src, u[2], &wE);
                W *= wE;
            } else {
                mu = 2.0 * u[2] - 1.0;
            }
            perp_unit(xh, e);
            double sn = sqrt(fmax(0.0, 1.0 - mu * mu));
            for (int j = 0; j < 3; ++j) d[j] = mu * xh[j] + sn * e[j];
            tauA = -log(u[3]);
            tauS = -log(u2[0]) / kS;
            kw = s->kscale;
            tA0 = tauA;
            tS0 = tauS;
            trA = 0.0;
        } else {
            /* scattering (Sect. 2.1, Henyey-Greenstein phase function) */
            for (int j = 0; j < 3; ++j) x[j] += lS * d[j];
            t->st.n_scat++;
            next_block(&rs, u);
            if (s->o.use_g_S) {
                double ct, wS;
                or_scatter_weighted(x, d, s->g[k], s->o.g_S, src, u[0], u[1], &ct, &wS);
                W *= wS;
            } else {
                double ct = hg_cos(s->g[k], u[0]);
                double ph = 2.0 * OR_PI * u[1];
                scatter_direction(x, d, ct, ph);
            }
            tauA = -log(u[2]);
            tauS = -log(u[3]) / kS;
            kw = s->kscale;
            tA0 = tauA;
            tS0 = tauS;
            trA = 0.0;
        }
        if (W < s->o.w_floor * W0) {
            t->st.terminated += eps * W;
            t->st.terminated_floor += eps * W;
            t->st.n_floor++;
            return;
        }
    }
}

int or_run(const or_model *m, const or_options *o, uint64_t n_ext, uint64_t n_ps,
           uint64_t seed, double *A, double *T, or_stats *st, double *reemit,
           double *first_abs, double *sed, double *sed_direct) {
    ostate s;
    int rc = state_init(&s, m, o);
    if (rc) return rc;
    const int n = m->n, K = m->K;
    if (n_ext > 0 && !(s.L[0] > 0.0)) { state_free(&s); return -2; }
    if (n_ps > 0 && !(s.L[1] > 0.0)) { state_free(&s); return -2; }
    s.eps[0] = n_ext ? s.L[0] / (double)n_ext : 0.0;
    s.eps[1] = n_ps ? s.L[1] / (double)n_ps : 0.0;

    tally_t t;
    memset(&t, 0, sizeof(t));
    t.A = calloc(s.nsh, sizeof(double));
    t.Acur = calloc(s.nsh, sizeof(double));
    t.reemit = reemit ? calloc((size_t)s.nsh * K, sizeof(double)) : NULL;
    t.first_abs = first_abs ? calloc(s.nsh, sizeof(double)) : NULL;
    if (sed) { memset(sed, 0, 2 * (size_t)K * sizeof(double)); t.sed = sed; }
    if (sed_direct) { memset(sed_direct, 0, 2 * (size_t)K * sizeof(double)); t.sed_direct = sed_direct; }
    if (!t.A || !t.Acur || (reemit && !t.reemit) || (first_abs && !t.first_abs)) {
        free(t.A); free(t.Acur); free(t.reemit); free(t.first_abs);
        state_free(&s);
        return -3;
    }
    t.st.L_ext = s.L[0];
    t.st.L_ps = s.L[1];

    /* external packages first, then point-source packages; with the
     * two-counter scheme the current-batch counters are folded every
     * (n_ext + n_ps) / n_batches packages */
    uint64_t total = n_ext + n_ps, done = 0;
    uint64_t nb = (s.o.acc_bits > 0 && s.o.n_batches > 1) ? (uint64_t)s.o.n_batches : 1;
    for (int src = 0; src < 2; ++src) {
        uint64_t N = src ? n_ps : n_ext;
        for (uint64_t p = 0; p < N; ++p) {
            trace_package(&s, &t, src, p, seed);
            done++;
            if (nb > 1 && (done * nb) / total != ((done - 1) * nb) / total) {
                for (int i = 0; i < s.nsh; ++i) {
                    t.A[i] = round_bits(t.A[i] + t.Acur[i], s.o.acc_bits);
                    t.Acur[i] = 0.0;
                }
            }
        }
    }
    for (int i = 0; i < n; ++i) {
        int ii = i + s.cav;
        double Ai = (nb > 1) ? round_bits(t.A[ii] + t.Acur[ii], s.o.acc_bits) : t.A[ii];
        if (A) A[i] = Ai;
        double a = Ai / s.M[ii];
        double Ti;
        if (!(a >= s.G[0])) { Ti = m->t_min; t.st.n_below++; }
        else if (a > s.G[m->n_t - 1]) { Ti = m->t_max; t.st.n_above++; }
        else Ti = s.o.table_mode ? T_table(&s, a) : T_exact(&s, a);
        if (T) T[i] = Ti;
        if (reemit)
            for (int k = 0; k < K; ++k) reemit[(size_t)i * K + k] = t.reemit[(size_t)ii * K + k];
        if (first_abs) first_abs[i] = t.first_abs[ii];
    }
    if (st) *st = t.st;
    free(t.A); free(t.Acur); free(t.reemit); free(t.first_abs);
    state_free(&s);
    return 0;
}

int or_tables(const or_model *m, double *w, double *G, double *D, double *cdf_ext,
              double *cdf_ps, double *mass, double *L) {
    ostate s;
    int rc = state_init(&s, m, NULL);
    if (rc) return rc;
    int K = m->K, nt = m->n_t;
    if (w) memcpy(w, s.w, K * sizeof(double));
    if (G) memcpy(G, s.G, nt * sizeof(double));
    if (D) memcpy(D, s.D, (size_t)nt * K * sizeof(double));
    if (cdf_ext) memcpy(cdf_ext, s.cdf[0], K * sizeof(double));
    if (cdf_ps) memcpy(cdf_ps, s.cdf[1], K * sizeof(double));
    if (mass) memcpy(mass, s.M + s.cav, m->n * sizeof(double));
    if (L) { L[0] = s.L[0]; L[1] = s.L[1]; }
    state_free(&s);
    return 0;
}

double or_temperature(const or_model *m, double a, int32_t table_mode) {
    ostate s;
    if (state_init(&s, m, NULL)) return NAN;
    double T = table_mode ? T_table(&s, a) : T_exact(&s, a);
    state_free(&s);
    return T;
}
