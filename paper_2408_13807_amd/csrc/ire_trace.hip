// IRE photon-package tracer for gfx950 (MI355X).
//
// One lane follows one package at a time in a persistent wavefront; a lane
// whose package has left the cloud takes the next package index from a global
// cursor (one atomic per wave per refill).  Shell geometry is one-dimensional:
// a straight flight is described by its squared impact parameter b2 (constant)
// and the signed distance t from the tangent point (r^2 = b2 + t^2), in units
// of the outer radius.  The shell index changes only by +-1 at a crossing and is
// never recomputed from r, so a package cannot stick on a boundary.
//
// The method (Juvela 2024, Sect. 2.1): two free paths tau_A and tau_S drawn as
// -ln u (Eq. 1); stepping one shell at a time decreasing both by kappa rho l
// (Eq. 4); scattering with the Henyey-Greenstein function; absorption deposits
// the package energy into the shell and re-emits it at once, isotropically, at
// a frequency drawn from the difference of the shell emission spectra at the new
// and old temperatures; both free paths are redrawn after every event.
// Weighting: centre-weighted background directions (Eq. 5) and forced first
// interaction (Eqs. 9-12).
//
// The difference-spectrum draw uses lookup tables: with the cumulative emission
// taken as linear in G(T) within a temperature bin, drawing a point a* uniformly
// in the slice [A_before, A_after]/M of absorbed power per mass, locating its bin
// in the G table and drawing the frequency from that bin's CDF of
// kappa_abs [B(T_hi) - B(T_lo)] w reproduces the difference spectrum, and the
// slices of all absorptions in a shell tile [0, A_final] in any order.  A_before
// is therefore the value returned by a returning FP64 atomic, optionally after a
// wave-level segmented scan of the energies of lanes absorbing in the same shell.
//
// Random numbers: Philox4x32-10 (Salmon et al. 2011), key = seed, counter =
// (block, package id lo, package id hi, source); launch and scattering use one
// block, an absorption two.  u = (x + 0.5) 2^-32.
//
// Two instantiations: float stepping with all tables in LDS, and double
// everywhere with tables read from global memory.  Absorbed-energy
// accumulators and package energies are FP64 in both.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ire_internal.h"

namespace ire {
namespace {

constexpr int kWave = 64;
constexpr int kBlockFP32 = 1024;

// ---------------------------------------------------------------------------
// Philox4x32-10

struct Rand4 { uint32_t x, y, z, w; };

__device__ __forceinline__ Rand4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Rand4{c0, c1, c2, c3};
}

// ---------------------------------------------------------------------------
// Precision policy

template <typename R> struct P;

template <> struct P<float> {
    using Shell = ShellF;
    using Dust = DustF;
    static __device__ __forceinline__ float uni(uint32_t x) {
        float u = __builtin_fmaf((float)x, 0x1p-32f, 0x1p-33f);
        return u < 0x1.fffffep-1f ? u : 0x1.fffffep-1f;
    }
    static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float nlog(float u) { return -__logf(u); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float cos2pi(float u) { return __builtin_amdgcn_cosf(u); }
    static __device__ __forceinline__ float powr(float a, float b) { return __powf(a, b); }
    static __device__ __forceinline__ float expm1_(float x) { return expm1f(x); }
    static __device__ __forceinline__ float log1p_(float x) { return log1pf(x); }
    static __device__ __forceinline__ float cbrt_(float x) { return cbrtf(x); }
    static __device__ __forceinline__ float inf() { return __builtin_huge_valf(); }
};

template <> struct P<double> {
    using Shell = ShellD;
    using Dust = DustD;
    static __device__ __forceinline__ double uni(uint32_t x) { return ((double)x + 0.5) * 0x1p-32; }
    static __device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
    static __device__ __forceinline__ double nlog(double u) { return -log(u); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double cos2pi(double u) { return cospi(2.0 * u); }
    static __device__ __forceinline__ double powr(double a, double b) { return pow(a, b); }
    static __device__ __forceinline__ double expm1_(double x) { return expm1(x); }
    static __device__ __forceinline__ double log1p_(double x) { return log1p(x); }
    static __device__ __forceinline__ double cbrt_(double x) { return cbrt(x); }
    static __device__ __forceinline__ double inf() { return __builtin_huge_val(); }
};

// Number of entries of the non-decreasing table t[0..n) that are <= x.
template <typename T, typename X>
__device__ __forceinline__ int count_le(const T *t, int n, X x) {
    int pos = 0;
    int step = 1;
    while (step * 2 <= n) step *= 2;
    for (; step > 0; step >>= 1) {
        const int q = pos + step;
        if (q <= n && (X)t[q - 1] <= x) pos = q;
    }
    return pos;
}

// ---------------------------------------------------------------------------
// Wave-level helpers (wave64)

__device__ __forceinline__ double wave_excl_scan(double v) {
    const int lane = __lane_id();
    double incl = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const double o = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += o;
    }
    double ex = __shfl_up(incl, 1, kWave);
    return lane == 0 ? 0.0 : ex;
}

// Returning fetch-add of E into A[i] for the lanes with act set; every lane of
// the wave must call it.  With AGG, lanes that hit the same shell are folded
// into one atomic and each receives base + (sum of E of lower lanes).
template <bool AGG>
__device__ __forceinline__ double fetch_add_energy(double *A, int i, double E, bool act) {
    double res = 0.0;
    if constexpr (!AGG) {
        if (act) res = unsafeAtomicAdd(&A[(size_t)i * kAccStride], E);
        return res;
    } else {
        const int lane = __lane_id();
        unsigned long long pending = __ballot(act);
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const int s = __shfl(i, leader, kWave);
            const unsigned long long grp = __ballot(act && i == s);
            pending &= ~grp;
            const bool mine = (grp >> lane) & 1ull;
            if (__popcll(grp) == 1) {
                if (mine) res = unsafeAtomicAdd(&A[(size_t)s * kAccStride], E);
            } else {
                const double v = mine ? E : 0.0;
                const double ex = wave_excl_scan(v);
                const double tot = __shfl(ex + v, kWave - 1, kWave);
                double base = 0.0;
                if (lane == leader) base = unsafeAtomicAdd(&A[(size_t)s * kAccStride], tot);
                base = __shfl(base, leader, kWave);
                if (mine) res = base + ex;
            }
        }
        return res;
    }
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// ---------------------------------------------------------------------------
// The tracer

template <typename R, bool AGG>
__device__ __forceinline__ void trace_body(const TraceParams &p, const typename P<R>::Shell *sh,
                                           const typename P<R>::Dust *dust, const R *cdf,
                                           const R *G, const R *D) {
    using Shell = typename P<R>::Shell;
    using Dust = typename P<R>::Dust;
    enum : int { ST_FLY = 0, ST_ABS = 1, ST_SCAT = 2, ST_DEAD = 3 };
    const int n = p.n, K = p.K, n_t = p.n_t;
    const uint32_t key0 = (uint32_t)p.seed, key1 = (uint32_t)(p.seed >> 32);
    const unsigned long long total = p.n_ext + p.n_ps;
    const int lane = __lane_id();
    const long long gtid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int batch = p.batch > 0 ? p.batch : 1;

    unsigned long long pool_next = 0, pool_end = 0;  // wave-uniform

    // package state
    int st = ST_DEAD;
    bool done = (p.max_lanes > 0) && (gtid >= p.max_lanes);
    int i = 0, k = 0, src = 0;
    R b2 = 0, t = 0, tauA = 0, tauS = 0, W = 1, W0 = 1;
    R kA = 0, kS = 0, gg = 0, alb = 0;
    uint32_t pid_lo = 0, pid_hi = 0, blk = 0;
    unsigned long long events = 0;

    // per-lane counters and tallies
    uint32_t c_launch = 0, c_cross = 0, c_scat = 0, c_abs = 0, c_escape = 0, c_direct = 0;
    uint32_t c_limit = 0, c_floor = 0, c_reabove = 0;
    double esc0 = 0.0, esc1 = 0.0, ffi_esc = 0.0, term = 0.0;

    auto escape = [&]() {
        const double e = p.eps[src] * (double)W;
        if (src == 0) esc0 += e; else esc1 += e;
        c_escape++;
        if (events == 0) c_direct++;
        st = ST_DEAD;
    };

    for (;;) {
        // ---- crossing sweep: lanes in flight step from boundary to boundary;
        // a lane that reaches an event (or loses its package) parks until
        // enough lanes of the wave are parked to process their events together
        for (;;) {
            const unsigned long long fly = __ballot(st == ST_FLY);
            const unsigned long long wait = __ballot(st != ST_FLY && !done);
            const int live = __popcll(fly | wait);
            const int want = batch < (live + 1) / 2 ? batch : ((live + 1) / 2 > 0 ? (live + 1) / 2 : 1);
            if (fly == 0 || __popcll(wait) >= want) break;
            if (st == ST_FLY) {
                const Shell s = sh[i];
                const bool inward = (t < (R)0) && (b2 < s.r2_in);
                const R arg = (inward ? s.r2_in : s.r2_out) - b2;
                const R sq = P<R>::sqrt_(arg > (R)0 ? arg : (R)0);
                const R tn = inward ? -sq : sq;
                const R lb = tn - t > (R)0 ? tn - t : (R)0;
                const R chiA = kA * s.rho, chiS = kS * s.rho;
                const R dA = chiA * lb, dS = chiS * lb;
                if (dA < tauA && dS < tauS) {
                    // boundary crossing (Eq. 4); the central cavity is crossed in one jump
                    tauA -= dA;
                    tauS -= dS;
                    const bool cav = inward && i == 0;
                    t = cav ? -tn : tn;
                    i += inward ? (cav ? 0 : -1) : 1;
                    c_cross += cav ? 2u : 1u;
                    if (i == n) {
                        c_cross--;
                        escape();
                    }
                } else if (events >= p.max_events) {
                    term += p.eps[src] * (double)W;
                    c_limit++;
                    st = ST_DEAD;
                } else {
                    // the free path that runs out first ends the flight (Sect. 2.1)
                    events++;
                    const R lA = chiA > (R)0 ? tauA * P<R>::rcp(chiA) : P<R>::inf();
                    const R lS = chiS > (R)0 ? tauS * P<R>::rcp(chiS) : P<R>::inf();
                    const bool ab = lA <= lS;
                    t += ab ? lA : lS;
                    st = ab ? ST_ABS : ST_SCAT;
                }
            }
        }
        if (__ballot(st != ST_FLY && !done) == 0) break;  // nothing in flight, nothing pending

        // ---- event batch
        // (package indices come from a wave-private pool refilled `chunk` at a time)
        bool launching = false;
        const unsigned long long need = __ballot(st == ST_DEAD && !done);
        if (need) {
            const unsigned long long cnt = __popcll(need);
            const unsigned long long avail = pool_end - pool_next;
            unsigned long long fresh = 0;
            if (avail < cnt) {
                const int leader = __ffsll((long long)need) - 1;
                if (lane == leader) fresh = atomicAdd(&p.stats->cursor, p.chunk);
                fresh = __shfl(fresh, leader, kWave);
            }
            if (st == ST_DEAD && !done) {
                const unsigned long long rank = __popcll(need & __lanemask_lt());
                const unsigned long long gidx = rank < avail ? pool_next + rank : fresh + (rank - avail);
                if (gidx >= total) {
                    done = true;
                } else {
                    src = gidx < p.n_ext ? 0 : 1;
                    const unsigned long long pid = p.pid0[src] + (src ? gidx - p.n_ext : gidx);
                    pid_lo = (uint32_t)pid;
                    pid_hi = (uint32_t)(pid >> 32);
                    blk = 0;
                    events = 0;
                    W = 1;
                    launching = true;
                }
            }
            if (avail < cnt) {
                pool_next = fresh + (cnt - avail);
                pool_end = fresh + p.chunk;
            } else {
                pool_next += cnt;
            }
        }
        const bool absorbing = st == ST_ABS;
        const bool scattering = st == ST_SCAT;
        const bool ev = launching || absorbing || scattering;

        // absorption: deposit E into the shell; A_before locates this package's
        // slice [A_before, A_before + E] of the shell's absorbed power
        const double E = absorbing ? p.eps[src] * (double)W : 0.0;
        double A_before = 0.0;
        if (__ballot(absorbing)) A_before = fetch_add_energy<AGG>(p.A, i, E, absorbing);

        Rand4 r1{0, 0, 0, 0}, r2b{0, 0, 0, 0};
        if (ev) r1 = philox(blk++, pid_lo, pid_hi, (uint32_t)src, key0, key1);
        if (absorbing) r2b = philox(blk++, pid_lo, pid_hi, (uint32_t)src, key0, key1);

        // new frequency: source spectrum at launch, difference spectrum at re-emission
        int row = 0;
        if (absorbing) {
            const double astar = (A_before + (((double)r1.x + 0.5) * 0x1p-32) * E) * p.invM[i];
            row = count_le(G, n_t, (R)astar);
            if (row > n_t - 1) { row = n_t - 1; c_reabove++; }
            c_abs++;
        }
        if (launching || absorbing) {
            const R *tab = launching ? cdf + src * K : D + (size_t)row * K;
            k = min(count_le(tab, K, P<R>::uni(launching ? r1.x : r1.y)), K - 1);
            const Dust d = dust[k];
            kA = d.kA; kS = d.kS; gg = d.g; alb = d.alb;
        }

        // new direction: isotropic re-emission or Henyey-Greenstein scattering
        if (absorbing || scattering) {
            R r2 = b2 + t * t;
            R rr = P<R>::sqrt_(r2);
            R mun;
            if (absorbing) {
                mun = (R)2 * P<R>::uni(r1.z) - (R)1;
                if (p.reemit_uniform) {
                    const Shell s = sh[i];
                    const R rin = s.r_in;
                    const R rout = P<R>::sqrt_(s.r2_out);
                    const R c3 = rin * rin * rin + P<R>::uni(r2b.y) * (rout * rout * rout - rin * rin * rin);
                    rr = P<R>::cbrt_(c3);
                    r2 = rr * rr;
                }
            } else {
                c_scat++;
                const R mu = rr > (R)0 ? t * P<R>::rcp(rr) : (R)1;
                const R u0 = P<R>::uni(r1.x);
                R ct;
                if (gg > (R)-1e-6 && gg < (R)1e-6) {
                    ct = (R)2 * u0 - (R)1;
                } else {
                    const R f = ((R)1 - gg * gg) * P<R>::rcp((R)1 - gg + (R)2 * gg * u0);
                    ct = ((R)1 + gg * gg - f * f) * P<R>::rcp((R)2 * gg);
                    ct = ct > (R)1 ? (R)1 : (ct < (R)-1 ? (R)-1 : ct);
                }
                const R st2 = ((R)1 - ct) * ((R)1 + ct);
                const R sp2 = ((R)1 - mu) * ((R)1 + mu);
                const R sn = P<R>::sqrt_((st2 > (R)0 ? st2 : (R)0) * (sp2 > (R)0 ? sp2 : (R)0));
                mun = mu * ct + sn * P<R>::cos2pi(P<R>::uni(r1.y));
                mun = mun > (R)1 ? (R)1 : (mun < (R)-1 ? (R)-1 : mun);
            }
            t = rr * mun;
            b2 = r2 * ((R)1 - mun) * ((R)1 + mun);
        }

        // both free paths are redrawn after every event (Eq. 1)
        if (ev) {
            tauA = P<R>::nlog(P<R>::uni(absorbing ? r1.w : r1.z));
            tauS = P<R>::nlog(P<R>::uni(absorbing ? r2b.x : r1.w));
            st = ST_FLY;
        }

        // launch geometry and launch weights (Eqs. 2-3, Eq. 5, Eqs. 9-12)
        if (launching) {
            c_launch++;
            if (src == 0) {
                const R u1 = P<R>::uni(r1.y);
                R mu;
                if (p.k_bg == 0.5) {
                    mu = P<R>::sqrt_(u1);
                } else {
                    const R kb = (R)p.k_bg;
                    mu = P<R>::powr(u1, kb);
                    W = (R)2 * kb * P<R>::powr(mu, (R)2 - (R)1 / kb);
                }
                i = n - 1;
                t = -mu;
                b2 = ((R)1 - mu) * ((R)1 + mu);
            } else {
                i = 0;
                b2 = 0;
                t = sh[0].r_in;
                if (p.cavity) c_cross++;
            }
            if (p.ffi) {
                // extinction optical depth along the whole first ray
                const R kext = kA + kS;
                R tau0 = 0, tt = t;
                int ii = i;
                for (;;) {
                    const Shell s = sh[ii];
                    const bool inward = (tt < (R)0) && (b2 < s.r2_in);
                    const R arg = (inward ? s.r2_in : s.r2_out) - b2;
                    const R sq = P<R>::sqrt_(arg > (R)0 ? arg : (R)0);
                    const R tn = inward ? -sq : sq;
                    const R lb = tn - tt > (R)0 ? tn - tt : (R)0;
                    tau0 += kext * s.rho * lb;
                    tt = tn;
                    if (inward) {
                        if (ii == 0) tt = -tt; else ii--;
                    } else if (++ii == n) {
                        break;
                    }
                }
                if (!(tau0 > (R)0)) {
                    escape();
                } else {
                    const R pf = -P<R>::expm1_(-tau0);
                    ffi_esc += p.eps[src] * (double)W * (double)(((R)1) - pf);
                    W *= pf;
                    const R tau = -P<R>::log1p_(-P<R>::uni(r1.z) * pf);
                    if (P<R>::uni(r1.w) < alb) { tauS = tau * alb; tauA = P<R>::inf(); }
                    else { tauA = tau * ((R)1 - alb); tauS = P<R>::inf(); }
                }
            }
            W0 = W;
        }

        // weight floor (Sect. 2.2.1)
        if ((absorbing || scattering) && W < (R)p.w_floor * W0) {
            term += p.eps[src] * (double)W;
            c_floor++;
            st = ST_DEAD;
        }
    }

    // ---- flush per-lane counters: one atomic per wave and counter
    const unsigned long long cs[9] = {c_launch, c_cross, c_scat, c_abs, c_escape,
                                      c_direct, c_limit, c_floor, c_reabove};
    const int cidx[9] = {C_LAUNCH, C_CROSS, C_SCAT, C_ABS, C_ESCAPE, C_DIRECT, C_LIMIT, C_FLOOR, C_REEMIT_ABOVE};
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        const unsigned long long v = wave_sum_u64(cs[j]);
        if (lane == 0 && v) atomicAdd(&p.stats->cnt[cidx[j]], v);
    }
    const double ts[4] = {esc0, esc1, ffi_esc, term};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double v = wave_sum_f64(ts[j]);
        if (lane == 0 && v != 0.0) unsafeAtomicAdd(&p.stats->tally[j], v);
    }
}

template <bool AGG>
__global__ __launch_bounds__(kBlockFP32) void ire_trace_f32(TraceParams p) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = p.n, K = p.K, n_t = p.n_t;
    ShellF *s_sh = reinterpret_cast<ShellF *>(smem);
    DustF *s_dust = reinterpret_cast<DustF *>(s_sh + n);
    float *s_cdf = reinterpret_cast<float *>(s_dust + K);
    float *s_G = s_cdf + 2 * K;
    float *s_D = s_G + n_t;
    for (int j = threadIdx.x; j < n; j += blockDim.x) s_sh[j] = p.shf[j];
    for (int j = threadIdx.x; j < K; j += blockDim.x) s_dust[j] = p.dustf[j];
    for (int j = threadIdx.x; j < 2 * K; j += blockDim.x) s_cdf[j] = p.cdff[j];
    for (int j = threadIdx.x; j < n_t; j += blockDim.x) s_G[j] = p.Gf[j];
    const int nd = n_t * K;
    for (int j = threadIdx.x; j < nd; j += blockDim.x) s_D[j] = p.Df[j];
    __syncthreads();
    trace_body<float, AGG>(p, s_sh, s_dust, s_cdf, s_G, s_D);
}

template <bool AGG>
__global__ __launch_bounds__(256) void ire_trace_f64(TraceParams p) {
    trace_body<double, AGG>(p, p.shd, p.dustd, p.cdfd, p.Gd, p.Dd);
}

__global__ void ire_zero(double *A, int n, DevStats *st, int clear_counts) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    for (int j = tid; j < n * kAccStride; j += gridDim.x * blockDim.x) A[j] = 0.0;
    if (tid == 0) {
        st->cursor = 0;
        if (clear_counts) {
            for (int j = 0; j < 16; ++j) st->cnt[j] = 0;
            for (int j = 0; j < 8; ++j) st->tally[j] = 0.0;
        }
    }
}

__global__ void ire_cursor_reset(DevStats *st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) st->cursor = 0;
}

// A -> T per shell by log-log interpolation of the G(T) table; values outside
// the table are clamped to [t_min, t_max] and counted.
__global__ void ire_finalize(FinalizeParams p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n) return;
    const double A = p.A[(size_t)i * kAccStride];
    const double a = A * p.invM[i];
    double T;
    if (!(a >= p.Gd[0])) {
        T = p.t_min;
        atomicAdd(&p.stats->cnt[C_BELOW], 1ull);
    } else if (a > p.Gd[p.n_t - 1]) {
        T = p.t_max;
        atomicAdd(&p.stats->cnt[C_ABOVE], 1ull);
    } else {
        int j = count_le(p.Gd, p.n_t, a) - 1;
        j = j < 0 ? 0 : (j > p.n_t - 2 ? p.n_t - 2 : j);
        const double f = (log(a) - p.lnG[j]) / (p.lnG[j + 1] - p.lnG[j]);
        T = exp(p.lnT[j] + f * (p.lnT[j + 1] - p.lnT[j]));
    }
    p.A_out[i] = A;
    p.T_out[i] = T;
}

}  // namespace

size_t trace_lds_bytes(int n, int K, int n_t) {
    return (size_t)n * sizeof(ShellF) + (size_t)K * sizeof(DustF) + (size_t)2 * K * sizeof(float) +
           (size_t)n_t * sizeof(float) + (size_t)n_t * K * sizeof(float);
}

hipError_t trace_configure(int fp64, int aggregate, size_t lds) {
    if (fp64) return hipSuccess;
    const void *f = aggregate ? reinterpret_cast<const void *>(&ire_trace_f32<true>)
                              : reinterpret_cast<const void *>(&ire_trace_f32<false>);
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_trace(const TraceParams &p, int fp64, int aggregate, int grid, int block,
                        size_t lds, hipStream_t s) {
    if (fp64) {
        if (aggregate) hipLaunchKernelGGL(ire_trace_f64<true>, dim3(grid), dim3(block), 0, s, p);
        else hipLaunchKernelGGL(ire_trace_f64<false>, dim3(grid), dim3(block), 0, s, p);
    } else {
        if (aggregate) hipLaunchKernelGGL(ire_trace_f32<true>, dim3(grid), dim3(block), lds, s, p);
        else hipLaunchKernelGGL(ire_trace_f32<false>, dim3(grid), dim3(block), lds, s, p);
    }
    return hipGetLastError();
}

hipError_t launch_zero(double *A, int n, DevStats *st, int clear_counts, hipStream_t s) {
    if (A) {
        int blocks = (n * kAccStride + 255) / 256;
        if (blocks < 1) blocks = 1;
        if (blocks > 1024) blocks = 1024;
        hipLaunchKernelGGL(ire_zero, dim3(blocks), dim3(256), 0, s, A, n, st, clear_counts);
    } else {
        hipLaunchKernelGGL(ire_cursor_reset, dim3(1), dim3(64), 0, s, st);
    }
    return hipGetLastError();
}

hipError_t launch_finalize(const FinalizeParams &p, hipStream_t s) {
    const int blocks = (p.n + 255) / 256;
    hipLaunchKernelGGL(ire_finalize, dim3(blocks), dim3(256), 0, s, p);
    return hipGetLastError();
}

// The block size the FP32 tracer is compiled for.
int trace_block_fp32() { return kBlockFP32; }

}  // namespace ire
