// IRE photon-package tracer for gfx950 (MI355X).
//
// One lane follows one package at a time in a persistent wavefront; a lane
// whose package has left the cloud takes the next package index from a
// wave-private pool that is refilled from a global cursor in chunks.  Shell geometry is one-dimensional:
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
// Weighting: centre-weighted background directions (Eq. 5), forced first
// interaction (Eqs. 9-12), weighted re-emission and scattering directions and
// scaled free paths (Table 1, Eqs. 6-8), density-dependent absorption scaling.
//
// The difference-spectrum draw uses lookup tables: with the cumulative emission
// taken as linear in G(T) within a temperature bin, drawing a point a* uniformly
// in the slice [A_before, A_after]/M of absorbed power per mass, locating its bin
// in the G table and drawing the frequency from that bin's CDF of
// kappa_abs [B(T_hi) - B(T_lo)] w reproduces the difference spectrum, and the
// slices of all absorptions in a shell tile [0, A_final] in any order.  A_before
// is therefore the value returned by a returning FP64 atomic; the absorptions of
// a pass that fall in the same shell share one atomic, grouped per wave or per
// workgroup (AGG = 1, 2), each lane taking its own offset inside the group's
// deposit.  With accumulator groups (`replicas`), workgroup b adds into copy
// b mod R and reads its slices as R times that copy's running total.
//
// Random numbers: Philox4x32-10 (Salmon et al. 2011), key = seed, counter =
// (block, package id lo, package id hi, source); one block per event and a
// second one for an absorption, which the FP32 kernels draw only when its slice
// reaches across a bin edge of the G table or the re-emission radius is
// redrawn.  u = (x + 0.5) 2^-32.
//
// Two instantiations: float stepping with all tables in LDS, and double
// everywhere with tables read from global memory.  Absorbed-energy
// accumulators and package energies are FP64 in both.

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

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
    using KRec = float2;   // per shell: {k rho, 1 / (k rho)} of the scaled absorption clock
    // one 128-bit load of a shell record
    static __device__ __forceinline__ ShellF shell(const ShellF *q) {
        const float4 v = *reinterpret_cast<const float4 *>(q);
        return ShellF{v.x, v.y, v.z, v.w};
    }
    static __device__ __forceinline__ float uni(uint32_t x) {
        float u = __builtin_fmaf((float)x, 0x1p-32f, 0x1p-33f);
        return u < 0x1.fffffep-1f ? u : 0x1.fffffep-1f;
    }
    static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
    // u is a normal number in (0, 1): the hardware log2 needs no range reduction
    static __device__ __forceinline__ float nlog(float u) { return -0x1.62e430p-1f * __builtin_amdgcn_logf(u); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float cos2pi(float u) { return __builtin_amdgcn_cosf(u); }
    // a in (0, 1]: 2^(b log2 a) with the hardware log2 and exp2
    static __device__ __forceinline__ float powr(float a, float b) {
        return __builtin_amdgcn_exp2f(b * __builtin_amdgcn_logf(a));
    }
    static __device__ __forceinline__ float expm1_(float x) { return expm1f(x); }
    // log(1 + x), accurate for small |x| with the hardware logarithm: w = 1 + x
    // rounded, and log(w) x / (w - 1) cancels the rounding of w (Goldberg 1991,
    // Theorem 4); x > -1.  A few ulp, at a sixth of the instructions of log1pf.
    static __device__ __forceinline__ float log1p_(float x) {
        const float w = 1.0f + x;
        const float d = w - 1.0f;
        return d == 0.0f ? x : 0x1.62e430p-1f * __builtin_amdgcn_logf(w) * (x * __builtin_amdgcn_rcpf(d));
    }
    static __device__ __forceinline__ float cbrt_(float x) { return cbrtf(x); }
    static __device__ __forceinline__ float inf() { return __builtin_huge_valf(); }
    static __device__ __forceinline__ float exp_(float x) { return __expf(x); }
};

template <> struct P<double> {
    using Shell = ShellD;
    using Dust = DustD;
    using KRec = double2;
    static __device__ __forceinline__ ShellD shell(const ShellD *q) { return *q; }
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
    static __device__ __forceinline__ double exp_(double x) { return exp(x); }
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

// Number of entries of the increasing table t[0..n) that are <= x, found by
// scanning from a starting guess in either direction (exact for any start in
// [0, n]; a guide table makes the scan short).
template <typename T, typename X>
__device__ __forceinline__ int count_le_from(const T *t, int n, X x, int pos) {
    while (pos > 0 && (X)t[pos - 1] > x) --pos;
    while (pos < n && (X)t[pos] <= x) ++pos;
    return pos;
}

// count_le_from, also returning the entry the forward scan stopped at
// (t[pos] > x, infinite past the end), which the caller would otherwise read
// again.
template <typename T, typename X>
__device__ __forceinline__ int count_le_next(const T *t, int n, X x, int pos, X inf, X &next) {
    while (pos > 0 && (X)t[pos - 1] > x) --pos;
    X v = pos < n ? (X)t[pos] : inf;
    while (pos < n && v <= x) {
        ++pos;
        v = pos < n ? (X)t[pos] : inf;
    }
    next = v;
    return pos;
}

// Guide start for a in the G(T) table: bins uniform in log2 a.
__device__ __forceinline__ int g_guide(const uint16_t *gg, int n_t, float lg0, float scale, float a) {
    const float x = (__log2f(a) - lg0) * scale;
    const int b = x > 0.0f ? (x < (float)(n_t - 1) ? (int)x : n_t - 1) : 0;
    return gg[b];
}

// Henyey-Greenstein: cos(theta) by inversion of the cumulative law for uniform
// u, and the probability density of cos(theta) (Eq. 6).
template <typename R>
__device__ __forceinline__ R hg_cos(R g, R u) {
    if (g > (R)-1e-6 && g < (R)1e-6) return (R)2 * u - (R)1;
    const R f = ((R)1 - g * g) * P<R>::rcp((R)1 - g + (R)2 * g * u);
    const R c = ((R)1 + g * g - f * f) * P<R>::rcp((R)2 * g);
    return c > (R)1 ? (R)1 : (c < (R)-1 ? (R)-1 : c);
}

template <typename R>
__device__ __forceinline__ R hg_pdf(R g, R mu) {
    const R q = (R)1 + g * g - (R)2 * g * mu;
    return (R)0.5 * ((R)1 - g * g) * P<R>::rcp(q * P<R>::sqrt_(q));
}

// ---------------------------------------------------------------------------
// Wave-level helpers (wave64)

// Orders the LDS accesses of the wave's lanes before it against those after it
// (the hardware runs a wave's LDS operations in order; this keeps the compiler
// from moving them across).
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave's LDS scratch for grouping its absorptions by shell.
struct AggScratch {
    double sum[kAggSlots];
    int owner[kAggSlots];
};

// A workgroup's LDS scratch for grouping the absorptions of all its waves:
// per slot the key (shell and thread of the owner), the group sum (zero
// between passes) and the group base; two words for the workgroup's vote
// whether any wave still has work, used in alternate passes; and the quorum
// word: waves that ended the current sweep (low half, cleared every pass) and
// waves without packages left (high half).
struct WgScratch {
    double sum[kWgSlots];
    double base[kWgSlots];
    unsigned key[kWgSlots];
    unsigned busy[2];
    unsigned quorum;
    unsigned pad_;
};

// Before the first pass: group sums, votes and the quorum word start at zero.
__device__ __forceinline__ void wg_scratch_init(WgScratch *wg) {
    for (int j = threadIdx.x; j < kWgSlots; j += blockDim.x) wg->sum[j] = 0.0;
    if (threadIdx.x < 2) wg->busy[threadIdx.x] = 0u;
    if (threadIdx.x == 2) wg->quorum = 0u;
}

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

// Returning fetch-add of E into A[i] for the lanes with act set, in two halves
// so that independent work can run while the atomics are in flight: issue()
// sends them, complete() waits and hands each lane the value of A[i] just
// before its own deposit.  Every lane of the wave must call both.  With AGG,
// the lanes that hit the same shell are folded into one deposit by a group
// leader, and each member receives the leader's base plus its own offset
// inside the group's deposit, so that the members' slices tile the deposit.
// Groups form in the wave's LDS scratch first: every lane writes its lane id
// into the slot (shell mod kAggSlots) and reads back the winner; the lanes of
// the winner's shell add their energies to the slot's sum with returning LDS
// atomics (the returned value is the offset).  The few lanes whose slot went
// to another shell are grouped with ballots and shuffles.  All leaders then
// issue their atomics as one instruction: one round trip per call, however
// many shells the wave hits.
struct PendingAdd {
    double raw = 0.0;     // the atomic's return value (group leaders, or every acting lane without AGG)
    double ex = 0.0;      // this lane's offset inside its group's deposit
    int leader_of = 0;    // lane holding this lane's group base
};

template <int AGG>
__device__ __forceinline__ PendingAdd fetch_add_issue(double *A, int i, double E, bool act, AggScratch *ws) {
    PendingAdd q;
    const int lane = __lane_id();
    q.leader_of = lane;
    if constexpr (AGG == 0) {
        if (act) q.raw = unsafeAtomicAdd(&A[(size_t)i * kAccStride], E);
        return q;
    } else {
        // groups by slot; the wave's LDS operations complete in program order
        const int slot = i & (kAggSlots - 1);
        if (act) ws->owner[slot] = lane;
        wave_sync_lds();
        const int owner = act ? ws->owner[slot] : lane;
        const bool member = act && __shfl(i, owner, kWave) == i;
        if (member && owner == lane) ws->sum[slot] = 0.0;
        wave_sync_lds();
        if (member) q.ex = atomicAdd(&ws->sum[slot], E);
        wave_sync_lds();
        double dep = 0.0;     // the leader's deposit: its group's total energy
        bool lead = false;
        if (member && owner == lane) {
            dep = ws->sum[slot];
            lead = true;
        }
        if (member) q.leader_of = owner;
        // the rest: groups by ballots over the lanes whose slot holds another shell
        const bool rest = act && !member;
        unsigned long long pending = __ballot(rest);
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const int s = __shfl(i, leader, kWave);
            const unsigned long long grp = __ballot(rest && i == s);
            pending &= ~grp;
            const bool mine = (grp >> lane) & 1ull;
            if (__popcll(grp) == 1) {
                if (mine) {
                    dep = E;
                    lead = true;
                }
            } else {
                const double v = mine ? E : 0.0;
                const double e = wave_excl_scan(v);
                const double tot = __shfl(e + v, kWave - 1, kWave);
                if (mine) {
                    q.ex = e;
                    q.leader_of = leader;
                }
                if (lane == leader) {
                    dep = tot;
                    lead = true;
                }
            }
        }
        if (lead) q.raw = unsafeAtomicAdd(&A[(size_t)i * kAccStride], dep);
        return q;
    }
}

template <int AGG>
__device__ __forceinline__ double fetch_add_complete(const PendingAdd &q, bool act) {
    if constexpr (AGG == 0) {
        return act ? q.raw : 0.0;
    } else {
        const double base = __shfl(q.raw, q.leader_of, kWave);
        return act ? base + q.ex : 0.0;
    }
}

// The same for all waves of a workgroup together (aggregate = 2): the lanes of
// every wave that hit a shell are folded into one deposit, so one atomic per
// shell and pass leaves the workgroup.  Slots are keyed by shell and thread
// (shell mod kWgSlots), claimed by the caller before a workgroup barrier; the
// lanes whose slot went to another shell fall back to their wave's ballot
// grouping.  Every thread of the workgroup must call both halves in every pass
// (they hold workgroup barriers).
struct PendingWg {
    PendingAdd w;          // the wave-level result for the lanes outside the slot groups
    double off = 0.0;      // offset inside the slot group's deposit
    int slot = 0;
    bool member = false, owner = false;
};

__device__ __forceinline__ PendingWg fetch_add_issue_wg(double *A, int i, double E, bool act, WgScratch *wg) {
    // every acting lane has written its key ((i << 10) | thread, i < 2^22) to
    // slot i mod kWgSlots before a workgroup barrier; one key per slot won
    PendingWg g;
    const int tid = (int)threadIdx.x;
    g.slot = i & (kWgSlots - 1);
    const unsigned kr = act ? wg->key[g.slot] : 0u;
    g.member = act && (int)(kr >> 10) == i;
    g.owner = g.member && (int)(kr & 1023u) == tid;
    // the slot's sum is zero here: it starts at zero and its last owner cleared it
    if (g.member) g.off = atomicAdd(&wg->sum[g.slot], E);
    __syncthreads();
    // slot owners deposit their group's total; the rest group within their wave
    const bool rest = act && !g.member;
    PendingAdd w;
    const int lane = __lane_id();
    w.leader_of = lane;
    double dep = 0.0;
    bool lead = false;
    if (g.owner) {
        dep = wg->sum[g.slot];
        lead = true;
    }
    unsigned long long pending = __ballot(rest);
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const int s = __shfl(i, leader, kWave);
        const unsigned long long grp = __ballot(rest && i == s);
        pending &= ~grp;
        const bool mine = (grp >> lane) & 1ull;
        const double v = mine ? E : 0.0;
        const double e = wave_excl_scan(v);
        const double tot = __shfl(e + v, kWave - 1, kWave);
        if (mine) {
            w.ex = e;
            w.leader_of = leader;
        }
        if (lane == leader) {
            dep = tot;
            lead = true;
        }
    }
    if (lead) w.raw = unsafeAtomicAdd(&A[(size_t)i * kAccStride], dep);
    g.w = w;
    return g;
}

__device__ __forceinline__ double fetch_add_complete_wg(const PendingWg &g, bool act, WgScratch *wg) {
    if (g.owner) wg->base[g.slot] = g.w.raw;
    const double wbase = __shfl(g.w.raw, g.w.leader_of, kWave);
    __syncthreads();
    if (g.owner) wg->sum[g.slot] = 0.0;     // every member has its offset: clear for the next pass
    if (!act) return 0.0;
    return g.member ? wg->base[g.slot] + g.off : wbase + g.w.ex;
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

// Per-lane event counters and energy tallies (flushed once per wave).
struct LaneCounters {
    uint32_t launch = 0, sent = 0, scat = 0, abs = 0, escape = 0, direct = 0, limit = 0, floor = 0,
             reabove = 0;
    // steps that moved a package, counted per wave (the same value in every
    // lane); the crossings are these less the steps into the sentinel (`sent`)
    unsigned long long steps = 0;
    uint32_t passes = 0;           // event passes of this wave (the same value in every lane)
    unsigned long long slots = 0;  // lane slots of its crossing sweeps: 64 per wave-level step
    double esc0 = 0.0, esc1 = 0.0, ffi = 0.0, term = 0.0;
};

// One cloud model as the tracer sees it.
template <typename R>
struct ModelCtx {
    const typename P<R>::Shell *sh;  // [empty cavity] + n shells + sentinel beyond the surface
    int n, cav;
    const double *invM;              // n: 1 / shell mass
    double *A;                       // n absorbed-energy accumulators, stride kAccStride
    double a_scale;                  // running total -> whole-run estimate (the number of groups)
    double eps[2];                   // package energy per source
    unsigned long long n_ext, n_ps;  // packages to trace per source
    unsigned long long pid0[2];      // first package id per source
    unsigned long long seed;
};

// Method options shared by every model of a launch.
struct MethodOpts {
    double k_bg;
    int ffi, reemit_uniform, batch;
    int quorum;                      // workgroup grouping: see the crossing sweep
    double w_floor;
    unsigned long long max_events;
    // weighted sampling (Table 1): HG re-emission / scattering directions
    // about the reference direction, scaled free paths
    int use_g_E, use_g_S;
    double g_E, g_S, k_A, k_S;
};

// Trace every package of one model with the lanes of this wave.  Package
// indices come from `cursor` (global or LDS memory) `chunk` at a time; the
// call returns when the cursor is exhausted and every lane is idle.
template <typename R, int AGG, int WT>
__device__ __forceinline__ void trace_model(const ModelCtx<R> &mc, const MethodOpts &o,
                                            const typename P<R>::Dust *dust, const R *cdf,
                                            const R *G, const R *D, int K, int n_t, int ldD,
                                            const unsigned char *guide, float g_lg0, float g_scale,
                                            const typename P<R>::KRec *rk,
                                            unsigned long long *cursor, unsigned long long chunk,
                                            bool lane_off, LaneCounters &lc, double *sed, AggScratch *agg,
                                            WgScratch *wg) {
    using Shell = typename P<R>::Shell;
    using Dust = typename P<R>::Dust;
    using KRec = typename P<R>::KRec;
    // WT: 0 plain; 1 weighted sampling (Table 1) with constant free-path
    // scaling; 2 also an absorption scaling that depends on the shell's
    // density, so the two free paths fall at different rates in every shell
    // and each flight carries two columns
    constexpr bool WTD = WT >= 1;
    constexpr bool KRHO = WT == 2;
    // lane status: in flight, parked at an interaction (or at the surface),
    // without a package, finished (no packages left)
    enum : int { ST_FLY = 0, ST_EVT = 1, ST_DEAD = 3, ST_DONE = 4 };
    // Shell table: [empty cavity] + the n shells + a sentinel beyond the surface.
    // A flight that leaves the cloud enters the sentinel, whose infinite density
    // ends the flight there; the event pass recognises it as an escape.
    const Shell *const sh = mc.sh;
    const int cav = mc.cav;
    const int n_int = mc.n + cav;
    const uint32_t key0 = (uint32_t)mc.seed, key1 = (uint32_t)(mc.seed >> 32);
    const unsigned long long total = mc.n_ext + mc.n_ps;
    const int lane = __lane_id();
    const int batch = o.batch > 0 ? o.batch : 1;
    const Shell *const sentinel = sh + n_int;
    const uint16_t *const gguide = reinterpret_cast<const uint16_t *>(guide);

    unsigned long long pool_next = 0, pool_end = 0;  // wave-uniform

    // package state, one package per lane
    int st = lane_off ? ST_DONE : ST_DEAD;
    const Shell *ps = sh;          // current shell
    Shell cur = P<R>::shell(sh);   // its record, kept in registers while the package flies
    KRec curk{};                   // its scaled absorption rate (k_A(rho) only)
    if constexpr (KRHO) curk = rk[0];
    int k = 0, src = 0;
    R b2 = 0, t = 0, W = 1, W0 = 1;
    R sig = 0;                     // column (rho-weighted length) left before the next interaction
    double eps = 0.0;              // package energy of the package's source
    bool ev_abs = false;           // that interaction is an absorption (else a scattering)
    uint32_t pid_lo = 0, pid_hi = 0, blk = 0;
    unsigned long long events = 0;
    // scaled free paths (Eq. 8): the flight's drawn column and whether its
    // free paths were scaled (not for the forced first flight)
    const bool kscale = KRHO || (WTD && (o.k_A != 1.0 || o.k_S != 1.0));
    const R kA1 = (R)(o.k_A - 1.0), kS1 = (R)(o.k_S - 1.0);
    const R inv_kA = (R)(1.0 / o.k_A), inv_kS = (R)(1.0 / o.k_S);
    R sig0 = 0;
    bool kw = false;
    // k_A(rho): the absorption clock's column left (units of k rho l) and drawn;
    // sig, sig0 then hold the scattering clock's (units of rho l, infinite where
    // the dust does not scatter); colT is the rho l column the flight has crossed
    R sigA = 0, sigA0 = 0, colT = 0;

    // FFI: the extinction column (per unit kappa) of the ray from the centre to the
    // surface, the first flight of every point-source package, summed once here in
    // the order of an outward walk through the shells
    R col_centre = 0;
    if (o.ffi && mc.n_ps > 0) {
        R r_in = 0;
        for (const Shell *q = sh; q < sentinel; ++q) {
            const Shell s = *q;
            const R r_out = P<R>::sqrt_(s.r2_out);
            col_centre += s.rho * (r_out - r_in);
            r_in = r_out;
        }
    }

    // One boundary step of a package in flight (Eq. 4), computed for every
    // lane and committed only where the package is in flight.  Both free
    // paths fall by kappa rho l along a flight, so the one that runs out
    // first is fixed when they are drawn: the flight carries the smaller of
    // tau_A / kappa_A and tau_S / kappa_S as a column of rho-weighted length
    // and the type of its interaction.  The shell a crossing leads into is
    // known before the crossing is computed (inward while the ray approaches
    // its tangent point inside the inner sphere, outward otherwise), so its
    // record is requested first and its LDS latency overlaps the arithmetic.
    // A package that does not cross parks with t and sig unchanged; the event
    // pass moves it to the interaction point.  `fly` marks the packages in
    // flight during a crossing sweep, held as the wave's lane mask.
    // In the FP32 kernels the record of the shell just entered replaces the
    // current one in every lane: a lane that did not move stops flying, and
    // the event pass reloads its record from `ps`; the LDS pad record below
    // the table keeps such a lane's stale reads in bounds.
    unsigned long long fly = 0;    // wave-uniform
    unsigned long long tneg = 0;   // wave-uniform: lanes with t < 0 (FP32 sweeps)
    int vote = 0;                  // workgroup grouping: the vote word of this pass
    uint32_t sweep_steps = 0;      // moving steps of the current sweep (a sweep ends before 2^32)
    constexpr bool kLoose = std::is_same<R, float>::value;
    auto step = [&]() {
        bool inward;
        if constexpr (kLoose) {
            // a flight approaches its tangent point (t < 0) exactly while its
            // crossings so far went inward, so the FP32 kernels carry the mask
            // of those lanes from step to step instead of comparing t
            tneg &= __builtin_amdgcn_ballot_w64(b2 < cur.r2_in);
            inward = __builtin_amdgcn_inverse_ballot_w64(tneg);
        } else {
            inward = (t < (R)0) && (b2 < cur.r2_in);
        }
        const Shell *const pn = inward ? ps - 1 : ps + 1;
        const Shell nx = P<R>::shell(pn);
        KRec nxk{};
        if constexpr (KRHO) nxk = rk[pn - sh];
        // the FP32 kernels issue the record's load before the step's arithmetic
        // (the scheduler would otherwise place it after the square root)
        if constexpr (kLoose) __builtin_amdgcn_sched_barrier(0);
        const R arg = (inward ? cur.r2_in : cur.r2_out) - b2;
        // arg >= 0 but for rounding at a tangent point or on a boundary: the FP32
        // kernels take |arg| (a free source modifier of the square root, within
        // rounding of the clamp), the FP64 ones clamp at 0
        R sq;
        if constexpr (kLoose) sq = P<R>::sqrt_(__builtin_fabsf(arg));
        else sq = P<R>::sqrt_(arg > (R)0 ? arg : (R)0);
        const R tn = inward ? -sq : sq;
        const R ds = cur.rho * (tn - t);
        bool cross = ds < sig;
        R dsA = 0;
        if constexpr (KRHO) {
            dsA = curk.x * (tn - t);
            cross = cross && dsA < sigA;
        }
        // the lanes that cross, as a mask first (a compare's mask needs no
        // per-lane boolean), then as the per-lane condition of the selects
        fly &= __ballot(cross);
        const bool mv = __builtin_amdgcn_inverse_ballot_w64(fly);
        sig = mv ? sig - ds : sig;
        if constexpr (KRHO) {
            sigA = mv ? sigA - dsA : sigA;
            colT = mv ? colT + ds : colT;
        }
        t = mv ? tn : t;
        ps = mv ? pn : ps;
        sweep_steps += (uint32_t)__popcll(fly);
        // keep the compiler from hoisting the use of the record (and with it
        // the wait for its LDS read) above the step's arithmetic
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (kLoose) {
            cur = nx;
            if constexpr (KRHO) curk = nxk;
        } else {
            cur.r2_in = mv ? nx.r2_in : cur.r2_in;
            cur.r2_out = mv ? nx.r2_out : cur.r2_out;
            cur.rho = mv ? nx.rho : cur.rho;
            cur.inv_rho = mv ? nx.inv_rho : cur.inv_rho;
            if constexpr (KRHO) {
                curk.x = mv ? nxk.x : curk.x;
                curk.y = mv ? nxk.y : curk.y;
            }
        }
    };

    // The event pass: escapes, the event-count limit, refills from the wave's
    // package pool, launches, scatterings and absorptions with immediate
    // re-emission, then new free paths.
    // The first part of an event pass: parked packages move to their interaction
    // points and take the weights of their flights' outcomes.
    auto pre_event = [&]() {
            if constexpr (kLoose) {
                cur = P<R>::shell(ps);
                if constexpr (KRHO) curk = rk[ps - sh];
            }
            // a parked package still stands where its last step began: move it
            // along the column left to the interaction point
            if constexpr (KRHO) {
                // two columns: the clock that runs out first in this shell fires
                if (st == ST_EVT) {
                    if (kw) {
                        const bool esc = ps == sentinel;
                        const R lS = sig * cur.inv_rho, lA = sigA * curk.y;
                        const R lev = lA < lS ? lA : lS;
                        ev_abs = lA <= lS;
                        t += lev;
                        // weight: e^{modified - true absorption depth} e^{(k_S - 1) tau_S} and the
                        // fired clock's 1/k (1/k_i = rho / (k rho) of this shell)
                        const Dust dk = dust[k];
                        const R cS = esc ? colT : colT + cur.rho * lev;
                        const R cA = esc ? sigA0 - sigA : sigA0 - sigA + curk.x * lev;
                        R f = P<R>::exp_(dk.kA * (cA - cS) + kS1 * dk.kS * cS);
                        if (!esc) f *= ev_abs ? cur.rho * curk.y : inv_kS;
                        W *= f;
                    } else {
                        t += sig * cur.inv_rho;   // a forced first flight: one column, type drawn
                    }
                }
            } else {
                if (st == ST_EVT) t += sig * cur.inv_rho;
            }
            // scaled free paths: the weight of the flight's outcome, the fired
            // clock's (1/k) e^{(k-1) tau} times the survival ratio e^{(k'-1) tau'}
            // of the other (both survival ratios at escape); tau = kappa x column
            if (WTD && !KRHO && kscale && st == ST_EVT && kw) {
                const Dust dk = dust[k];
                const bool esc = ps == sentinel;
                const R c = esc ? sig0 - sig : sig0;
                R f = P<R>::exp_((kA1 * dk.kA + kS1 * dk.kS) * c);
                if (!esc) f *= ev_abs ? inv_kA : inv_kS;
                W *= f;
            }
    };

    auto event_pass = [&]() {
            const int i = (int)(ps - sh);        // internal shell index
            bool absorbing = false, scattering = false;
            if (st == ST_EVT) {
                if (ps == sentinel) {
                    // the flight left the cloud (the step into the sentinel is no crossing)
                    const double e = eps * (double)W;
                    if (src == 0) lc.esc0 += e; else lc.esc1 += e;
                    if (sed) {
                        // escaping spectrum per source and frequency (LDS, this workgroup)
                        atomicAdd(&sed[src * K + k], e);
                        if (events == 0) atomicAdd(&sed[2 * K + src * K + k], e);
                    }
                    lc.escape++;
                    lc.sent++;
                    if (events == 0) lc.direct++;
                    st = ST_DEAD;
                } else if (events >= o.max_events) {
                    lc.term += eps * (double)W;
                    lc.limit++;
                    st = ST_DEAD;
                } else {
                    events++;
                    absorbing = ev_abs;
                    scattering = !ev_abs;
                }
            }

            // refill lanes without a package from the wave-private pool, which takes
            // `chunk` package indices from the global cursor at a time
            bool launching = false;
            const unsigned long long need = __ballot(st == ST_DEAD);
            if (need) {
                const unsigned long long cnt = __popcll(need);
                const unsigned long long avail = pool_end - pool_next;
                unsigned long long fresh = 0;
                if (avail < cnt) {
                    const int leader = __ffsll((long long)need) - 1;
                    if (lane == leader) fresh = atomicAdd(cursor, chunk);
                    fresh = __shfl(fresh, leader, kWave);
                }
                if (st == ST_DEAD) {
                    const unsigned long long rank = __popcll(need & __lanemask_lt());
                    const unsigned long long gidx = rank < avail ? pool_next + rank : fresh + (rank - avail);
                    if (gidx >= total) {
                        st = ST_DONE;
                    } else {
                        src = gidx < mc.n_ext ? 0 : 1;
                        const unsigned long long pid = (src ? mc.pid0[1] + (gidx - mc.n_ext) : mc.pid0[0] + gidx);
                        eps = src ? mc.eps[1] : mc.eps[0];
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
                    pool_end = fresh + chunk;
                } else {
                    pool_next += cnt;
                }
            }
            const bool ev = launching || absorbing || scattering;

            // absorption: deposit E into the shell; A_before locates this package's
            // slice [A_before, A_before + E] of the shell's absorbed power
            const double E = absorbing ? eps * (double)W : 0.0;
            const double invM = absorbing ? mc.a_scale * mc.invM[i - cav] : 0.0;   // issued before the atomic's round trip
            // the atomics go out first; the shared Philox block is computed while they are in flight
            const bool any_abs = __ballot(absorbing) != 0;
            PendingAdd pend;
            PendingWg pwg;
            if constexpr (AGG == 2) pwg = fetch_add_issue_wg(mc.A, i - cav, E, absorbing, wg);
            else if (any_abs) pend = fetch_add_issue<AGG>(mc.A, i - cav, E, absorbing, agg);

            Rand4 r1{0, 0, 0, 0}, r2b{0, 0, 0, 0};
            if (ev) r1 = philox(blk++, pid_lo, pid_hi, (uint32_t)src, key0, key1);
            double A_before = 0.0;
            if constexpr (AGG == 2) A_before = fetch_add_complete_wg(pwg, absorbing, wg);
            else if (any_abs) A_before = fetch_add_complete<AGG>(pend, absorbing);

            // re-emission: a* uniform in the package's slice [A_before, A_before + E] / M
            // selects the G(T) bin whose difference spectrum is drawn.  A slice almost
            // never reaches across a bin edge (it is ~1e-6 of the shell's total), and
            // then the bin does not depend on a*.  The FP32 kernels use that: a* is
            // drawn only for a slice that does reach across, so the first Philox block
            // usually covers all five draws (a* or tau_S, frequency, direction,
            // tau_A).  The FP64 kernels take the plain layout of two blocks per
            // absorption, (a*, frequency, direction, tau_A) and (tau_S, re-emission
            // radius), whether or not a* changes the bin: the same draws and the
            // same distribution, one more block.
            constexpr bool kTwoBlocks = std::is_same<R, double>::value;
            int row = 0;
            bool straddle = false;
            if (absorbing) {
                const R alo = (R)(A_before * invM), ahi = (R)((A_before + E) * invM);
                R g_next;
                row = count_le_next(G, n_t, alo, g_guide(gguide, n_t, g_lg0, g_scale, (float)alo), P<R>::inf(), g_next);
                straddle = g_next <= ahi;
                lc.abs++;
            }
            if (absorbing && (kTwoBlocks || straddle || o.reemit_uniform))
                r2b = philox(blk++, pid_lo, pid_hi, (uint32_t)src, key0, key1);
            if (absorbing) {
                if (straddle) {
                    const double astar = (A_before + (((double)r1.x + 0.5) * 0x1p-32) * E) * invM;
                    row = count_le_from(G, n_t, (R)astar, row);
                }
                if (row > n_t - 1) { row = n_t - 1; lc.reabove++; }
            }
            if (launching || absorbing) {
                const R *tab = launching ? cdf + src * K : D + (size_t)row * ldD;
                const R u = P<R>::uni(launching ? r1.x : r1.y);
                k = min(count_le4(tab, K, u), K - 1);
            }
            const Dust d = dust[k];

            // new direction: isotropic re-emission or Henyey-Greenstein scattering
            if (absorbing || scattering) {
                R r2 = b2 + t * t;
                R rr = P<R>::sqrt_(r2);
                R mun;
                if (absorbing) {
                    if (WTD && o.use_g_E) {
                        // Eq. 6: cosine about the reference direction (inwards for the
                        // external field, outwards for the point source) from HG(g_E),
                        // weight = isotropic density / HG density
                        const R gE = (R)o.g_E;
                        const R mup = hg_cos(gE, P<R>::uni(r1.z));
                        W *= (R)0.5 * P<R>::rcp(hg_pdf(gE, mup));
                        mun = src == 0 ? -mup : mup;
                    } else {
                        mun = (R)2 * P<R>::uni(r1.z) - (R)1;
                    }
                    if (o.reemit_uniform) {
                        const Shell s = cur;
                        const R rin = P<R>::sqrt_(s.r2_in);
                        const R rout = P<R>::sqrt_(s.r2_out);
                        const R c3 = rin * rin * rin + P<R>::uni(r2b.y) * (rout * rout * rout - rin * rin * rin);
                        rr = P<R>::cbrt_(c3);
                        r2 = rr * rr;
                    }
                } else {
                    lc.scat++;
                    const R mu = rr > (R)0 ? t * P<R>::rcp(rr) : (R)1;
                    const R sp2 = ((R)1 - mu) * ((R)1 + mu);
                    if (WTD && o.use_g_S) {
                        // Eq. 7 (a ratio of densities): the new cosine about the reference
                        // direction from HG(g_S), the azimuth about the radius vector
                        // uniform from the plane of the old direction and the radius
                        // vector; weight = dust HG density at the scattering angle / HG(g_S)
                        const R gS = (R)o.g_S;
                        const R mup = hg_cos(gS, P<R>::uni(r1.x));
                        mun = src == 0 ? -mup : mup;
                        const R sn2 = ((R)1 - mun) * ((R)1 + mun);
                        const R ct = mu * mun + P<R>::sqrt_((sp2 > (R)0 ? sp2 : (R)0) * (sn2 > (R)0 ? sn2 : (R)0)) *
                                                    P<R>::cos2pi(P<R>::uni(r1.y));
                        W *= hg_pdf((R)d.g, ct > (R)1 ? (R)1 : (ct < (R)-1 ? (R)-1 : ct)) * P<R>::rcp(hg_pdf(gS, mup));
                    } else {
                        const R ct = hg_cos((R)d.g, P<R>::uni(r1.x));
                        const R st2 = ((R)1 - ct) * ((R)1 + ct);
                        const R sn = P<R>::sqrt_((st2 > (R)0 ? st2 : (R)0) * (sp2 > (R)0 ? sp2 : (R)0));
                        mun = mu * ct + sn * P<R>::cos2pi(P<R>::uni(r1.y));
                    }
                    mun = mun > (R)1 ? (R)1 : (mun < (R)-1 ? (R)-1 : mun);
                }
                t = rr * mun;
                b2 = r2 * ((R)1 - mun) * ((R)1 + mun);
            }

            // both free paths are redrawn after every event (Eq. 1), from
            // k e^{-k tau} when scaled (Eq. 8)
            R tauA = P<R>::nlog(P<R>::uni(absorbing ? r1.w : r1.z)) * inv_kA;
            R tauS = P<R>::nlog(P<R>::uni(absorbing ? ((kTwoBlocks || straddle) ? r2b.x : r1.x) : r1.w)) * inv_kS;
            bool kw_new = kscale;

            // launch geometry and launch weights (Eqs. 2-3, Eq. 5, Eqs. 9-12)
            if (launching) {
                lc.launch++;
                if (src == 0) {
                    const R u1 = P<R>::uni(r1.y);
                    R mu;
                    if (o.k_bg == 0.5) {
                        mu = P<R>::sqrt_(u1);
                    } else {
                        const R kb = (R)o.k_bg;
                        // mu^(2 - 1/k) = mu^2 / u since mu^(1/k) = u
                        mu = P<R>::powr(u1, kb);
                        W = (R)2 * kb * mu * mu * P<R>::rcp(u1);
                    }
                    ps = sentinel - 1;
                    t = -mu;
                    b2 = ((R)1 - mu) * ((R)1 + mu);
                } else {
                    ps = sh;            // the centre (inside the cavity shell when there is one)
                    b2 = 0;
                    t = 0;
                }
                if (o.ffi) {
                    // extinction optical depth along the whole first ray.  Its shells are
                    // known in advance (inward from the surface down to the shell of the
                    // tangent point and out again), so each record is requested one shell
                    // ahead of its use.  The outward half of an inward ray mirrors its
                    // inward half; the radial ray from the centre is the same for all.
                    R col = 0;
                    if (src == 0) {
                        const Shell *q = sentinel - 1;
                        Shell s = *q;
                        const R a0 = s.r2_out - b2;
                        R s_out = P<R>::sqrt_(a0 > (R)0 ? a0 : (R)0);
                        for (;;) {
                            const Shell nx = *(q > sh ? q - 1 : q);
                            // the innermost record has r2_in = 0, so the loop ends there at the latest
                            const bool tangent = !(b2 < s.r2_in);
                            const R s_in = tangent ? (R)0 : P<R>::sqrt_(s.r2_in - b2);
                            col += s.rho * (s_out - s_in);
                            if (tangent) break;
                            s_out = s_in;
                            s = nx;
                            --q;
                        }
                        col *= (R)2;
                    } else {
                        col = col_centre;
                    }
                    const R tau0 = d.kext * col;
                    if (!(tau0 > (R)0)) {
                        // no matter on the ray: the package leaves untouched
                        if (src == 0) lc.esc0 += eps * (double)W; else lc.esc1 += eps * (double)W;
                        if (sed) {
                            atomicAdd(&sed[src * K + k], eps * (double)W);
                            atomicAdd(&sed[2 * K + src * K + k], eps * (double)W);
                        }
                        lc.escape++;
                        lc.direct++;
                        launching = false;
                        st = ST_DEAD;
                    } else {
                        const R pf = -P<R>::expm1_(-tau0);
                        const double unforced = eps * (double)W * (double)(((R)1) - pf);
                        lc.ffi += unforced;
                        if (sed) {
                            // the unforced fraction leaves unscattered at the launch frequency
                            atomicAdd(&sed[src * K + k], unforced);
                            atomicAdd(&sed[2 * K + src * K + k], unforced);
                        }
                        R tau;
                        if (WTD && o.ffi == 2) {
                            // Eqs. 10, 12 in absorption depth: the interaction point is
                            // drawn in absorption depth tA < tau0 (1 - a); its extinction
                            // depth is tA / (1 - a); weight = ratio of the densities of
                            // the point in extinction depth
                            const R a1 = (R)1 - d.alb;
                            const R pA = -P<R>::expm1_(-tau0 * a1);
                            const R tA = -P<R>::log1p_(-P<R>::uni(r1.z) * pA);
                            tau = tA * P<R>::rcp(a1);
                            W *= pA * P<R>::rcp(a1) * P<R>::exp_(tA - tau);
                        } else {
                            W *= pf;
                            tau = -P<R>::log1p_(-P<R>::uni(r1.z) * pf);
                        }
                        if (P<R>::uni(r1.w) < d.alb) { tauS = tau * d.alb; tauA = P<R>::inf(); }
                        else { tauA = tau * ((R)1 - d.alb); tauS = P<R>::inf(); }
                        kw_new = false;
                    }
                }
                W0 = W;
            }

            // weight floor (Sect. 2.2.1)
            if ((absorbing || scattering) && W < (R)o.w_floor * W0) {
                lc.term += eps * (double)W;
                lc.floor++;
                st = ST_DEAD;
            } else if (launching || absorbing || scattering) {
                const R sA = tauA * d.inv_kA;
                const R sS = tauS * d.inv_kS;
                ev_abs = sA <= sS;
                sig = ev_abs ? sA : sS;
                if constexpr (KRHO) {
                    // scaled flights carry both columns; the forced first flight one
                    sigA = kw_new ? sA : P<R>::inf();
                    sig = kw_new ? sS : sig;
                    sigA0 = sigA;
                    colT = 0;
                }
                sig0 = sig;
                kw = kw_new;
                st = ST_FLY;
            }
    };

    // workgroup grouping: the waves of the workgroup; the quorum word's high half
    // counts those without packages left
    const int n_waves = (int)(blockDim.x / kWave);
    bool wave_done = false;
    constexpr int kStepsPerCheck = AGG == 1 ? 16 : 8;
    for (;;) {
        // ---- crossing sweep: packages in flight step from boundary to boundary;
        // a package that reaches its interaction parks, and the wave stops stepping
        // when enough of its packages are parked to process their events together.
        // Several steps per check (a step of a parked package changes nothing):
        // sixteen with per-wave grouping, eight with workgroup grouping, where
        // stopping soon after the quorum matters more, and with one atomic per
        // lane (measured: fewer checks cost less than the extra steps).  With
        // workgroup grouping every wave waits for the others at the pass, so a
        // wave also stops once `quorum` of the waves that still have packages have
        // ended their sweeps (a wave counts itself only after its own sweep, so
        // at least one wave always ends by its own count).
        {
            const int live = __popcll(__ballot(st != ST_DONE));
            const int want = batch < live ? batch : (live > 0 ? live : 1);
            fly = __ballot(st == ST_FLY);
            tneg = __ballot(t < (R)0);
            sweep_steps = 0;
            if constexpr (AGG == 2) {
                if (live == 0 && !wave_done) {
                    wave_done = true;
                    if (lane == 0) atomicAdd(&wg->quorum, 1u << 16);
                }
            }
            bool stop = false;
            for (;;) {
                const int nfly = __popcll(fly);
                if (nfly == 0 || live - nfly >= want || stop) break;
                unsigned qw = 0;
                if constexpr (AGG == 2) qw = __hip_atomic_load(&wg->quorum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
                for (int u = 0; u < kStepsPerCheck; ++u) step();
                lc.slots += kStepsPerCheck * kWave;
                if constexpr (AGG == 2) {
                    // with `quorum` or fewer waves left with packages the count is never
                    // reached (the others can end at most with_pkgs - 1 sweeps)
                    qw = __builtin_amdgcn_readfirstlane(qw);
                    const int with_pkgs = n_waves - (int)(qw >> 16);
                    stop = (int)(qw & 0xffffu) >= (o.quorum < with_pkgs ? o.quorum : with_pkgs);
                }
            }
            st = (st == ST_FLY && !__builtin_amdgcn_inverse_ballot_w64(fly)) ? (int)ST_EVT : st;
            lc.steps += sweep_steps;
            if constexpr (AGG == 2) {
                if (!wave_done && lane == 0) atomicAdd(&wg->quorum, 1u);
            }
        }
        // nothing in flight, nothing parked: all packages done (with workgroup
        // grouping, the waves of the workgroup run their passes together until
        // every wave is done)
        const bool busy = __ballot(st != ST_DONE && st != ST_FLY) != 0;
        if constexpr (AGG == 2) {
            // the absorptions of this pass claim their slots before the barrier of the
            // vote (the pass's absorbing lanes, exactly as the event pass decides them)
            pre_event();
            if (st == ST_EVT && ps != sentinel && events < o.max_events && ev_abs) {
                const int ia = (int)(ps - sh) - cav;
                wg->key[ia & (kWgSlots - 1)] = ((unsigned)ia << 10) | (unsigned)threadIdx.x;
            }
            // the vote of this pass goes to busy[vote]; the other word, used by the
            // next pass, is cleared once every wave has read it in the previous one
            if (busy && lane == 0) atomicOr(&wg->busy[vote], 1u);
            __syncthreads();
            const bool any = wg->busy[vote] != 0u;
            if (threadIdx.x == 0) {
                wg->busy[vote ^ 1] = 0u;
                // every wave has ended its sweep; the next sweeps begin after the
                // event pass's workgroup barriers
                atomicAnd(&wg->quorum, 0xffff0000u);
            }
            vote ^= 1;
            if (!any) break;
        } else {
            if (!busy) break;
            pre_event();
        }

        // ---- event batch
        if (busy) lc.passes++;
        event_pass();
        cur = P<R>::shell(ps);
        if constexpr (KRHO) curk = rk[ps - sh];
    }
}

// Sum the per-lane counters over the wave and add them to the launch statistics.
__device__ __forceinline__ void flush_counters(const LaneCounters &lc, DevStats *stats) {
    const int lane = __lane_id();
    // modular: the wave's sum is the number of crossings
    const unsigned long long cross = (lane == 0 ? lc.steps : 0ull) - (unsigned long long)lc.sent;
    const unsigned long long cs[11] = {lc.launch, cross, lc.scat, lc.abs, lc.escape,
                                       lc.direct, lc.limit, lc.floor, lc.reabove,
                                       lane == 0 ? (unsigned long long)lc.passes : 0ull,
                                       lane == 0 ? lc.slots : 0ull};
    const int cidx[11] = {C_LAUNCH, C_CROSS, C_SCAT, C_ABS, C_ESCAPE, C_DIRECT, C_LIMIT, C_FLOOR, C_REEMIT_ABOVE,
                          C_PASS, C_SLOTS};
#pragma unroll
    for (int j = 0; j < 11; ++j) {
        const unsigned long long v = wave_sum_u64(cs[j]);
        if (lane == 0 && v) atomicAdd(&stats->cnt[cidx[j]], v);
    }
    const double ts[4] = {lc.esc0, lc.esc1, lc.ffi, lc.term};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double v = wave_sum_f64(ts[j]);
        if (lane == 0 && v != 0.0) unsafeAtomicAdd(&stats->tally[j], v);
    }
}

// Add this workgroup's escaping spectrum (LDS) to the launch's (global).
__device__ __forceinline__ void flush_sed(const double *s_sed, int n, double *sed) {
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += blockDim.x)
        if (s_sed[j] != 0.0) unsafeAtomicAdd(&sed[j], s_sed[j]);
}

template <typename R>
__device__ __forceinline__ void single_model(const TraceParams &p, const typename P<R>::Shell *sh,
                                             ModelCtx<R> &mc, MethodOpts &o) {
    mc.sh = sh;
    mc.n = p.n;
    mc.cav = p.cavity;
    mc.invM = p.invM;
    // accumulator group of this workgroup: an independent run over the packages its
    // waves take, whose running total times the number of groups estimates the whole
    const int rep = p.replicas > 1 ? (int)(blockIdx.x % (unsigned)p.replicas) : 0;
    mc.A = p.A + (size_t)rep * p.n * kAccStride;
    mc.a_scale = p.replicas > 1 ? (double)p.replicas : 1.0;
    mc.eps[0] = p.eps[0];
    mc.eps[1] = p.eps[1];
    mc.n_ext = p.n_ext;
    mc.n_ps = p.n_ps;
    mc.pid0[0] = p.pid0[0];
    mc.pid0[1] = p.pid0[1];
    mc.seed = p.seed;
    o.k_bg = p.k_bg;
    o.ffi = p.ffi;
    o.reemit_uniform = p.reemit_uniform;
    o.batch = p.batch;
    o.quorum = p.quorum;
    o.w_floor = p.w_floor;
    o.max_events = p.max_events;
    o.use_g_E = p.use_g_E;
    o.g_E = p.g_E;
    o.use_g_S = p.use_g_S;
    o.g_S = p.g_S;
    o.k_A = p.k_A;
    o.k_S = p.k_S;
}

template <int AGG, int WT>
__global__ __launch_bounds__(kBlockFP32) void ire_trace_f32(TraceParams p) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int nsh = p.n + p.cavity + kSentinels, K = p.K, n_t = p.n_t;
    const LdsLayout L = lds_layout(nsh, K, n_t, true, true, kBlockFP32);
    ShellF *s_sh = reinterpret_cast<ShellF *>(smem + L.sh) + kPadBelow;
    DustF *s_dust = reinterpret_cast<DustF *>(smem + L.dust);
    float *s_cdf = reinterpret_cast<float *>(smem + L.cdf);
    float *s_G = reinterpret_cast<float *>(smem + L.G);
    float *s_D = reinterpret_cast<float *>(smem + L.D);
    uint32_t *s_guide = reinterpret_cast<uint32_t *>(smem + L.guide);
    for (int j = threadIdx.x - kPadBelow; j < nsh; j += blockDim.x) s_sh[j] = j < 0 ? ShellF{0, 0, 0, 0} : p.shf[j];
    for (int j = threadIdx.x; j < K; j += blockDim.x) s_dust[j] = p.dustf[j];
    for (int j = threadIdx.x; j < 2 * K; j += blockDim.x) s_cdf[j] = p.cdff[j];
    for (int j = threadIdx.x; j < n_t; j += blockDim.x) s_G[j] = p.Gf[j];
    const int nd = n_t * K, ldD = d_stride(K);
    for (int j = threadIdx.x; j < nd; j += blockDim.x) {
        const int r = j / K;
        s_D[r * ldD + (j - r * K)] = p.Df[j];
    }
    const int ng = (int)(guide_bytes(n_t) / 4);
    for (int j = threadIdx.x; j < ng; j += blockDim.x) s_guide[j] = reinterpret_cast<const uint32_t *>(p.guide)[j];
    double *s_sed = reinterpret_cast<double *>(smem + L.sed);
    for (int j = threadIdx.x; j < 4 * K; j += blockDim.x) s_sed[j] = 0.0;
    float2 *s_rk = reinterpret_cast<float2 *>(smem + L.rk) + kPadBelow;
    if constexpr (WT == 2)
        for (int j = threadIdx.x - kPadBelow; j < nsh; j += blockDim.x) s_rk[j] = j < 0 ? float2{0, 0} : p.rkf[j];
    AggScratch *s_agg = reinterpret_cast<AggScratch *>(smem + L.agg);
    if constexpr (AGG == 2) wg_scratch_init(reinterpret_cast<WgScratch *>(s_agg));
    __syncthreads();
    ModelCtx<float> mc;
    MethodOpts o;
    single_model<float>(p, s_sh, mc, o);
    const long long gtid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    LaneCounters lc;
    trace_model<float, AGG, WT>(mc, o, s_dust, s_cdf, s_G, s_D, K, n_t, d_stride(K),
                                reinterpret_cast<const unsigned char *>(s_guide),
                                p.g_lg0, p.g_scale, s_rk, &p.stats->cursor, p.chunk,
                                 p.max_lanes > 0 && gtid >= p.max_lanes, lc, s_sed, s_agg + threadIdx.x / kWave,
                                 reinterpret_cast<WgScratch *>(s_agg));
    flush_counters(lc, p.stats);
    flush_sed(s_sed, 4 * K, p.sed);
}

template <int AGG, int WT>
__global__ __launch_bounds__(256) void ire_trace_f64(TraceParams p) {
    extern __shared__ __align__(16) unsigned char smem[];
    double *s_sed = reinterpret_cast<double *>(smem);
    for (int j = threadIdx.x; j < 4 * p.K; j += blockDim.x) s_sed[j] = 0.0;
    if constexpr (AGG == 2) wg_scratch_init(reinterpret_cast<WgScratch *>(s_sed + 4 * p.K));
    __syncthreads();
    ModelCtx<double> mc;
    MethodOpts o;
    single_model<double>(p, p.shd, mc, o);
    const long long gtid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    LaneCounters lc;
    trace_model<double, AGG, WT>(mc, o, p.dustd, p.cdfd, p.Gd, p.Dd, p.K, p.n_t, p.K, p.guide, p.g_lg0, p.g_scale,
                                 p.rkd, &p.stats->cursor, p.chunk, p.max_lanes > 0 && gtid >= p.max_lanes, lc, s_sed,
                                 reinterpret_cast<AggScratch *>(s_sed + 4 * p.K) + threadIdx.x / kWave,
                                 reinterpret_cast<WgScratch *>(s_sed + 4 * p.K));
    flush_counters(lc, p.stats);
    flush_sed(s_sed, 4 * p.K, p.sed);
}

__global__ void ire_zero(double *A, int n, DevStats *st, int clear_counts, double *sed, int n_sed) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    for (int j = tid; j < n * kAccStride; j += gridDim.x * blockDim.x) A[j] = 0.0;
    if (clear_counts)
        for (int j = tid; j < n_sed; j += gridDim.x * blockDim.x) sed[j] = 0.0;
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
    double A = 0.0;
    for (int r = 0; r < p.replicas; ++r) A += p.A[((size_t)r * p.n + i) * kAccStride];
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

// ---------------------------------------------------------------------------
// Batched persistent launch: each workgroup takes work items (a range of one
// model's packages) from a global cursor, stages that model's shells in LDS
// next to the shared dust / G / re-emission tables, traces the range with all
// its waves (package indices from an LDS cursor), and drains before the next.

template <int AGG, int WT>
__global__ __launch_bounds__(kBlockFP32) void ire_trace_batch(BatchParams p) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned long long s_item;
    __shared__ unsigned long long s_cursor;
    const int K = p.K, n_t = p.n_t;
    const LdsLayout L = lds_layout(p.max_table, K, n_t, false, WT == 2, kBlockFP32);
    ShellF *s_sh = reinterpret_cast<ShellF *>(smem + L.sh) + kPadBelow;
    DustF *s_dust = reinterpret_cast<DustF *>(smem + L.dust);
    if (threadIdx.x == 0) s_sh[-1] = ShellF{0, 0, 0, 0};
    float2 *s_rk = WT == 2 ? reinterpret_cast<float2 *>(smem + L.rk) + kPadBelow : nullptr;
    if (WT == 2 && threadIdx.x == 0) s_rk[-1] = float2{0, 0};
    float *s_cdf = reinterpret_cast<float *>(smem + L.cdf);
    float *s_G = reinterpret_cast<float *>(smem + L.G);
    float *s_D = reinterpret_cast<float *>(smem + L.D);
    uint32_t *s_guide = reinterpret_cast<uint32_t *>(smem + L.guide);
    for (int j = threadIdx.x; j < K; j += blockDim.x) s_dust[j] = p.dustf[j];
    for (int j = threadIdx.x; j < 2 * K; j += blockDim.x) s_cdf[j] = p.cdff[j];
    for (int j = threadIdx.x; j < n_t; j += blockDim.x) s_G[j] = p.Gf[j];
    const int nd = n_t * K, ldD = d_stride(K);
    for (int j = threadIdx.x; j < nd; j += blockDim.x) {
        const int r = j / K;
        s_D[r * ldD + (j - r * K)] = p.Df[j];
    }
    const int ng = (int)(guide_bytes(n_t) / 4);
    for (int j = threadIdx.x; j < ng; j += blockDim.x) s_guide[j] = reinterpret_cast<const uint32_t *>(p.guide)[j];
    AggScratch *s_agg = reinterpret_cast<AggScratch *>(smem + L.agg);

    MethodOpts o;
    o.k_bg = p.k_bg;
    o.ffi = p.ffi;
    o.reemit_uniform = p.reemit_uniform;
    o.batch = p.batch;
    o.quorum = 16;
    o.w_floor = p.w_floor;
    o.max_events = p.max_events;
    o.use_g_E = p.use_g_E;
    o.g_E = p.g_E;
    o.use_g_S = p.use_g_S;
    o.g_S = p.g_S;
    o.k_A = p.k_A;
    o.k_S = p.k_S;
    LaneCounters lc;
    for (;;) {
        __syncthreads();  // every wave has finished the previous item: the shell slot is free
        if (threadIdx.x == 0) {
            s_item = atomicAdd(&p.stats->cursor, 1ull);
            s_cursor = 0;
        }
        __syncthreads();
        const unsigned long long it = s_item;
        if (it >= (unsigned long long)p.n_items) break;
        const BatchItemDev item = p.items[it];
        const BatchModelDev bm = p.models[item.model];
        const int nt = bm.n + bm.cav + kSentinels;
        for (int j = threadIdx.x; j < nt; j += blockDim.x) s_sh[j] = p.shells[bm.shell_off + j];
        if constexpr (WT == 2)
            for (int j = threadIdx.x; j < nt; j += blockDim.x) s_rk[j] = p.rkf[bm.shell_off + j];
        __syncthreads();
        ModelCtx<float> mc;
        mc.sh = s_sh;
        mc.n = bm.n;
        mc.cav = bm.cav;
        mc.invM = p.invM + bm.acc_off;
        mc.A = p.A + (size_t)bm.acc_off * kAccStride;
        mc.a_scale = 1.0;
        mc.eps[0] = bm.eps;
        mc.eps[1] = bm.eps;
        mc.n_ext = bm.src == 0 ? item.count : 0;
        mc.n_ps = bm.src == 0 ? 0 : item.count;
        mc.pid0[0] = item.first;
        mc.pid0[1] = item.first;
        mc.seed = bm.seed;
        trace_model<float, AGG, WT>(mc, o, s_dust, s_cdf, s_G, s_D, K, n_t, d_stride(K),
                                    reinterpret_cast<const unsigned char *>(s_guide), p.g_lg0, p.g_scale, s_rk,
                                    &s_cursor,
                                     64ull, false, lc, nullptr, s_agg + threadIdx.x / kWave, nullptr);
    }
    flush_counters(lc, p.stats);
}

__global__ void ire_zero_batch(double *A, size_t n_shells, DevStats *st) {
    const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (size_t j = tid; j < n_shells; j += (size_t)gridDim.x * blockDim.x) A[j * kAccStride] = 0.0;
    if (tid == 0) {
        st->cursor = 0;
        for (int j = 0; j < 16; ++j) st->cnt[j] = 0;
        for (int j = 0; j < 8; ++j) st->tally[j] = 0.0;
    }
}

// A -> T for every shell of every model (the models share the G(T) table)
__global__ void ire_finalize_batch(BatchFinalizeParams p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n_shells) return;
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

size_t trace_lds_bytes(int n_table, int K, int n_t) {
    return lds_layout(n_table, K, n_t, true, true, kBlockFP32).total;
}

size_t batch_lds_bytes(int max_table, int K, int n_t, bool k_A_rho) {
    return lds_layout(max_table, K, n_t, false, k_A_rho, kBlockFP32).total;
}

size_t sed_lds_bytes(int K) { return (size_t)4 * K * sizeof(double); }

template <int WT>
static const void *f32_kernel_wt(int aggregate) {
    if (aggregate == 2) return reinterpret_cast<const void *>(&ire_trace_f32<2, WT>);
    if (aggregate == 1) return reinterpret_cast<const void *>(&ire_trace_f32<1, WT>);
    return reinterpret_cast<const void *>(&ire_trace_f32<0, WT>);
}

static const void *f32_kernel(int aggregate, int wt) {
    if (wt == 2) return f32_kernel_wt<2>(aggregate);
    if (wt == 1) return f32_kernel_wt<1>(aggregate);
    return f32_kernel_wt<0>(aggregate);
}

// the batched launch groups by wave (aggregate 2 is a single-model schedule)
static const void *batch_kernel(int aggregate, int wt) {
    if (wt == 2) return aggregate ? reinterpret_cast<const void *>(&ire_trace_batch<1, 2>)
                                  : reinterpret_cast<const void *>(&ire_trace_batch<0, 2>);
    if (wt == 1) return aggregate ? reinterpret_cast<const void *>(&ire_trace_batch<1, 1>)
                                  : reinterpret_cast<const void *>(&ire_trace_batch<0, 1>);
    return aggregate ? reinterpret_cast<const void *>(&ire_trace_batch<1, 0>)
                     : reinterpret_cast<const void *>(&ire_trace_batch<0, 0>);
}

template <int WT>
static const void *f64_kernel_wt(int aggregate) {
    if (aggregate == 2) return reinterpret_cast<const void *>(&ire_trace_f64<2, WT>);
    if (aggregate == 1) return reinterpret_cast<const void *>(&ire_trace_f64<1, WT>);
    return reinterpret_cast<const void *>(&ire_trace_f64<0, WT>);
}

static const void *f64_kernel(int aggregate, int wt) {
    if (wt == 2) return f64_kernel_wt<2>(aggregate);
    if (wt == 1) return f64_kernel_wt<1>(aggregate);
    return f64_kernel_wt<0>(aggregate);
}

// The weighted-sampling instantiations are used only when an option needs
// them, so that the default path keeps its register budget.
static int weighting(const TraceParams &p) {
    if (p.k_A_rho) return 2;
    return (p.use_g_E || p.use_g_S || p.k_A != 1.0 || p.k_S != 1.0 || p.ffi == 2) ? 1 : 0;
}

static int weighting(const BatchParams &p) {
    if (p.k_A_rho) return 2;
    return (p.use_g_E || p.use_g_S || p.k_A != 1.0 || p.k_S != 1.0 || p.ffi == 2) ? 1 : 0;
}

hipError_t trace_configure(int fp64, int aggregate, size_t lds) {
    if (fp64) return hipSuccess;
    for (int wt = 0; wt < 3; ++wt) {
        const hipError_t e = hipFuncSetAttribute(f32_kernel(aggregate, wt), hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_trace(const TraceParams &p, int fp64, int aggregate, int grid, int block, size_t lds,
                        hipStream_t s) {
    TraceParams q = p;
    void *args[] = {&q};
    if (fp64) return hipLaunchKernel(f64_kernel(aggregate, weighting(p)), dim3(grid), dim3(block), args,
                                     sed_lds_bytes(p.K) + agg_lds_bytes(block), s);
    return hipLaunchKernel(f32_kernel(aggregate, weighting(p)), dim3(grid), dim3(block), args, lds, s);
}

hipError_t launch_zero(double *A, int n, DevStats *st, int clear_counts, double *sed, int n_sed, hipStream_t s) {
    if (A) {
        int blocks = (n * kAccStride + 255) / 256;
        if (blocks < 1) blocks = 1;
        if (blocks > 1024) blocks = 1024;
        hipLaunchKernelGGL(ire_zero, dim3(blocks), dim3(256), 0, s, A, n, st, clear_counts, sed, n_sed);
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

// The block size the FP32 tracers are compiled for.
int trace_block_fp32() { return kBlockFP32; }

hipError_t batch_configure(int aggregate, size_t lds) {
    for (int wt = 0; wt < 3; ++wt) {
        const hipError_t e = hipFuncSetAttribute(batch_kernel(aggregate, wt), hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_trace_batch(const BatchParams &p, int aggregate, int grid, size_t lds, hipStream_t s) {
    BatchParams q = p;
    void *args[] = {&q};
    return hipLaunchKernel(batch_kernel(aggregate, weighting(p)), dim3(grid), dim3(kBlockFP32), args, lds, s);
}

hipError_t launch_zero_batch(double *A, size_t n_shells, DevStats *st, hipStream_t s) {
    size_t blocks = (n_shells + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 4096 ? 4096 : blocks);
    hipLaunchKernelGGL(ire_zero_batch, dim3((unsigned)blocks), dim3(256), 0, s, A, n_shells, st);
    return hipGetLastError();
}

hipError_t launch_finalize_batch(const BatchFinalizeParams &p, hipStream_t s) {
    const int blocks = (p.n_shells + 255) / 256;
    hipLaunchKernelGGL(ire_finalize_batch, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, p);
    return hipGetLastError();
}

}  // namespace ire
