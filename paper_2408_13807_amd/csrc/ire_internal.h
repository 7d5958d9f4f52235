// Internal layouts shared by the host library and the HIP kernels of libire.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ire {

// Absorbed-energy accumulators are FP64, one per shell, each on its own
// 128-byte line so that returning atomics on different shells never share a line.
constexpr int kAccStride = 16;
// Shell tables end in two sentinel records beyond the surface (infinite
// density): a flight that leaves the cloud ends in the first; the second keeps
// the tracer's one-record-ahead reads inside the table for every lane.
constexpr int kSentinels = 2;
// The FP32 kernels stage the table in LDS behind one pad record: a lane that is
// not in flight keeps stepping with a stale record, and its reads then stay
// within one record of its shell, so inside [pad, second sentinel].
constexpr int kPadBelow = 1;
// Largest number of independent accumulator groups of a single-model run.
constexpr int kMaxReplicas = 8;
// Slots of a wave's LDS scratch for grouping its absorptions by shell (a power
// of two), and the scratch of a workgroup of `block` threads (plus 8 bytes for
// aligning it after tables of 4-byte entries).
constexpr int kAggSlots = 32;
// Slots of a workgroup's LDS scratch for grouping the absorptions of all its
// waves by shell (aggregate = 2): key, group sum and group base per slot.
constexpr int kWgSlots = 256;
__host__ __device__ inline size_t agg_lds_bytes(int block) {
    const size_t wave = (size_t)(block / 64) * kAggSlots * (sizeof(double) + sizeof(int));
    const size_t wg = (size_t)kWgSlots * (2 * sizeof(double) + sizeof(unsigned)) + 4 * sizeof(unsigned);
    return (wave > wg ? wave : wg) + 8;
}
// A guide table (cut-point method, Chen & Asau 1974) accelerates the search
// of the G(T) table; the search stays exact (a bidirectional scan from the
// guide's start).  Layout of the guide bytes: uint16 gg[n_t], bins uniform in
// log2 G.  (The frequency CDFs are searched four ways, count_le4.)
__host__ __device__ inline size_t guide_bytes(int n_t) { return ((size_t)n_t * 2 + 15) / 16 * 16; }
constexpr int kMaxK = 255;            // frequencies of a model (the API's limit)
constexpr int kMaxGuideNt = 65535;    // temperature points a 16-bit guide can index

// Number of entries of the non-decreasing table t[0..n) (n >= 1) that are
// <= x, by a four-way search: each round reads several entries at once (their
// LDS latencies overlap) and keeps one of four equal parts of the range; the
// first round also tests the range's end, so a 64-entry row takes three
// rounds (4 + 3 + 3 reads) in every lane.  A lane scanning from a guide start
// is fast on average, but a wave waits for its longest scan, and the far
// tails of a spectrum (many frequencies with a tiny share of the power) make
// some scans long.
template <typename T, typename X>
__host__ __device__ inline int count_le4(const T *t, int n, X x) {
    int step = 1;
    while (step * 4 < n) step *= 4;     // the answer, in [0, n], is at most 4 * step
    int pos = 0;
    {
        int c = 0;
#pragma unroll
        for (int j = 1; j <= 4; ++j) {
            const int q = j * step;
            const X v = (X)t[(q < n ? q : n) - 1];
            c += (int)(q <= n && v <= x);
        }
        pos = step * c;
    }
    for (step >>= 2; step > 0; step >>= 2) {
        const int q1 = pos + step, q2 = q1 + step, q3 = q2 + step;
        const X v1 = (X)t[(q1 < n ? q1 : n) - 1];
        const X v2 = (X)t[(q2 < n ? q2 : n) - 1];
        const X v3 = (X)t[(q3 < n ? q3 : n) - 1];
        pos += step * ((int)(q1 <= n && v1 <= x) + (int)(q2 <= n && v2 <= x) + (int)(q3 <= n && v3 <= x));
    }
    return pos;
}

// Shell geometry in units of the outer radius: squared inner and outer radius,
// density times the outer radius (so kappa * rho_hat * l_hat is an optical depth
// when l_hat is a length in outer radii) and its reciprocal (0 for an empty shell).
struct ShellF { float r2_in, r2_out, rho, inv_rho; };
struct ShellD { double r2_in, r2_out, rho, inv_rho; };

// Per-frequency dust coefficients: kappa_abs and kappa_sca, their reciprocals
// (infinite for kappa_sca = 0), HG g, albedo, extinction kappa_abs + kappa_sca.
struct DustF { float kA, kS, inv_kA, inv_kS, g, alb, kext, pad; };
struct DustD { double kA, kS, inv_kA, inv_kS, g, alb, kext, pad; };

// Byte offsets of the regions of an FP32 tracer's LDS.  Every region starts on
// a 16-byte boundary: the tables before the escaping spectrum and the grouping
// scratch hold 4-byte and 1-byte entries in counts that need not be even,
// while those two regions hold doubles updated by LDS atomics, which must be
// 8-byte aligned.  The shell table begins with kPadBelow pad records.  `sed`
// and `rk` (the escaping spectrum and the k_A(rho) records) are absent from
// the batched launch.
struct LdsLayout { size_t sh, dust, cdf, G, D, guide, sed, rk, agg, total; };
// Row stride (floats) of the re-emission CDF rows in LDS: odd, so that the
// lanes of a wave reading the same column of different rows (the first
// rounds of a four-way search) fall into different banks.
__host__ __device__ inline int d_stride(int K) { return K | 1; }
__host__ __device__ inline size_t lds_align16(size_t x) { return (x + 15) & ~(size_t)15; }
__host__ __device__ inline LdsLayout lds_layout(int n_table, int K, int n_t, bool sed, bool rk, int block) {
    LdsLayout L{};
    size_t o = 0;
    L.sh = o;    o = lds_align16(o + (size_t)(n_table + kPadBelow) * sizeof(ShellF));
    L.dust = o;  o = lds_align16(o + (size_t)K * sizeof(DustF));
    L.cdf = o;   o = lds_align16(o + (size_t)2 * K * sizeof(float));
    L.G = o;     o = lds_align16(o + (size_t)n_t * sizeof(float));
    L.D = o;     o = lds_align16(o + (size_t)n_t * d_stride(K) * sizeof(float));
    L.guide = o; o = lds_align16(o + guide_bytes(n_t));
    L.sed = o;   o = lds_align16(o + (sed ? (size_t)4 * K * sizeof(double) : 0));
    L.rk = o;    o = lds_align16(o + (rk ? (size_t)(n_table + kPadBelow) * 2 * sizeof(float) : 0));
    L.agg = o;   o = lds_align16(o + agg_lds_bytes(block));
    L.total = o;
    return L;
}

enum Counter {
    C_LAUNCH, C_CROSS, C_SCAT, C_ABS, C_ESCAPE, C_DIRECT, C_LIMIT, C_FLOOR,
    C_REEMIT_ABOVE, C_BELOW, C_ABOVE, C_PASS, C_SLOTS, C_COUNT
};
enum Tally { T_ESC_EXT, T_ESC_PS, T_FFI, T_TERM, T_COUNT };

struct DevStats {
    unsigned long long cnt[16];
    double tally[8];
    unsigned long long cursor;   // next package index of the current launch
    unsigned long long pad[7];
};

struct TraceParams {
    int n, K, n_t;
    int cavity;                       // 1 if r_edges[0] > 0 (empty central cavity)
    // FP32 tables in global memory (staged into LDS by each workgroup)
    const ShellF *shf;                // cavity + n + 1: [empty cavity], shells, sentinel beyond the surface
    const DustF *dustf;
    const float *cdff;                // 2*K: source CDFs, external then point source
    const float *Gf;                  // n_t: emitted power per mass on the T grid
    const float *Df;                  // n_t*K: re-emission CDF rows
    // FP64 tables (read from global memory by the FP64 instantiation)
    const ShellD *shd;
    const DustD *dustd;
    const double *cdfd;
    const double *Gd;
    const double *Dd;
    const double *invM;               // n: 1 / shell mass
    const unsigned char *guide;       // guide_bytes(n_t) (staged into LDS by the FP32 path)
    float g_lg0, g_scale;             // G guide bin = (log2 a - g_lg0) * g_scale
    double eps[2];                    // package energy per source
    unsigned long long n_ext, n_ps;   // packages of this launch per source
    unsigned long long pid0[2];       // first package id per source (chunked runs)
    unsigned long long seed;
    double k_bg;
    int ffi;
    int reemit_uniform;
    double w_floor;
    unsigned long long max_events;
    int use_g_E, use_g_S;             // weighted sampling (Table 1)
    double g_E, g_S, k_A, k_S;
    int k_A_rho;                      // absorption scaling by density: per-shell {k rho, 1/(k rho)} below
    const float2 *rkf;                // cavity + n + kSentinels records (table units), FP32 path
    const double2 *rkd;               // the same, FP64 path
    int max_lanes;                    // 0 = no limit
    int replicas;                     // accumulator groups: workgroup b adds into copy b % replicas
    unsigned long long chunk;         // package indices a wave takes from the cursor at once (>= 64)
    int batch;                        // parked lanes that trigger an event pass (1..64)
    int quorum;                       // workgroup grouping: waves at their batch that end every wave's sweep
    double *A;                        // n accumulators, stride kAccStride
    double *sed;                      // 4*K: escaped power per source and frequency, then its unscattered part
    DevStats *stats;
};

struct FinalizeParams {
    int n, n_t;
    const double *A;                  // stride kAccStride; `replicas` copies of n, summed
    int replicas;
    const double *invM;
    const double *Gd, *lnG, *lnT;
    double t_min, t_max;
    double *A_out;                    // n compact
    double *T_out;                    // n
    DevStats *stats;
};

// ---- batched launch: many cloud models sharing the dust and temperature tables

struct BatchModelDev {
    int shell_off;                    // first entry of the model's shell table ([cavity] + n + sentinel)
    int n, cav, src;                  // shells, cavity flag, source (0 external, 1 point)
    int acc_off;                      // first shell of the model in the flat per-shell arrays
    int pad;
    double eps;                       // package energy
    unsigned long long n_pkg, seed;
};

struct BatchItemDev {                 // a range of one model's packages
    int model, pad;
    unsigned long long first, count;
};

struct BatchParams {
    int K, n_t, n_items, max_table;   // max_table: largest per-model shell table
    const ShellF *shells;             // all models' shell tables
    const DustF *dustf;
    const float *cdff;                // 2*K source CDFs (external field, point source)
    const float *Gf, *Df;
    const unsigned char *guide;       // guide_bytes(n_t)
    float g_lg0, g_scale;
    const double *invM;               // per shell, flat
    double *A;                        // per shell, flat, stride kAccStride
    const BatchModelDev *models;
    const BatchItemDev *items;
    double k_bg;
    int ffi, reemit_uniform, batch, pad;
    double w_floor;
    unsigned long long max_events;
    int use_g_E, use_g_S;             // weighted sampling (Table 1)
    double g_E, g_S, k_A, k_S;
    int k_A_rho;                      // absorption scaling by density: per-shell {k rho, 1/(k rho)} below
    const float2 *rkf;                // laid out as `shells` (each model's table at its shell_off)
    DevStats *stats;                  // stats->cursor counts taken items
};

struct BatchFinalizeParams {
    int n_shells, n_t;
    const double *A, *invM, *Gd, *lnG, *lnT;
    double t_min, t_max;
    double *A_out, *T_out;
    DevStats *stats;
};

size_t trace_lds_bytes(int n_table, int K, int n_t);  // n_table = cavity + n + kSentinels
size_t batch_lds_bytes(int max_table, int K, int n_t, bool k_A_rho);
size_t sed_lds_bytes(int K);
hipError_t launch_trace(const TraceParams &p, int fp64, int aggregate, int grid, int block,
                        size_t lds, hipStream_t s);
hipError_t trace_configure(int fp64, int aggregate, size_t lds);
hipError_t launch_zero(double *A, int n, DevStats *st, int clear_counts, double *sed, int n_sed, hipStream_t s);
hipError_t launch_finalize(const FinalizeParams &p, hipStream_t s);
hipError_t batch_configure(int aggregate, size_t lds);
hipError_t launch_trace_batch(const BatchParams &p, int aggregate, int grid, size_t lds, hipStream_t s);
hipError_t launch_zero_batch(double *A, size_t n_shells, DevStats *st, hipStream_t s);
hipError_t launch_finalize_batch(const BatchFinalizeParams &p, hipStream_t s);
int trace_block_fp32();

}  // namespace ire
