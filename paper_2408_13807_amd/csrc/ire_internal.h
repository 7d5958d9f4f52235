// Internal layouts shared by the host library and the HIP kernels of libire.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ire {

// Absorbed-energy accumulators are FP64, one per shell, each on its own
// 128-byte line so that returning atomics on different shells never share a line.
constexpr int kAccStride = 16;

// Shell geometry in units of the outer radius: squared inner and outer radius,
// and density times the outer radius, so kappa * rho_hat * l_hat is an optical
// depth when l_hat is a length in outer radii.
struct ShellF { float r2_in, r2_out, rho, r_in; };
struct ShellD { double r2_in, r2_out, rho, r_in; };

// Per-frequency dust coefficients: kappa_abs, kappa_sca, HG g, albedo.
struct DustF { float kA, kS, g, alb; };
struct DustD { double kA, kS, g, alb; };

enum Counter {
    C_LAUNCH, C_CROSS, C_SCAT, C_ABS, C_ESCAPE, C_DIRECT, C_LIMIT, C_FLOOR,
    C_REEMIT_ABOVE, C_BELOW, C_ABOVE, C_COUNT
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
    const ShellF *shf;
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
    double eps[2];                    // package energy per source
    unsigned long long n_ext, n_ps;   // packages of this launch per source
    unsigned long long pid0[2];       // first package id per source (chunked runs)
    unsigned long long seed;
    double k_bg;
    int ffi;
    int reemit_uniform;
    double w_floor;
    unsigned long long max_events;
    int max_lanes;                    // 0 = no limit
    unsigned long long chunk;         // package indices a wave takes from the cursor at once (>= 64)
    int batch;                        // parked lanes that trigger an event pass (1..64)
    double *A;                        // n accumulators, stride kAccStride
    DevStats *stats;
};

struct FinalizeParams {
    int n, n_t;
    const double *A;                  // stride kAccStride
    const double *invM;
    const double *Gd, *lnG, *lnT;
    double t_min, t_max;
    double *A_out;                    // n compact
    double *T_out;                    // n
    DevStats *stats;
};

size_t trace_lds_bytes(int n, int K, int n_t);
hipError_t launch_trace(const TraceParams &p, int fp64, int aggregate, int grid, int block,
                        size_t lds, hipStream_t s);
hipError_t trace_configure(int fp64, int aggregate, size_t lds);
hipError_t launch_zero(double *A, int n, DevStats *st, int clear_counts, hipStream_t s);
hipError_t launch_finalize(const FinalizeParams &p, hipStream_t s);

}  // namespace ire
