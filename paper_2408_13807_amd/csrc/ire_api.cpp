// C-ABI of libire (include/ire.h): argument validation, host-side FP64 table
// construction, device buffers and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "ire.h"
#include "ire_host.h"
#include "ire_internal.h"

namespace ire {
int trace_block_fp32();
}

using ire::host::DevBuf;
using ire::host::finite_all;
using ire::host::kPi;

struct ire_model {
    int device = 0;
    std::string err;
    // problem definition (host, FP64)
    std::vector<double> r_edges, rho;
    std::vector<double> nu, kabs, albedo, g;
    double t_min = 3.0, t_max = 1600.0;
    int n_t = 512;
    std::vector<double> J;          // empty = no external field
    double L_ps = 0.0;
    std::vector<double> S;          // empty = no point source
    ire_options opt{};
    bool dirty = true;
    // derived host tables
    double L_ext = 0.0;
    std::vector<double> lnT, lnG;
    // device buffers
    DevBuf<ire::ShellF> shf;
    DevBuf<ire::ShellD> shd;
    DevBuf<float2> rkf;
    DevBuf<double2> rkd;
    DevBuf<ire::DustF> dustf;
    DevBuf<ire::DustD> dustd;
    DevBuf<float> cdff, Gf, Df;
    DevBuf<double> cdfd, Gd, Dd, invM, lnGd, lnTd;
    DevBuf<unsigned char> guide;
    float g_lg0 = 0.0f, g_scale = 0.0f;
    DevBuf<double> A, A_out, T_out;
    DevBuf<ire::DevStats> stats;
    DevBuf<double> sed;               // 4*K escaping spectrum (total, then unscattered)
    // run state
    bool begun = false;
    int replicas = 1;                 // accumulator groups of the current run
    unsigned long long n_total[2] = {0, 0};
    unsigned long long n_done[2] = {0, 0};
    unsigned long long seed = 0;
    double eps[2] = {0.0, 0.0};
    hipStream_t last_stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    float ms_tables = 0.0f, ms_trace = 0.0f, ms_finalize = 0.0f;
    bool timed = false;
    int n_cu = 0;
    size_t max_lds = 0;

    int fail(int code, const char *fmt, ...) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        err = buf;
        return code;
    }
    int hip_fail(hipError_t e, const char *what) {
        return fail(IRE_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
    }
};

namespace {

// Build every table in FP64 on the host and upload FP32 and FP64 copies.
int build_tables(ire_model *m) {
    const int n = (int)m->rho.size();
    const int K = (int)m->nu.size();
    const double Rout = m->r_edges[n];
    ire::host::DustTables dt;
    const std::string err = ire::host::build_dust_tables(m->nu, m->kabs, m->albedo, m->g, m->t_min, m->t_max,
                                                         m->n_t, dt);
    if (!err.empty()) return m->fail(IRE_E_INVALID, "%s", err.c_str());
    std::vector<ire::ShellF> shf;
    std::vector<ire::ShellD> shd;
    std::vector<double> invM;
    ire::host::build_shell_table(m->r_edges.data(), m->rho.data(), n, shf, shd, invM);
    std::vector<float2> rkf;
    std::vector<double2> rkd;
    ire::host::build_absorption_scaling(m->r_edges.data(), m->rho.data(), n, m->opt.k_A_lowest, m->opt.k_A_highest,
                                        rkf, rkd);
    const std::vector<ire::DustF> &df = dt.df;
    const std::vector<ire::DustD> &dd = dt.dd;
    const std::vector<double> &G = dt.G, &D = dt.D, &w = dt.w;

    // sources: frequency CDFs of J w and S w; the external luminosity is the
    // inward flux pi J through the surface
    std::vector<double> q(K), cdf(2 * K);
    double sumJ = 0.0;
    for (int k = 0; k < K; ++k) {
        q[k] = m->J.empty() ? 0.0 : m->J[k] * w[k];
        sumJ += q[k];
    }
    ire::host::cumulative(q.data(), K, cdf.data());
    for (int k = 0; k < K; ++k) q[k] = m->S.empty() ? 0.0 : m->S[k] * w[k];
    ire::host::cumulative(q.data(), K, cdf.data() + K);
    m->L_ext = 4.0 * kPi * Rout * Rout * kPi * sumJ;
    m->lnT = dt.lnT;
    m->lnG = dt.lnG;

    std::vector<float> cdff(cdf.begin(), cdf.end()), Gf(G.begin(), G.end()), Df(D.begin(), D.end());
    std::vector<unsigned char> guide;
    ire::host::build_guides(dt, guide, m->g_lg0, m->g_scale);
    hipError_t e;
    if ((e = hipSetDevice(m->device)) != hipSuccess) return m->hip_fail(e, "hipSetDevice");
    if ((e = m->shf.upload(shf)) != hipSuccess || (e = m->shd.upload(shd)) != hipSuccess ||
        (e = m->dustf.upload(df)) != hipSuccess || (e = m->dustd.upload(dd)) != hipSuccess ||
        (e = m->cdff.upload(cdff)) != hipSuccess || (e = m->cdfd.upload(cdf)) != hipSuccess ||
        (e = m->Gf.upload(Gf)) != hipSuccess || (e = m->Gd.upload(G)) != hipSuccess ||
        (e = m->Df.upload(Df)) != hipSuccess || (e = m->Dd.upload(D)) != hipSuccess ||
        (e = m->invM.upload(invM)) != hipSuccess || (e = m->lnGd.upload(m->lnG)) != hipSuccess ||
        (e = m->lnTd.upload(m->lnT)) != hipSuccess || (e = m->guide.upload(guide)) != hipSuccess ||
        (e = m->rkf.upload(rkf)) != hipSuccess || (e = m->rkd.upload(rkd)) != hipSuccess)
        return e == hipErrorOutOfMemory ? m->fail(IRE_E_NOMEM, "device allocation failed")
                                        : m->hip_fail(e, "table upload");
    if ((e = m->A.ensure((size_t)ire::kMaxReplicas * n * ire::kAccStride)) != hipSuccess ||
        (e = m->A_out.ensure(n)) != hipSuccess || (e = m->T_out.ensure(n)) != hipSuccess ||
        (e = m->stats.ensure(1)) != hipSuccess || (e = m->sed.ensure((size_t)4 * K)) != hipSuccess)
        return m->fail(IRE_E_NOMEM, "device allocation failed: %s", hipGetErrorString(e));
    m->dirty = false;
    return IRE_OK;
}

int check_ready(ire_model *m) {
    if (m->rho.empty()) return m->fail(IRE_E_STATE, "shells are not set");
    if (m->nu.empty()) return m->fail(IRE_E_STATE, "dust is not set");
    if (!m->J.empty() && m->J.size() != m->nu.size())
        return m->fail(IRE_E_STATE, "external field was set for a different frequency grid");
    if (!m->S.empty() && m->S.size() != m->nu.size())
        return m->fail(IRE_E_STATE, "point-source spectrum was set for a different frequency grid");
    return IRE_OK;
}

// Shape and parameters of one trace launch of the handle's current model and
// options (everything but the package energies, ids, seed and the accumulator,
// counter and spectrum buffers, which the caller fills in).
struct TraceLaunch {
    ire::TraceParams p{};
    int fp64 = 0, agg = 0, grid = 1, block = 64;
    size_t lds = 0;
};

int trace_launch_setup(ire_model *m, int replicas, uint64_t n_ext, uint64_t n_ps, TraceLaunch &L) {
    // schedule: with one running total per shell, per-lane or per-wave atomics on the few addresses bound
    // the launch, and grouping the absorptions of the whole workgroup (its waves pass together, at 48 parked
    // lanes, or once 2 waves are there) makes the fewest; with accumulator groups the launch is
    // instruction-bound, and per-wave grouping at 40 parked lanes is the better balance
    const int agg = m->opt.aggregate >= 0 ? m->opt.aggregate : (replicas > 1 ? 1 : 2);
    if (agg == 2 && m->rho.size() >= (1u << 22))
        return m->fail(IRE_E_INVALID, "aggregate = 2 supports fewer than 2^22 shells");
    hipError_t e;
    const int n = (int)m->rho.size(), K = (int)m->nu.size();
    const int fp64 = m->opt.stepping == IRE_FP64;
    // packages per lane: one for FP64 and for runs with a cap on packages in flight
    size_t lds = 0;
    int block, grid;
    if (fp64) {
        block = 256;
        grid = m->n_cu * 8;
    } else {
        lds = ire::trace_lds_bytes(n + (m->r_edges[0] > 0.0 ? 1 : 0) + ire::kSentinels, K, m->n_t);
        if (lds > m->max_lds)
            return m->fail(IRE_E_INVALID, "FP32 tables need %zu bytes of LDS, the device has %zu; use IRE_FP64",
                           lds, m->max_lds);
        if ((e = ire::trace_configure(0, agg, lds)) != hipSuccess) return m->hip_fail(e, "configure tracer");
        block = ire::trace_block_fp32();
        grid = m->n_cu;
    }
    if (m->opt.max_lanes > 0) {
        const int waves = (m->opt.max_lanes + 63) / 64;
        const int wpb = block / 64;
        grid = std::min(grid, (waves + wpb - 1) / wpb);
        if (grid < 1) grid = 1;
    }
    ire::TraceParams &p = L.p;
    p = ire::TraceParams{};
    p.n = n; p.K = K; p.n_t = m->n_t;
    p.cavity = m->r_edges[0] > 0.0 ? 1 : 0;
    p.shf = m->shf.p; p.dustf = m->dustf.p; p.cdff = m->cdff.p; p.Gf = m->Gf.p; p.Df = m->Df.p;
    p.shd = m->shd.p; p.dustd = m->dustd.p; p.cdfd = m->cdfd.p; p.Gd = m->Gd.p; p.Dd = m->Dd.p;
    p.invM = m->invM.p;
    p.guide = m->guide.p;
    p.g_lg0 = m->g_lg0;
    p.g_scale = m->g_scale;
    p.n_ext = n_ext; p.n_ps = n_ps;
    p.k_bg = m->opt.k_bg; p.ffi = m->opt.ffi; p.reemit_uniform = m->opt.reemit_uniform;
    p.w_floor = m->opt.w_floor; p.max_events = m->opt.max_events; p.max_lanes = m->opt.max_lanes;
    p.use_g_E = m->opt.use_g_E; p.g_E = m->opt.g_E; p.use_g_S = m->opt.use_g_S; p.g_S = m->opt.g_S;
    p.k_A = m->opt.k_A; p.k_S = m->opt.k_S;
    p.k_A_rho = m->opt.k_A_rho; p.rkf = m->rkf.p; p.rkd = m->rkd.p;
    p.replicas = replicas;
    {
        // packages a wave takes from the global cursor at a time: about 64 grabs
        // per wave and launch keep the waves' last grabs short (the launch ends
        // with its slowest wave), and one grab must cover a whole wave's refill
        const unsigned long long waves = (unsigned long long)grid * (block / 64);
        unsigned long long c = (n_ext + n_ps) / (waves * 64ull);
        p.chunk = std::min<unsigned long long>(std::max<unsigned long long>(c, 64ull), 4096ull);
    }
    // (forced first interactions add an absorption or scattering to every package: fuller passes, more
    // parked lanes and a larger quorum, then pay)
    p.batch = m->opt.batch > 0 ? m->opt.batch : (agg == 2 ? (m->opt.ffi ? 56 : 48) : (replicas > 1 ? 40 : 64));
    p.quorum = m->opt.quorum > 0 ? m->opt.quorum : (m->opt.ffi ? 3 : 2);
    L.fp64 = fp64;
    L.agg = agg;
    L.grid = grid;
    L.block = block;
    L.lds = lds;
    return IRE_OK;
}

// ---- the scratch of ire_run_noalloc: a fixed device array per GPU holding the
// run's event counters, tallies and package cursor, its escaping spectrum and
// its absorbed-energy accumulators, so that the call allocates nothing.
constexpr int kNoAllocShellCopies = 4096;    // shells x accumulator groups
constexpr int kNoAllocMaxK = 255;            // frequencies (the guide tables' limit too)
constexpr size_t kScratchStatsBytes = 256;
constexpr size_t kScratchSedBytes = 8192;    // >= 4 * kNoAllocMaxK doubles
constexpr size_t kScratchBytes =
    kScratchStatsBytes + kScratchSedBytes + (size_t)kNoAllocShellCopies * ire::kAccStride * sizeof(double);
static_assert(sizeof(ire::DevStats) <= kScratchStatsBytes, "scratch counters");
static_assert(4 * kNoAllocMaxK * sizeof(double) <= kScratchSedBytes, "scratch spectrum");

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};   // the array's device address on each GPU (HIP_SYMBOL is host-side only)

// Resolve the array's address on `device`, which must be current.  Once per
// device; later calls return the kept address.
hipError_t resolve_scratch(int device, void **out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_dev[device] = ptr;
    }
    *out = g_scratch_dev[device];
    return hipSuccess;
}

struct NoAllocScratch {
    ire::DevStats *stats = nullptr;
    double *sed = nullptr;
    double *A = nullptr;
};

int noalloc_scratch(ire_model *m, NoAllocScratch &sc) {
    void *base = nullptr;
    const hipError_t e = resolve_scratch(m->device, &base);
    if (e != hipSuccess) return m->hip_fail(e, "scratch address");
    unsigned char *b = static_cast<unsigned char *>(base);
    sc.stats = reinterpret_cast<ire::DevStats *>(b);
    sc.sed = reinterpret_cast<double *>(b + kScratchStatsBytes);
    sc.A = reinterpret_cast<double *>(b + kScratchStatsBytes + kScratchSedBytes);
    return IRE_OK;
}

}  // namespace

extern "C" {

int ire_default_options(ire_options *o) {
    if (!o) return IRE_E_INVALID;
    o->k_bg = 0.5;
    o->ffi = 0;
    o->w_floor = 1e-10;
    o->max_events = 1000000;
    o->stepping = IRE_FP32;
    o->max_lanes = 0;
    o->reemit_uniform = 0;
    o->aggregate = -1;
    o->batch = 0;
    o->use_g_E = 0;
    o->g_E = 0.0;
    o->use_g_S = 0;
    o->g_S = 0.0;
    o->k_A = 1.0;
    o->k_S = 1.0;
    o->k_A_rho = 0;
    o->k_A_lowest = 3.0;
    o->k_A_highest = 1.0;
    o->replicas = 1;
    o->quorum = 0;
    return IRE_OK;
}

int ire_create(int hip_device, ire_model **out) {
    if (!out) return IRE_E_INVALID;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || hip_device < 0 || hip_device >= count)
        return IRE_E_DEVICE;
    ire_model *m = new (std::nothrow) ire_model();
    if (!m) return IRE_E_NOMEM;
    m->device = hip_device;
    ire_default_options(&m->opt);
    if (hipSetDevice(hip_device) != hipSuccess ||
        hipDeviceGetAttribute(&m->n_cu, hipDeviceAttributeMultiprocessorCount, hip_device) != hipSuccess) {
        delete m;
        return IRE_E_DEVICE;
    }
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, hip_device) != hipSuccess) {
        delete m;
        return IRE_E_DEVICE;
    }
    m->max_lds = (size_t)lds;
    if (hipEventCreate(&m->ev0) != hipSuccess || hipEventCreate(&m->ev1) != hipSuccess) {
        delete m;
        return IRE_E_DEVICE;
    }
    // the no-allocation entry point's scratch address on this device, resolved
    // here with the device current (once per device)
    void *scratch_ptr = nullptr;
    if (resolve_scratch(hip_device, &scratch_ptr) != hipSuccess) {
        delete m;
        return IRE_E_DEVICE;
    }
    *out = m;
    return IRE_OK;
}

void ire_destroy(ire_model *m) {
    if (!m) return;
    (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    m->shf.release(); m->shd.release(); m->dustf.release(); m->dustd.release();
    m->cdff.release(); m->Gf.release(); m->Df.release(); m->cdfd.release(); m->Gd.release();
    m->Dd.release(); m->invM.release(); m->lnGd.release(); m->lnTd.release(); m->guide.release(); m->sed.release(); m->rkf.release(); m->rkd.release(); m->A.release();
    m->A_out.release(); m->T_out.release(); m->stats.release();
    if (m->ev0) (void)hipEventDestroy(m->ev0);
    if (m->ev1) (void)hipEventDestroy(m->ev1);
    delete m;
}

const char *ire_last_error(const ire_model *m) {
    return m ? m->err.c_str() : "null handle";
}

int ire_set_shells(ire_model *m, int32_t n, const double *r_edges, const double *rho) {
    if (!m) return IRE_E_INVALID;
    if (n < 1 || !r_edges || !rho) return m->fail(IRE_E_INVALID, "need n >= 1 shells and both arrays");
    if (!finite_all(r_edges, n + 1) || !finite_all(rho, n)) return m->fail(IRE_E_INVALID, "non-finite shell data");
    if (!(r_edges[0] >= 0.0)) return m->fail(IRE_E_INVALID, "r_edges[0] must be >= 0");
    for (int i = 0; i < n; ++i) {
        if (!(r_edges[i + 1] > r_edges[i])) return m->fail(IRE_E_INVALID, "r_edges must increase strictly (index %d)", i);
        if (!(rho[i] >= 0.0)) return m->fail(IRE_E_INVALID, "rho[%d] < 0", i);
    }
    m->r_edges.assign(r_edges, r_edges + n + 1);
    m->rho.assign(rho, rho + n);
    m->dirty = true;
    m->begun = false;
    return IRE_OK;
}

int ire_set_dust(ire_model *m, int32_t K, const double *nu, const double *kappa_abs,
                 const double *albedo, const double *g) {
    if (!m) return IRE_E_INVALID;
    if (K < 1 || K > ire::kMaxK || !nu || !kappa_abs || !albedo || !g)
        return m->fail(IRE_E_INVALID, "need 1 <= K <= %d and all dust arrays", ire::kMaxK);
    if (!finite_all(nu, K) || !finite_all(kappa_abs, K) || !finite_all(albedo, K) || !finite_all(g, K))
        return m->fail(IRE_E_INVALID, "non-finite dust data");
    for (int k = 0; k < K; ++k) {
        if (!(nu[k] > 0.0) || (k > 0 && !(nu[k] > nu[k - 1]))) return m->fail(IRE_E_INVALID, "nu must be positive and increase strictly (index %d)", k);
        if (!(kappa_abs[k] > 0.0)) return m->fail(IRE_E_INVALID, "kappa_abs[%d] must be > 0", k);
        if (!(albedo[k] >= 0.0 && albedo[k] < 1.0)) return m->fail(IRE_E_INVALID, "albedo[%d] must be in [0,1)", k);
        if (!(g[k] > -1.0 && g[k] < 1.0)) return m->fail(IRE_E_INVALID, "g[%d] must be in (-1,1)", k);
    }
    if (!m->J.empty() && (int)m->J.size() != K) m->J.clear();
    if (!m->S.empty() && (int)m->S.size() != K) { m->S.clear(); m->L_ps = 0.0; }
    m->nu.assign(nu, nu + K);
    m->kabs.assign(kappa_abs, kappa_abs + K);
    m->albedo.assign(albedo, albedo + K);
    m->g.assign(g, g + K);
    m->dirty = true;
    m->begun = false;
    return IRE_OK;
}

int ire_set_temperature_grid(ire_model *m, double t_min, double t_max, int32_t n_t) {
    if (!m) return IRE_E_INVALID;
    if (!(t_min > 0.0) || !(t_max > t_min) || !std::isfinite(t_max) || n_t < 2 || n_t > ire::kMaxGuideNt)
        return m->fail(IRE_E_INVALID, "need 0 < t_min < t_max and 2 <= n_t <= %d", ire::kMaxGuideNt);
    m->t_min = t_min;
    m->t_max = t_max;
    m->n_t = n_t;
    m->dirty = true;
    m->begun = false;
    return IRE_OK;
}

int ire_set_external_field(ire_model *m, const double *J_nu) {
    if (!m) return IRE_E_INVALID;
    if (!J_nu) { m->J.clear(); m->dirty = true; m->begun = false; return IRE_OK; }
    if (m->nu.empty()) return m->fail(IRE_E_STATE, "set the dust (frequency grid) before the external field");
    const int K = (int)m->nu.size();
    if (!finite_all(J_nu, K)) return m->fail(IRE_E_INVALID, "non-finite J_nu");
    for (int k = 0; k < K; ++k)
        if (!(J_nu[k] >= 0.0)) return m->fail(IRE_E_INVALID, "J_nu[%d] < 0", k);
    m->J.assign(J_nu, J_nu + K);
    m->dirty = true;
    m->begun = false;
    return IRE_OK;
}

int ire_set_point_source(ire_model *m, double L, const double *spectrum) {
    if (!m) return IRE_E_INVALID;
    if (L == 0.0) { m->S.clear(); m->L_ps = 0.0; m->dirty = true; m->begun = false; return IRE_OK; }
    if (!(L > 0.0) || !std::isfinite(L) || !spectrum) return m->fail(IRE_E_INVALID, "need L > 0 and a spectrum");
    if (m->nu.empty()) return m->fail(IRE_E_STATE, "set the dust (frequency grid) before the point source");
    const int K = (int)m->nu.size();
    if (!finite_all(spectrum, K)) return m->fail(IRE_E_INVALID, "non-finite spectrum");
    double tot = 0.0;
    for (int k = 0; k < K; ++k) {
        if (!(spectrum[k] >= 0.0)) return m->fail(IRE_E_INVALID, "spectrum[%d] < 0", k);
        tot += spectrum[k];
    }
    if (!(tot > 0.0)) return m->fail(IRE_E_INVALID, "spectrum is all zero");
    m->S.assign(spectrum, spectrum + K);
    m->L_ps = L;
    m->dirty = true;
    m->begun = false;
    return IRE_OK;
}

int ire_set_options(ire_model *m, const ire_options *o) {
    if (!m) return IRE_E_INVALID;
    if (!o) return m->fail(IRE_E_INVALID, "null options");
    if (!(o->k_bg > 0.0 && o->k_bg <= 1.0)) return m->fail(IRE_E_INVALID, "k_bg must be in (0,1]");
    if (!(o->w_floor >= 0.0 && o->w_floor < 1.0)) return m->fail(IRE_E_INVALID, "w_floor must be in [0,1)");
    if (o->stepping != IRE_FP32 && o->stepping != IRE_FP64) return m->fail(IRE_E_INVALID, "stepping must be IRE_FP32 or IRE_FP64");
    if (o->max_lanes < 0) return m->fail(IRE_E_INVALID, "max_lanes must be >= 0");
    if (o->ffi < 0 || o->ffi > 2) return m->fail(IRE_E_INVALID, "ffi must be 0, 1 or 2");
    const std::string we = ire::host::check_weights(o->use_g_E, o->g_E, o->use_g_S, o->g_S, o->k_A, o->k_S);
    if (!we.empty()) return m->fail(IRE_E_INVALID, "%s", we.c_str());
    if (o->k_A_rho != 0 && o->k_A_rho != 1) return m->fail(IRE_E_INVALID, "k_A_rho must be 0 or 1");
    if (o->k_A_rho && (o->k_A != 1.0 || !(o->k_A_lowest > 0.0) || !(o->k_A_highest > 0.0) ||
                       !std::isfinite(o->k_A_lowest) || !std::isfinite(o->k_A_highest)))
        return m->fail(IRE_E_INVALID, "k_A_rho needs k_A = 1 and finite k_A_lowest, k_A_highest > 0");
    if (o->k_A_lowest != m->opt.k_A_lowest || o->k_A_highest != m->opt.k_A_highest) m->dirty = true;
    if (o->reemit_uniform != 0 && o->reemit_uniform != 1) return m->fail(IRE_E_INVALID, "reemit_uniform must be 0 or 1");
    if (o->aggregate < -1 || o->aggregate > 2) return m->fail(IRE_E_INVALID, "aggregate must be -1, 0, 1 or 2");
    if (o->batch < 0 || o->batch > 64) return m->fail(IRE_E_INVALID, "batch must be in [0, 64]");
    if (o->replicas < 1 || o->replicas > ire::kMaxReplicas)
        return m->fail(IRE_E_INVALID, "replicas must be in [1, %d]", ire::kMaxReplicas);
    if (o->replicas > 1 && o->max_lanes > 0) return m->fail(IRE_E_INVALID, "replicas > 1 needs max_lanes = 0");
    if (o->quorum < 0 || o->quorum > 16) return m->fail(IRE_E_INVALID, "quorum must be in [0, 16]");
    m->opt = *o;
    return IRE_OK;
}

int ire_begin(ire_model *m, uint64_t n_ext_total, uint64_t n_ps_total, uint64_t seed) {
    if (!m) return IRE_E_INVALID;
    int rc = check_ready(m);
    if (rc) return rc;
    if (n_ext_total > 0 && m->J.empty()) return m->fail(IRE_E_STATE, "external packages requested but no external field is set");
    if (n_ps_total > 0 && m->S.empty()) return m->fail(IRE_E_STATE, "point-source packages requested but no point source is set");
    hipError_t e;
    if ((e = hipSetDevice(m->device)) != hipSuccess) return m->hip_fail(e, "hipSetDevice");
    if (m->dirty) {
        const auto start = std::chrono::steady_clock::now();
        rc = build_tables(m);
        if (rc) return rc;
        m->ms_tables = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - start).count();
    }
    if (n_ext_total > 0 && !(m->L_ext > 0.0)) return m->fail(IRE_E_STATE, "the external field carries no power on this grid");
    m->n_total[0] = n_ext_total;
    m->n_total[1] = n_ps_total;
    m->n_done[0] = m->n_done[1] = 0;
    m->seed = seed;
    m->eps[0] = n_ext_total ? m->L_ext / (double)n_ext_total : 0.0;
    m->eps[1] = n_ps_total ? m->L_ps / (double)n_ps_total : 0.0;
    m->ms_trace = 0.0f;
    m->ms_finalize = 0.0f;
    m->timed = false;
    m->replicas = m->opt.replicas;   // fixed for the run: every ire_advance of it uses the same groups
    if ((e = ire::launch_zero(m->A.p, ire::kMaxReplicas * (int)m->rho.size(), m->stats.p, 1, m->sed.p,
                              4 * (int)m->nu.size(), nullptr)) != hipSuccess)
        return m->hip_fail(e, "zero accumulators");
    if ((e = hipStreamSynchronize(nullptr)) != hipSuccess) return m->hip_fail(e, "zero accumulators");
    m->begun = true;
    return IRE_OK;
}

int ire_advance(ire_model *m, uint64_t n_ext, uint64_t n_ps, void *hip_stream) {
    if (!m) return IRE_E_INVALID;
    if (!m->begun || m->dirty) return m->fail(IRE_E_STATE, "ire_begin must precede ire_advance (and follow any setter)");
    if (n_ext > m->n_total[0] - m->n_done[0] || n_ps > m->n_total[1] - m->n_done[1])
        return m->fail(IRE_E_INVALID, "more packages requested than remain in the run");
    if (n_ext + n_ps == 0) return IRE_OK;
    if (m->replicas > 1 && m->opt.max_lanes > 0)
        return m->fail(IRE_E_STATE, "a run begun with replicas > 1 cannot continue with max_lanes > 0");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    hipError_t e;
    if ((e = hipSetDevice(m->device)) != hipSuccess) return m->hip_fail(e, "hipSetDevice");
    TraceLaunch L;
    int rc = trace_launch_setup(m, m->replicas, n_ext, n_ps, L);
    if (rc) return rc;
    ire::TraceParams &p = L.p;
    p.eps[0] = m->eps[0]; p.eps[1] = m->eps[1];
    p.pid0[0] = m->n_done[0]; p.pid0[1] = m->n_done[1];
    p.seed = m->seed;
    p.A = m->A.p; p.stats = m->stats.p; p.sed = m->sed.p;
    if ((e = ire::launch_zero(nullptr, 0, m->stats.p, 0, nullptr, 0, s)) != hipSuccess) return m->hip_fail(e, "cursor reset");
    if ((e = hipEventRecord(m->ev0, s)) != hipSuccess) return m->hip_fail(e, "event");
    if ((e = ire::launch_trace(p, L.fp64, L.agg, L.grid, L.block, L.lds, s)) != hipSuccess)
        return m->hip_fail(e, "trace launch");
    if ((e = hipEventRecord(m->ev1, s)) != hipSuccess) return m->hip_fail(e, "event");
    m->timed = true;
    m->last_stream = s;
    m->n_done[0] += n_ext;
    m->n_done[1] += n_ps;
    return IRE_OK;
}

int ire_run_noalloc(ire_model *m, uint64_t n_ext, uint64_t n_ps, uint64_t seed, double *absorbed_dev,
                    double *T_dev, void *hip_stream) {
    if (!m) return IRE_E_INVALID;
    int rc = check_ready(m);
    if (rc) return rc;
    if (m->dirty)
        return m->fail(IRE_E_STATE, "the model's tables are not on the device: call ire_run (or ire_begin) after "
                                    "the last setter before ire_run_noalloc");
    if (n_ext > 0 && m->J.empty()) return m->fail(IRE_E_STATE, "external packages requested but no external field is set");
    if (n_ps > 0 && m->S.empty()) return m->fail(IRE_E_STATE, "point-source packages requested but no point source is set");
    if (n_ext > 0 && !(m->L_ext > 0.0)) return m->fail(IRE_E_STATE, "the external field carries no power on this grid");
    const int n = (int)m->rho.size(), K = (int)m->nu.size();
    if (n > 0 && (!absorbed_dev || !T_dev)) return m->fail(IRE_E_INVALID, "null output");
    const int R = m->opt.replicas;
    if ((long long)n * R > kNoAllocShellCopies)
        return m->fail(IRE_E_INVALID, "ire_run_noalloc holds at most %d shells x accumulator groups, not %d x %d",
                       kNoAllocShellCopies, n, R);
    if (K > kNoAllocMaxK) return m->fail(IRE_E_INVALID, "ire_run_noalloc holds at most %d frequencies", kNoAllocMaxK);
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    hipError_t e;
    if ((e = hipSetDevice(m->device)) != hipSuccess) return m->hip_fail(e, "hipSetDevice");
    NoAllocScratch sc;
    if ((rc = noalloc_scratch(m, sc)) != IRE_OK) return rc;
    // the scratch keeps the last call's contents: clear the accumulators, counters,
    // tallies, cursor and escaping spectrum with a fill kernel
    if ((e = ire::launch_zero(sc.A, R * n, sc.stats, 1, sc.sed, 4 * K, s)) != hipSuccess)
        return m->hip_fail(e, "clear scratch");
    if (n_ext + n_ps > 0) {
        TraceLaunch L;
        if ((rc = trace_launch_setup(m, R, n_ext, n_ps, L)) != IRE_OK) return rc;
        ire::TraceParams &p = L.p;
        p.eps[0] = n_ext ? m->L_ext / (double)n_ext : 0.0;
        p.eps[1] = n_ps ? m->L_ps / (double)n_ps : 0.0;
        p.pid0[0] = 0; p.pid0[1] = 0;
        p.seed = seed;
        p.A = sc.A; p.stats = sc.stats; p.sed = sc.sed;
        if ((e = ire::launch_trace(p, L.fp64, L.agg, L.grid, L.block, L.lds, s)) != hipSuccess)
            return m->hip_fail(e, "trace launch");
    }
    ire::FinalizeParams f{};
    f.n = n;
    f.n_t = m->n_t;
    f.A = sc.A; f.invM = m->invM.p; f.Gd = m->Gd.p; f.lnG = m->lnGd.p; f.lnT = m->lnTd.p;
    f.replicas = R;
    f.t_min = m->t_min; f.t_max = m->t_max;
    f.A_out = absorbed_dev; f.T_out = T_dev;
    f.stats = sc.stats;
    if ((e = ire::launch_finalize(f, s)) != hipSuccess) return m->hip_fail(e, "finalize launch");
    return IRE_OK;
}

int ire_run(ire_model *m, uint64_t n_ext, uint64_t n_ps, uint64_t seed, void *hip_stream) {
    int rc = ire_begin(m, n_ext, n_ps, seed);
    if (rc) return rc;
    return ire_advance(m, n_ext, n_ps, hip_stream);
}

int ire_reset(ire_model *m) {
    if (!m) return IRE_E_INVALID;
    if (!m->begun) return IRE_OK;
    return ire_begin(m, m->n_total[0], m->n_total[1], m->seed);
}

int ire_tune_schedule(ire_model *m, uint64_t n_ext, uint64_t n_ps, int32_t *quorum, int32_t *batch) {
    if (!m) return IRE_E_INVALID;
    if (n_ext + n_ps == 0) return m->fail(IRE_E_INVALID, "no packages to tune with");
    if (m->opt.max_lanes > 0) return m->fail(IRE_E_INVALID, "tuning needs max_lanes = 0");
    // a sample of at most 2e7 packages in the run's proportions
    const double cap = 2e7, tot = (double)n_ext + (double)n_ps;
    const double f = tot > cap ? cap / tot : 1.0;
    uint64_t ne = (uint64_t)((double)n_ext * f), np = (uint64_t)((double)n_ps * f);
    if (n_ext && !ne) ne = 1;
    if (n_ps && !np) np = 1;
    const int agg = m->opt.aggregate >= 0 ? m->opt.aggregate : (m->opt.replicas > 1 ? 1 : 2);
    std::vector<std::pair<int, int>> cand;   // (quorum, batch)
    if (agg == 2 && m->opt.stepping == IRE_FP32) {
        for (int q : {2, 3, 4, 6})
            for (int b : {36, 40, 44, 48, 52}) cand.emplace_back(q, b);
    } else {
        for (int b : {24, 32, 40, 48, 64}) cand.emplace_back(m->opt.quorum, b);
    }
    const ire_options keep = m->opt;
    float best_ms = -1.0f;
    std::pair<int, int> best = cand[0];
    int rc = IRE_OK;
    for (size_t c = 0; c <= cand.size() && rc == IRE_OK; ++c) {
        // candidate 0 runs twice: the first launch is not timed
        const auto &qb = cand[c == 0 ? 0 : c - 1];
        m->opt.quorum = qb.first;
        m->opt.batch = qb.second;
        if ((rc = ire_begin(m, ne, np, 1)) != IRE_OK || (rc = ire_advance(m, ne, np, nullptr)) != IRE_OK) break;
        hipError_t e;
        if ((e = hipEventSynchronize(m->ev1)) != hipSuccess) { rc = m->hip_fail(e, "tuning launch"); break; }
        float ms = 0.0f;
        if ((e = hipEventElapsedTime(&ms, m->ev0, m->ev1)) != hipSuccess) { rc = m->hip_fail(e, "tuning timer"); break; }
        if (c > 0 && (best_ms < 0.0f || ms < best_ms)) {
            best_ms = ms;
            best = qb;
        }
    }
    m->opt = keep;
    m->begun = false;
    m->timed = false;
    if (rc != IRE_OK) return rc;
    m->opt.quorum = best.first;
    m->opt.batch = best.second;
    if (quorum) *quorum = best.first;
    if (batch) *batch = best.second;
    return IRE_OK;
}

int ire_sync(ire_model *m) {
    if (!m) return IRE_E_INVALID;
    hipError_t e;
    if ((e = hipSetDevice(m->device)) != hipSuccess) return m->hip_fail(e, "hipSetDevice");
    if ((e = hipDeviceSynchronize()) != hipSuccess) return m->hip_fail(e, "synchronize");
    return IRE_OK;
}

static int finalize(ire_model *m, hipStream_t s) {
    ire::FinalizeParams f{};
    f.n = (int)m->rho.size();
    f.n_t = m->n_t;
    f.A = m->A.p; f.invM = m->invM.p; f.Gd = m->Gd.p; f.lnG = m->lnGd.p; f.lnT = m->lnTd.p;
    f.replicas = m->replicas;
    f.t_min = m->t_min; f.t_max = m->t_max;
    f.A_out = m->A_out.p; f.T_out = m->T_out.p;
    f.stats = m->stats.p;
    hipError_t e = ire::launch_finalize(f, s);
    if (e != hipSuccess) return m->hip_fail(e, "finalize launch");
    return IRE_OK;
}

static void fill_stats(const ire_model *m, const ire::DevStats &hs, ire_stats *stats) {
    if (stats) {
        stats->L_ext = m->n_total[0] ? m->L_ext : 0.0;
        stats->L_ps = m->n_total[1] ? m->L_ps : 0.0;
        stats->escaped[0] = hs.tally[ire::T_ESC_EXT];
        stats->escaped[1] = hs.tally[ire::T_ESC_PS];
        stats->ffi_escaped = hs.tally[ire::T_FFI];
        stats->terminated = hs.tally[ire::T_TERM];
        stats->n_launch = hs.cnt[ire::C_LAUNCH];
        stats->n_cross = hs.cnt[ire::C_CROSS];
        stats->n_scat = hs.cnt[ire::C_SCAT];
        stats->n_abs = hs.cnt[ire::C_ABS];
        stats->n_escape = hs.cnt[ire::C_ESCAPE];
        stats->n_direct = hs.cnt[ire::C_DIRECT];
        stats->n_limit = hs.cnt[ire::C_LIMIT];
        stats->n_floor = hs.cnt[ire::C_FLOOR];
        stats->n_below = hs.cnt[ire::C_BELOW];
        stats->n_above = hs.cnt[ire::C_ABOVE];
        stats->n_reemit_above = hs.cnt[ire::C_REEMIT_ABOVE];
        stats->n_pass = hs.cnt[ire::C_PASS];
        stats->n_step_slots = hs.cnt[ire::C_SLOTS];
        stats->ms_tables = m->ms_tables;
        stats->ms_trace = m->ms_trace;
        stats->ms_finalize = m->ms_finalize;
    }
}

int ire_get_results(ire_model *m, double *absorbed, double *T, ire_stats *stats) {
    if (!m) return IRE_E_INVALID;
    if (!m->begun) return m->fail(IRE_E_STATE, "no run to report");
    hipError_t e;
    if ((e = hipSetDevice(m->device)) != hipSuccess) return m->hip_fail(e, "hipSetDevice");
    hipStream_t s = m->last_stream;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return m->hip_fail(e, "synchronize");
    if (m->timed) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, m->ev0, m->ev1) == hipSuccess) m->ms_trace = ms;
    }
    // the clamp counters are recomputed by each finalize
    ire::DevStats hs;
    if ((e = hipMemcpy(&hs, m->stats.p, sizeof(hs), hipMemcpyDeviceToHost)) != hipSuccess)
        return m->hip_fail(e, "stats copy");
    hs.cnt[ire::C_BELOW] = 0;
    hs.cnt[ire::C_ABOVE] = 0;
    if ((e = hipMemcpy(m->stats.p, &hs, sizeof(hs), hipMemcpyHostToDevice)) != hipSuccess)
        return m->hip_fail(e, "stats copy");
    if ((e = hipEventRecord(m->ev0, s)) != hipSuccess) return m->hip_fail(e, "event");
    int rc = finalize(m, s);
    if (rc) return rc;
    if ((e = hipEventRecord(m->ev1, s)) != hipSuccess) return m->hip_fail(e, "event");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return m->hip_fail(e, "finalize");
    float msf = 0.0f;
    if (hipEventElapsedTime(&msf, m->ev0, m->ev1) == hipSuccess) m->ms_finalize = msf;
    m->timed = false;
    const size_t n = m->rho.size();
    if (absorbed && (e = hipMemcpy(absorbed, m->A_out.p, n * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess)
        return m->hip_fail(e, "copy absorbed");
    if (T && (e = hipMemcpy(T, m->T_out.p, n * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess)
        return m->hip_fail(e, "copy T");
    if ((e = hipMemcpy(&hs, m->stats.p, sizeof(hs), hipMemcpyDeviceToHost)) != hipSuccess)
        return m->hip_fail(e, "stats copy");
    fill_stats(m, hs, stats);
    if (hs.cnt[ire::C_LIMIT] > 0) return m->fail(IRE_E_LIMIT, "%llu packages reached max_events", hs.cnt[ire::C_LIMIT]);
    return IRE_OK;
}

int ire_get_stats(ire_model *m, ire_stats *stats) {
    if (!m) return IRE_E_INVALID;
    if (!m->begun) return m->fail(IRE_E_STATE, "no run to report");
    hipError_t e;
    if ((e = hipSetDevice(m->device)) != hipSuccess) return m->hip_fail(e, "hipSetDevice");
    if ((e = hipStreamSynchronize(m->last_stream)) != hipSuccess) return m->hip_fail(e, "synchronize");
    if (m->timed) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, m->ev0, m->ev1) == hipSuccess) m->ms_trace = ms;
    }
    ire::DevStats hs;
    if ((e = hipMemcpy(&hs, m->stats.p, sizeof(hs), hipMemcpyDeviceToHost)) != hipSuccess)
        return m->hip_fail(e, "stats copy");
    fill_stats(m, hs, stats);
    return IRE_OK;
}

int ire_get_sed(ire_model *m, double *sed, double *sed_direct) {
    if (!m) return IRE_E_INVALID;
    if (!m->begun) return m->fail(IRE_E_STATE, "no run to report");
    const size_t K = m->nu.size();
    hipError_t e;
    if ((e = hipSetDevice(m->device)) != hipSuccess) return m->hip_fail(e, "hipSetDevice");
    if ((e = hipStreamSynchronize(m->last_stream)) != hipSuccess) return m->hip_fail(e, "synchronize");
    std::vector<double> h(4 * K);
    if ((e = hipMemcpy(h.data(), m->sed.p, h.size() * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess)
        return m->hip_fail(e, "spectrum copy");
    if (sed) std::copy(h.begin(), h.begin() + 2 * K, sed);
    if (sed_direct) std::copy(h.begin() + 2 * K, h.end(), sed_direct);
    return IRE_OK;
}

int ire_get_results_dev(ire_model *m, double *absorbed_dev, double *T_dev, void *hip_stream) {
    if (!m) return IRE_E_INVALID;
    if (!m->begun) return m->fail(IRE_E_STATE, "no run to report");
    hipError_t e;
    if ((e = hipSetDevice(m->device)) != hipSuccess) return m->hip_fail(e, "hipSetDevice");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    ire::FinalizeParams f{};
    f.n = (int)m->rho.size();
    f.n_t = m->n_t;
    f.A = m->A.p; f.invM = m->invM.p; f.Gd = m->Gd.p; f.lnG = m->lnGd.p; f.lnT = m->lnTd.p;
    f.replicas = m->replicas;
    f.t_min = m->t_min; f.t_max = m->t_max;
    f.A_out = absorbed_dev ? absorbed_dev : m->A_out.p;
    f.T_out = T_dev ? T_dev : m->T_out.p;
    f.stats = m->stats.p;
    if ((e = ire::launch_finalize(f, s)) != hipSuccess) return m->hip_fail(e, "finalize launch");
    return IRE_OK;
}

int ire_planck(int32_t K, const double *nu, double T, double *out) {
    if (K < 1 || !nu || !out || !std::isfinite(T)) return IRE_E_INVALID;
    for (int k = 0; k < K; ++k) out[k] = ire::host::planck(nu[k], T);
    return IRE_OK;
}

}  // extern "C"
