// Batched parameter studies (include/ire.h, ire_batch_*): many cloud models in
// one persistent launch, replayed as a captured HIP graph, with a schedule
// autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "ire.h"
#include "ire_host.h"
#include "ire_internal.h"

using ire::host::DevBuf;
using ire::host::kPi;

struct ire_batch {
    int device = 0;
    std::string err;
    // shared physics
    std::vector<double> nu, kabs, albedo, g;
    double t_min = 3.0, t_max = 1600.0;
    int n_t = 512;
    std::vector<double> J, S;
    // models
    std::vector<ire_model_desc> models;
    std::vector<double> r_edges, rho;  // flat
    ire_batch_options opt{};
    bool dirty = true;
    // derived
    ire::host::DustTables dt;
    std::vector<ire::BatchModelDev> mdev;
    std::vector<ire::BatchItemDev> items;
    size_t n_shells = 0;
    int max_table = 0;
    double L_total = 0.0;
    // device
    DevBuf<ire::ShellF> shells;
    DevBuf<float2> rkf;               // k_A(rho) records, laid out as `shells` (only with k_A_rho)
    DevBuf<ire::DustF> dustf;
    DevBuf<float> cdff, Gf, Df;
    DevBuf<unsigned char> guide;
    float g_lg0 = 0.0f, g_scale = 0.0f;
    DevBuf<double> Gd, lnG, lnT, invM, A, A_out, T_out;
    DevBuf<ire::BatchModelDev> models_d;
    DevBuf<ire::BatchItemDev> items_d;
    DevBuf<ire::DevStats> stats;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipStream_t last_stream = nullptr;
    bool ran = false;
    int n_cu = 0;
    size_t max_lds = 0;
    std::string dev_name;

    int fail(int code, const char *fmt, ...) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        err = buf;
        return code;
    }
    int hip_fail(hipError_t e, const char *what) { return fail(IRE_E_DEVICE, "%s: %s", what, hipGetErrorString(e)); }
    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
};

namespace {

size_t lds_bytes(const ire_batch *b) {
    return ire::batch_lds_bytes(b->max_table, (int)b->nu.size(), b->n_t, b->opt.k_A_rho != 0);
}

// Build all tables, the per-model records and the ordered work items; upload.
int prepare(ire_batch *b) {
    if (b->nu.empty()) return b->fail(IRE_E_STATE, "dust is not set");
    if (b->models.empty()) return b->fail(IRE_E_STATE, "models are not set");
    const int K = (int)b->nu.size();
    std::string e = ire::host::build_dust_tables(b->nu, b->kabs, b->albedo, b->g, b->t_min, b->t_max, b->n_t, b->dt);
    if (!e.empty()) return b->fail(IRE_E_INVALID, "%s", e.c_str());
    const std::vector<double> &w = b->dt.w;

    // source spectra: CDFs and the external field's integral
    std::vector<double> q(K), cdf(2 * K, 1.0);
    double sumJ = 0.0;
    if (!b->J.empty()) {
        for (int k = 0; k < K; ++k) { q[k] = b->J[k] * w[k]; sumJ += q[k]; }
        ire::host::cumulative(q.data(), K, cdf.data());
    }
    if (!b->S.empty()) {
        for (int k = 0; k < K; ++k) q[k] = b->S[k] * w[k];
        ire::host::cumulative(q.data(), K, cdf.data() + K);
    }
    // median frequency of each source spectrum (for the cost estimate)
    int kmed[2] = {0, 0};
    for (int s = 0; s < 2; ++s)
        while (kmed[s] < K - 1 && cdf[s * K + kmed[s]] < 0.5) kmed[s]++;

    std::vector<ire::ShellF> shf;
    std::vector<float2> rkf;
    std::vector<ire::ShellD> shd;
    std::vector<double> invM;
    b->mdev.clear();
    b->max_table = 0;
    b->L_total = 0.0;
    struct Cost { double per_pkg; };
    std::vector<Cost> cost;
    size_t r_off = 0, d_off = 0;
    for (size_t m = 0; m < b->models.size(); ++m) {
        const ire_model_desc &md = b->models[m];
        const int n = md.n_shells;
        const double *re = b->r_edges.data() + r_off;
        const double *rh = b->rho.data() + d_off;
        ire::BatchModelDev dm{};
        dm.shell_off = (int)shf.size();
        dm.n = n;
        dm.cav = re[0] > 0.0 ? 1 : 0;
        dm.src = md.source;
        dm.acc_off = (int)d_off;
        ire::host::build_shell_table(re, rh, n, shf, shd, invM);
        if (b->opt.k_A_rho) {
            // the model's absorption scaling over its own shells' densities, at its shell_off
            std::vector<float2> mf;
            std::vector<double2> md;
            ire::host::build_absorption_scaling(re, rh, n, b->opt.k_A_lowest, b->opt.k_A_highest, mf, md);
            rkf.insert(rkf.end(), mf.begin(), mf.end());
        }
        const double R = re[n];
        const double L = md.source == IRE_SRC_EXTERNAL ? 4.0 * kPi * R * R * kPi * sumJ * md.scale : md.scale;
        dm.eps = L / (double)md.n_packages;
        dm.n_pkg = md.n_packages;
        dm.seed = md.seed;
        b->L_total += L;
        b->mdev.push_back(dm);
        b->max_table = std::max(b->max_table, n + dm.cav + ire::kSentinels);
        // cost per package: shells crossed per flight times (1 + extinction depth at the median frequency)
        const int km = kmed[md.source == IRE_SRC_EXTERNAL ? 0 : 1];
        const double kext = b->kabs[km] / (1.0 - b->albedo[km]);
        double tau = 0.0;
        for (int i = 0; i < n; ++i) tau += kext * rh[i] * (re[i + 1] - re[i]);
        cost.push_back(Cost{(double)(n + dm.cav) * (1.0 + tau)});
        r_off += (size_t)n + 1;
        d_off += (size_t)n;
    }
    b->n_shells = d_off;

    // work items, most expensive first
    const unsigned long long item = b->opt.item_packages ? b->opt.item_packages : 524288ull;
    b->items.clear();
    std::vector<double> icost;
    for (size_t m = 0; m < b->models.size(); ++m) {
        const unsigned long long N = b->models[m].n_packages;
        for (unsigned long long f = 0; f < N; f += item) {
            const unsigned long long c = std::min(item, N - f);
            b->items.push_back(ire::BatchItemDev{(int)m, 0, f, c});
            icost.push_back(cost[m].per_pkg * (double)c);
        }
    }
    std::vector<size_t> order(b->items.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return icost[x] > icost[y]; });
    std::vector<ire::BatchItemDev> sorted;
    sorted.reserve(order.size());
    for (size_t j : order) sorted.push_back(b->items[j]);
    b->items.swap(sorted);

    if (lds_bytes(b) > b->max_lds)
        return b->fail(IRE_E_INVALID, "tables need %zu bytes of LDS, the device has %zu", lds_bytes(b), b->max_lds);

    std::vector<float> cdff(cdf.begin(), cdf.end()), Gf(b->dt.G.begin(), b->dt.G.end()), Df(b->dt.D.begin(), b->dt.D.end());
    std::vector<unsigned char> guide;
    ire::host::build_guides(b->dt, guide, b->g_lg0, b->g_scale);
    hipError_t he;
    if ((he = hipSetDevice(b->device)) != hipSuccess) return b->hip_fail(he, "hipSetDevice");
    if (b->opt.k_A_rho && (he = b->rkf.upload(rkf)) != hipSuccess)
        return he == hipErrorOutOfMemory ? b->fail(IRE_E_NOMEM, "device allocation failed") : b->hip_fail(he, "upload");
    if ((he = b->shells.upload(shf)) != hipSuccess || (he = b->dustf.upload(b->dt.df)) != hipSuccess ||
        (he = b->cdff.upload(cdff)) != hipSuccess || (he = b->Gf.upload(Gf)) != hipSuccess ||
        (he = b->Df.upload(Df)) != hipSuccess || (he = b->Gd.upload(b->dt.G)) != hipSuccess ||
        (he = b->lnG.upload(b->dt.lnG)) != hipSuccess || (he = b->lnT.upload(b->dt.lnT)) != hipSuccess ||
        (he = b->invM.upload(invM)) != hipSuccess || (he = b->models_d.upload(b->mdev)) != hipSuccess ||
        (he = b->items_d.upload(b->items)) != hipSuccess || (he = b->guide.upload(guide)) != hipSuccess)
        return he == hipErrorOutOfMemory ? b->fail(IRE_E_NOMEM, "device allocation failed") : b->hip_fail(he, "upload");
    if ((he = b->A.ensure(b->n_shells * ire::kAccStride)) != hipSuccess || (he = b->A_out.ensure(b->n_shells)) != hipSuccess ||
        (he = b->T_out.ensure(b->n_shells)) != hipSuccess || (he = b->stats.ensure(1)) != hipSuccess)
        return b->fail(IRE_E_NOMEM, "device allocation failed: %s", hipGetErrorString(he));
    b->drop_graph();
    b->dirty = false;
    return IRE_OK;
}

// Queue zero + trace + finalize on stream s.
int enqueue(ire_batch *b, hipStream_t s) {
    ire::BatchParams p{};
    p.K = (int)b->nu.size();
    p.n_t = b->n_t;
    p.n_items = (int)b->items.size();
    p.max_table = b->max_table;
    p.shells = b->shells.p;
    p.dustf = b->dustf.p;
    p.cdff = b->cdff.p;
    p.Gf = b->Gf.p;
    p.Df = b->Df.p;
    p.invM = b->invM.p;
    p.guide = b->guide.p;
    p.g_lg0 = b->g_lg0;
    p.g_scale = b->g_scale;
    p.A = b->A.p;
    p.models = b->models_d.p;
    p.items = b->items_d.p;
    p.k_bg = b->opt.k_bg;
    p.ffi = b->opt.ffi;
    p.reemit_uniform = b->opt.reemit_uniform;
    p.batch = b->opt.batch > 0 ? b->opt.batch : 32;
    p.w_floor = b->opt.w_floor;
    p.max_events = b->opt.max_events;
    p.use_g_E = b->opt.use_g_E;
    p.g_E = b->opt.g_E;
    p.use_g_S = b->opt.use_g_S;
    p.g_S = b->opt.g_S;
    p.k_A = b->opt.k_A;
    p.k_S = b->opt.k_S;
    p.k_A_rho = b->opt.k_A_rho;
    p.rkf = b->opt.k_A_rho ? b->rkf.p : nullptr;
    p.stats = b->stats.p;
    const size_t lds = lds_bytes(b);
    hipError_t e;
    if ((e = ire::launch_zero_batch(b->A.p, b->n_shells, b->stats.p, s)) != hipSuccess) return b->hip_fail(e, "zero");
    const int grid = std::max(1, std::min(b->n_cu, p.n_items));
    if ((e = ire::launch_trace_batch(p, b->opt.aggregate, grid, lds, s)) != hipSuccess)
        return b->hip_fail(e, "trace");
    ire::BatchFinalizeParams f{};
    f.n_shells = (int)b->n_shells;
    f.n_t = b->n_t;
    f.A = b->A.p;
    f.invM = b->invM.p;
    f.Gd = b->Gd.p;
    f.lnG = b->lnG.p;
    f.lnT = b->lnT.p;
    f.t_min = b->t_min;
    f.t_max = b->t_max;
    f.A_out = b->A_out.p;
    f.T_out = b->T_out.p;
    f.stats = b->stats.p;
    if ((e = ire::launch_finalize_batch(f, s)) != hipSuccess) return b->hip_fail(e, "finalize");
    return IRE_OK;
}

int run_on(ire_batch *b, hipStream_t s) {
    hipError_t e;
    if ((e = hipSetDevice(b->device)) != hipSuccess) return b->hip_fail(e, "hipSetDevice");
    if (b->dirty) {
        int rc = prepare(b);
        if (rc) return rc;
    }
    if ((e = ire::batch_configure(b->opt.aggregate, lds_bytes(b))) != hipSuccess)
        return b->hip_fail(e, "configure");
    if ((e = hipEventRecord(b->ev0, s)) != hipSuccess) return b->hip_fail(e, "event");
    if (b->opt.use_graph) {
        if (!b->exec) {
            if ((e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
                return b->hip_fail(e, "begin capture");
            int rc = enqueue(b, b->cap);
            hipGraph_t gph = nullptr;
            hipError_t e2 = hipStreamEndCapture(b->cap, &gph);
            if (rc) { if (gph) (void)hipGraphDestroy(gph); return rc; }
            if (e2 != hipSuccess) return b->hip_fail(e2, "end capture");
            b->graph = gph;
            if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess) {
                b->drop_graph();
                return b->hip_fail(e, "graph instantiate");
            }
        }
        if ((e = hipGraphLaunch(b->exec, s)) != hipSuccess) return b->hip_fail(e, "graph launch");
    } else {
        int rc = enqueue(b, s);
        if (rc) return rc;
    }
    if ((e = hipEventRecord(b->ev1, s)) != hipSuccess) return b->hip_fail(e, "event");
    b->last_stream = s;
    b->ran = true;
    return IRE_OK;
}

std::string class_key(const ire_batch *b) {
    // device, dust grid, and the batch's size class (models, mean shells, mean packages)
    double shells = 0.0, pk = 0.0;
    for (const auto &m : b->models) {
        shells += m.n_shells;
        pk += (double)m.n_packages;
    }
    const double M = (double)std::max<size_t>(1, b->models.size());
    char buf[256];
    snprintf(buf, sizeof(buf), "%s|K=%zu|nt=%d|logM=%d|shells=%d|logN=%d|ffi=%d", b->dev_name.c_str(), b->nu.size(),
             b->n_t, (int)std::lround(std::log2(M)), (int)std::lround(shells / M / 20.0) * 20,
             (int)std::lround(std::log10(std::max(1.0, pk / M))), b->opt.ffi);
    return buf;
}

bool cache_lookup(const char *path, const std::string &key, int &batch, unsigned long long &item) {
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        const std::string kq = "\"key\": \"" + key + "\"";
        if (line.find(kq) == std::string::npos) continue;
        int bt = 0;
        unsigned long long it = 0;
        const size_t pb = line.find("\"batch\": ");
        const size_t pi = line.find("\"item_packages\": ");
        if (pb == std::string::npos || pi == std::string::npos) continue;
        bt = std::atoi(line.c_str() + pb + 9);
        it = std::strtoull(line.c_str() + pi + 17, nullptr, 10);
        if (bt > 0 && it > 0) {
            batch = bt;
            item = it;
            found = true;
        }
    }
    return found;
}

}  // namespace

extern "C" {

int ire_batch_default_options(ire_batch_options *o) {
    if (!o) return IRE_E_INVALID;
    o->k_bg = 0.5;
    o->ffi = 0;
    o->w_floor = 1e-10;
    o->max_events = 1000000;
    o->reemit_uniform = 0;
    o->aggregate = 1;
    o->batch = 0;
    o->item_packages = 524288;
    o->use_graph = 1;
    o->use_g_E = 0;
    o->g_E = 0.0;
    o->use_g_S = 0;
    o->g_S = 0.0;
    o->k_A = 1.0;
    o->k_S = 1.0;
    o->k_A_rho = 0;
    o->k_A_lowest = 3.0;
    o->k_A_highest = 1.0;
    return IRE_OK;
}

int ire_batch_create(int hip_device, ire_batch **out) {
    if (!out) return IRE_E_INVALID;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || hip_device < 0 || hip_device >= count) return IRE_E_DEVICE;
    ire_batch *b = new (std::nothrow) ire_batch();
    if (!b) return IRE_E_NOMEM;
    b->device = hip_device;
    ire_batch_default_options(&b->opt);
    int lds = 0;
    hipDeviceProp_t prop;
    if (hipSetDevice(hip_device) != hipSuccess ||
        hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount, hip_device) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, hip_device) != hipSuccess ||
        hipGetDeviceProperties(&prop, hip_device) != hipSuccess || hipStreamCreate(&b->cap) != hipSuccess ||
        hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess) {
        delete b;
        return IRE_E_DEVICE;
    }
    b->max_lds = (size_t)lds;
    b->dev_name = prop.gcnArchName;
    *out = b;
    return IRE_OK;
}

void ire_batch_destroy(ire_batch *b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();
    b->drop_graph();
    b->shells.release(); b->dustf.release(); b->cdff.release(); b->Gf.release(); b->Df.release();
    b->Gd.release(); b->lnG.release(); b->lnT.release(); b->invM.release(); b->guide.release(); b->A.release();
    b->A_out.release(); b->T_out.release(); b->models_d.release(); b->items_d.release(); b->stats.release();
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    delete b;
}

const char *ire_batch_last_error(const ire_batch *b) { return b ? b->err.c_str() : "null handle"; }

int ire_batch_set_dust(ire_batch *b, int32_t K, const double *nu, const double *kappa_abs, const double *albedo,
                       const double *g) {
    if (!b) return IRE_E_INVALID;
    const std::string e = ire::host::check_dust(K, nu, kappa_abs, albedo, g);
    if (!e.empty()) return b->fail(IRE_E_INVALID, "%s", e.c_str());
    b->nu.assign(nu, nu + K);
    b->kabs.assign(kappa_abs, kappa_abs + K);
    b->albedo.assign(albedo, albedo + K);
    b->g.assign(g, g + K);
    b->J.clear();
    b->S.clear();
    b->dirty = true;
    return IRE_OK;
}

int ire_batch_set_temperature_grid(ire_batch *b, double t_min, double t_max, int32_t n_t) {
    if (!b) return IRE_E_INVALID;
    if (!(t_min > 0.0) || !(t_max > t_min) || !std::isfinite(t_max) || n_t < 2 || n_t > ire::kMaxGuideNt)
        return b->fail(IRE_E_INVALID, "need 0 < t_min < t_max and 2 <= n_t <= %d", ire::kMaxGuideNt);
    b->t_min = t_min;
    b->t_max = t_max;
    b->n_t = n_t;
    b->dirty = true;
    return IRE_OK;
}

int ire_batch_set_sources(ire_batch *b, const double *J_shape, const double *S_shape) {
    if (!b) return IRE_E_INVALID;
    if (b->nu.empty()) return b->fail(IRE_E_STATE, "set the dust (frequency grid) before the sources");
    const int K = (int)b->nu.size();
    for (const double *a : {J_shape, S_shape}) {
        if (!a) continue;
        if (!ire::host::finite_all(a, K)) return b->fail(IRE_E_INVALID, "non-finite source spectrum");
        double tot = 0.0;
        for (int k = 0; k < K; ++k) {
            if (!(a[k] >= 0.0)) return b->fail(IRE_E_INVALID, "negative source spectrum");
            tot += a[k];
        }
        if (!(tot > 0.0)) return b->fail(IRE_E_INVALID, "source spectrum is all zero");
    }
    b->J = J_shape ? std::vector<double>(J_shape, J_shape + K) : std::vector<double>();
    b->S = S_shape ? std::vector<double>(S_shape, S_shape + K) : std::vector<double>();
    b->dirty = true;
    return IRE_OK;
}

int ire_batch_set_models(ire_batch *b, int32_t M, const ire_model_desc *models, const double *r_edges_flat,
                         const double *rho_flat) {
    if (!b) return IRE_E_INVALID;
    if (M < 1 || !models || !r_edges_flat || !rho_flat) return b->fail(IRE_E_INVALID, "need M >= 1 and all arrays");
    size_t r_off = 0, d_off = 0;
    for (int m = 0; m < M; ++m) {
        const ire_model_desc &d = models[m];
        const std::string e = ire::host::check_shells(d.n_shells, r_edges_flat + r_off, rho_flat + d_off);
        if (!e.empty()) return b->fail(IRE_E_INVALID, "model %d: %s", m, e.c_str());
        if (d.source != IRE_SRC_EXTERNAL && d.source != IRE_SRC_POINT)
            return b->fail(IRE_E_INVALID, "model %d: unknown source type", m);
        if (!(d.scale > 0.0) || !std::isfinite(d.scale)) return b->fail(IRE_E_INVALID, "model %d: scale must be > 0", m);
        if (d.n_packages < 1) return b->fail(IRE_E_INVALID, "model %d: needs at least one package", m);
        if (d.source == IRE_SRC_EXTERNAL && b->J.empty())
            return b->fail(IRE_E_STATE, "model %d is externally heated but no J shape is set", m);
        if (d.source == IRE_SRC_POINT && b->S.empty())
            return b->fail(IRE_E_STATE, "model %d has a point source but no spectrum shape is set", m);
        r_off += (size_t)d.n_shells + 1;
        d_off += (size_t)d.n_shells;
    }
    if (d_off > (size_t)0x7fffffff) return b->fail(IRE_E_INVALID, "too many shells in one batch");
    b->models.assign(models, models + M);
    b->r_edges.assign(r_edges_flat, r_edges_flat + r_off);
    b->rho.assign(rho_flat, rho_flat + d_off);
    b->dirty = true;
    return IRE_OK;
}

int ire_batch_set_options(ire_batch *b, const ire_batch_options *o) {
    if (!b) return IRE_E_INVALID;
    if (!o) return b->fail(IRE_E_INVALID, "null options");
    if (!(o->k_bg > 0.0 && o->k_bg <= 1.0)) return b->fail(IRE_E_INVALID, "k_bg must be in (0,1]");
    if (!(o->w_floor >= 0.0 && o->w_floor < 1.0)) return b->fail(IRE_E_INVALID, "w_floor must be in [0,1)");
    if (o->ffi < 0 || o->ffi > 2) return b->fail(IRE_E_INVALID, "ffi must be 0, 1 or 2");
    const std::string we = ire::host::check_weights(o->use_g_E, o->g_E, o->use_g_S, o->g_S, o->k_A, o->k_S);
    if (!we.empty()) return b->fail(IRE_E_INVALID, "%s", we.c_str());
    if (o->reemit_uniform != 0 && o->reemit_uniform != 1) return b->fail(IRE_E_INVALID, "reemit_uniform must be 0 or 1");
    if (o->aggregate != 0 && o->aggregate != 1) return b->fail(IRE_E_INVALID, "aggregate must be 0 or 1");
    if (o->batch < 0 || o->batch > 64) return b->fail(IRE_E_INVALID, "batch must be in [0, 64]");
    if (o->use_graph != 0 && o->use_graph != 1) return b->fail(IRE_E_INVALID, "use_graph must be 0 or 1");
    if (o->k_A_rho != 0 && o->k_A_rho != 1) return b->fail(IRE_E_INVALID, "k_A_rho must be 0 or 1");
    if (o->k_A_rho && (o->k_A != 1.0 || !(o->k_A_lowest > 0.0) || !(o->k_A_highest > 0.0) ||
                       !std::isfinite(o->k_A_lowest) || !std::isfinite(o->k_A_highest)))
        return b->fail(IRE_E_INVALID, "k_A_rho needs k_A = 1 and finite k_A_lowest, k_A_highest > 0");
    // item sizes and the k_A(rho) records are built with the tables
    const bool tables_change = o->item_packages != b->opt.item_packages || o->k_A_rho != b->opt.k_A_rho ||
                               (o->k_A_rho && (o->k_A_lowest != b->opt.k_A_lowest ||
                                               o->k_A_highest != b->opt.k_A_highest));
    b->opt = *o;
    if (tables_change) b->dirty = true;
    b->drop_graph();
    return IRE_OK;
}

int ire_batch_run(ire_batch *b, void *hip_stream) {
    if (!b) return IRE_E_INVALID;
    return run_on(b, reinterpret_cast<hipStream_t>(hip_stream));
}

int ire_batch_get(ire_batch *b, double *A_flat, double *T_flat, ire_batch_stats *st) {
    if (!b) return IRE_E_INVALID;
    if (!b->ran) return b->fail(IRE_E_STATE, "no run to report");
    hipError_t e;
    if ((e = hipSetDevice(b->device)) != hipSuccess) return b->hip_fail(e, "hipSetDevice");
    if ((e = hipStreamSynchronize(b->last_stream)) != hipSuccess) return b->hip_fail(e, "synchronize");
    if (A_flat && (e = hipMemcpy(A_flat, b->A_out.p, b->n_shells * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess)
        return b->hip_fail(e, "copy A");
    if (T_flat && (e = hipMemcpy(T_flat, b->T_out.p, b->n_shells * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess)
        return b->hip_fail(e, "copy T");
    ire::DevStats hs;
    if ((e = hipMemcpy(&hs, b->stats.p, sizeof(hs), hipMemcpyDeviceToHost)) != hipSuccess) return b->hip_fail(e, "stats");
    if (st) {
        memset(st, 0, sizeof(*st));
        st->L_total = b->L_total;
        st->escaped = hs.tally[ire::T_ESC_EXT] + hs.tally[ire::T_ESC_PS];
        st->ffi_escaped = hs.tally[ire::T_FFI];
        st->terminated = hs.tally[ire::T_TERM];
        st->n_launch = hs.cnt[ire::C_LAUNCH];
        st->n_cross = hs.cnt[ire::C_CROSS];
        st->n_scat = hs.cnt[ire::C_SCAT];
        st->n_abs = hs.cnt[ire::C_ABS];
        st->n_escape = hs.cnt[ire::C_ESCAPE];
        st->n_limit = hs.cnt[ire::C_LIMIT];
        st->n_floor = hs.cnt[ire::C_FLOOR];
        st->n_below = hs.cnt[ire::C_BELOW];
        st->n_above = hs.cnt[ire::C_ABOVE];
        st->n_pass = hs.cnt[ire::C_PASS];
        st->n_step_slots = hs.cnt[ire::C_SLOTS];
        st->n_models = b->models.size();
        st->n_items = b->items.size();
        st->n_shells = b->n_shells;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, b->ev0, b->ev1) == hipSuccess) st->ms_run = ms;
    }
    if (hs.cnt[ire::C_LIMIT] > 0) return b->fail(IRE_E_LIMIT, "%llu packages reached max_events", hs.cnt[ire::C_LIMIT]);
    return IRE_OK;
}

int ire_batch_autotune(ire_batch *b, double fraction, const char *cache_path, ire_batch_options *chosen) {
    if (!b) return IRE_E_INVALID;
    if (!(fraction > 0.0 && fraction <= 1.0)) return b->fail(IRE_E_INVALID, "fraction must be in (0, 1]");
    if (b->models.empty() || b->nu.empty()) return b->fail(IRE_E_STATE, "set dust, sources and models first");
    const std::string key = class_key(b);
    ire_batch_options best = b->opt;
    int cb = 0;
    unsigned long long ci = 0;
    if (cache_path && cache_lookup(cache_path, key, cb, ci)) {
        best.batch = cb;
        best.item_packages = ci;
        int rc = ire_batch_set_options(b, &best);
        if (rc) return rc;
        if (chosen) *chosen = b->opt;
        return IRE_OK;
    }
    // sample: every model, budgets scaled by `fraction` (at least one item per model)
    const std::vector<ire_model_desc> full = b->models;
    std::vector<ire_model_desc> sample = full;
    for (auto &m : sample)
        m.n_packages = std::max<uint64_t>(1, (uint64_t)std::llround((double)m.n_packages * fraction));
    const ire_batch_options saved = b->opt;
    b->models = sample;
    b->dirty = true;
    // candidate work-item sizes are scaled with the budgets, so that the
    // sample splits every model into as many items as the full run would
    const int batches[] = {24, 32, 48};
    const unsigned long long items[] = {65536ull, 262144ull, 524288ull, 1048576ull};
    float best_ms = 1e30f;
    int rc = IRE_OK;
    for (int bt : batches) {
        for (unsigned long long it : items) {
            ire_batch_options o = saved;
            o.batch = bt;
            o.item_packages = std::max<unsigned long long>(64ull, (unsigned long long)std::llround((double)it * fraction));
            o.use_graph = 0;
            if ((rc = ire_batch_set_options(b, &o))) break;
            if ((rc = run_on(b, nullptr))) break;
            ire_batch_stats st;
            rc = ire_batch_get(b, nullptr, nullptr, &st);
            if (rc && rc != IRE_E_LIMIT) break;
            rc = IRE_OK;
            if (st.ms_run < best_ms) {
                best_ms = st.ms_run;
                best = o;
                best.item_packages = it;
            }
        }
        if (rc) break;
    }
    b->models = full;
    b->dirty = true;
    best.use_graph = saved.use_graph;
    if (rc) {
        b->opt = saved;
        return rc;
    }
    rc = ire_batch_set_options(b, &best);
    if (rc) return rc;
    b->dirty = true;
    if (cache_path) {
        std::ofstream f(cache_path, std::ios::app);
        if (f)
            f << "{\"key\": \"" << key << "\", \"batch\": " << best.batch << ", \"item_packages\": " << best.item_packages
              << ", \"sample_ms\": " << best_ms << ", \"fraction\": " << fraction << "}\n";
    }
    if (chosen) *chosen = b->opt;
    return IRE_OK;
}

}  // extern "C"
