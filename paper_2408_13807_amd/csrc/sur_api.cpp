// C-ABI of the MLP surrogate (include/ire.h, sur_*): parameters, training loop
// (one step captured as a HIP graph and replayed), ensemble prediction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <string>
#include <vector>

#include "ire.h"
#include "ire_host.h"
#include "sur_internal.h"

using ire::host::DevBuf;

struct sur_net {
    int device = 0;
    int members = 0, depth = 0;
    std::string err;
    size_t p_stride = 0, w_stride = 0, b_stride = 0, off_b = 0, off_wout = 0, off_bout = 0;
    float x_mean[sur::kFeatures] = {0}, x_std[sur::kFeatures] = {1, 1, 1, 1, 1, 1};
    float y_mean = 0.0f, y_std = 1.0f;
    bool norm_set = false;
    DevBuf<__bf16> WT, Wf;
    DevBuf<float> b, wout, bout, master, grad, adam_m, adam_v;
    // training workspace
    int64_t cap_batch = 0;
    DevBuf<float> xb, yb, ds, out, g, loss, data_x, data_y;
    DevBuf<__bf16> x16, h, delta;
    DevBuf<unsigned long long> step;
    hipStream_t cap = nullptr;

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

    sur::NetView view() const {
        sur::NetView v{};
        v.members = members;
        v.depth = depth;
        v.WT = WT.p;
        v.Wf = Wf.p;
        v.b = b.p;
        v.wout = wout.p;
        v.bout = bout.p;
        v.w_stride = w_stride;
        v.b_stride = b_stride;
        v.p_stride = p_stride;
        v.off_b = off_b;
        v.off_wout = off_wout;
        v.off_bout = off_bout;
        for (int c = 0; c < sur::kFeatures; ++c) {
            v.x_mean[c] = x_mean[c];
            v.x_inv_std[c] = 1.0f / x_std[c];
        }
        v.y_mean = y_mean;
        v.y_std = y_std;
        v.y_inv_std = 1.0f / y_std;
        return v;
    }
    sur::TrainView tview(int64_t batch) const {
        sur::TrainView t{};
        t.batch = batch;
        t.ld = (batch + 15) / 16 * 16;
        t.xb = xb.p;
        t.yb = yb.p;
        t.x16 = x16.p;
        t.h = h.p;
        t.ds = ds.p;
        t.delta = delta.p;
        t.out = out.p;
        t.g = g.p;
        t.loss = loss.p;
        t.grad = grad.p;
        t.master = master.p;
        t.adam_m = adam_m.p;
        t.adam_v = adam_v.p;
        return t;
    }
};

namespace {

uint64_t splitmix(uint64_t &x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int ensure_workspace(sur_net *s, int64_t batch) {
    if (batch <= s->cap_batch) return IRE_OK;
    // batch is a multiple of 128 here, so it also covers the feature-major arrays' padded stride
    const size_t M = s->members, L = s->depth, B = (size_t)batch, W = sur::kWidth;
    hipError_t e;
    if ((e = s->xb.ensure(M * B * sur::kFeatures)) != hipSuccess || (e = s->yb.ensure(M * B)) != hipSuccess ||
        (e = s->x16.ensure(M * B * sur::kIn)) != hipSuccess || (e = s->h.ensure(M * L * B * W)) != hipSuccess ||
        (e = s->ds.ensure(M * L * B * W)) != hipSuccess || (e = s->delta.ensure(M * L * B * W)) != hipSuccess ||
        (e = s->out.ensure(M * B)) != hipSuccess || (e = s->g.ensure(M * B)) != hipSuccess ||
        (e = s->loss.ensure(M)) != hipSuccess)
        return s->fail(IRE_E_NOMEM, "training workspace: %s", hipGetErrorString(e));
    s->cap_batch = batch;
    return IRE_OK;
}

int upload_params(sur_net *s, const std::vector<float> &p) {
    hipError_t e;
    if ((e = hipMemcpy(s->master.p, p.data(), p.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
        return s->hip_fail(e, "parameter upload");
    if ((e = sur::launch_sync_params(s->view(), s->master.p, nullptr)) != hipSuccess) return s->hip_fail(e, "sync");
    if ((e = hipDeviceSynchronize()) != hipSuccess) return s->hip_fail(e, "sync");
    return IRE_OK;
}

bool finite_f(const float *a, size_t n) {
    for (size_t j = 0; j < n; ++j)
        if (!std::isfinite(a[j])) return false;
    return true;
}

}  // namespace

extern "C" {

int sur_default_train_opts(sur_train_opts *o) {
    if (!o) return IRE_E_INVALID;
    o->batch = 4096;
    o->steps = 2000;
    o->lr = 1e-3;
    o->lr_min = 1e-5;
    o->beta1 = 0.9;
    o->beta2 = 0.999;
    o->eps = 1e-8;
    o->seed = 1;
    o->use_graph = 1;
    return IRE_OK;
}

int sur_create(int hip_device, int32_t members, int32_t width, int32_t depth, uint64_t seed, sur_net **out) {
    if (!out) return IRE_E_INVALID;
    *out = nullptr;
    if (members < 1 || members > 64 || width != sur::kWidth || depth < 1 || depth > 16) return IRE_E_INVALID;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || hip_device < 0 || hip_device >= count) return IRE_E_DEVICE;
    sur_net *s = new (std::nothrow) sur_net();
    if (!s) return IRE_E_NOMEM;
    s->device = hip_device;
    s->members = members;
    s->depth = depth;
    const size_t W = sur::kWidth;
    s->w_stride = W * sur::kIn + (size_t)(depth - 1) * W * W;
    s->b_stride = (size_t)depth * W;
    s->off_b = s->w_stride;
    s->off_wout = s->off_b + s->b_stride;
    s->off_bout = s->off_wout + W;
    s->p_stride = s->off_bout + 1;
    const size_t M = members;
    if (hipSetDevice(hip_device) != hipSuccess || hipStreamCreate(&s->cap) != hipSuccess ||
        s->WT.ensure(M * s->w_stride) != hipSuccess || s->Wf.ensure(M * s->w_stride) != hipSuccess ||
        s->b.ensure(M * s->b_stride) != hipSuccess || s->wout.ensure(M * W) != hipSuccess ||
        s->bout.ensure(M) != hipSuccess || s->master.ensure(M * s->p_stride) != hipSuccess ||
        s->grad.ensure(M * s->p_stride) != hipSuccess || s->adam_m.ensure(M * s->p_stride) != hipSuccess ||
        s->adam_v.ensure(M * s->p_stride) != hipSuccess || s->step.ensure(1) != hipSuccess ||
        sur::configure() != hipSuccess) {
        sur_destroy(s);
        return IRE_E_DEVICE;
    }
    // He-uniform weights (fan-in: the 6 real inputs and the derived one for the first layer), zero biases
    std::vector<float> p(M * s->p_stride, 0.0f);
    for (size_t m = 0; m < M; ++m) {
        uint64_t st = seed * 0x100000001B3ull + m + 1;
        auto uni = [&]() { return (float)((splitmix(st) >> 11) * 0x1p-53); };
        float *q = p.data() + m * s->p_stride;
        const float a0 = std::sqrt(6.0f / sur::kNetInputs);
        for (size_t o = 0; o < W; ++o)
            for (int i = 0; i < sur::kNetInputs; ++i) q[o * sur::kIn + i] = a0 * (2.0f * uni() - 1.0f);
        const float a = std::sqrt(6.0f / (float)W);
        for (size_t j = W * sur::kIn; j < s->w_stride; ++j) q[j] = a * (2.0f * uni() - 1.0f);
        const float ao = std::sqrt(3.0f / (float)W);
        for (size_t j = 0; j < W; ++j) q[s->off_wout + j] = ao * (2.0f * uni() - 1.0f);
    }
    hipError_t e;
    if (upload_params(s, p) || (e = sur::launch_zero(s->grad.p, M * s->p_stride, nullptr)) != hipSuccess ||
        (e = sur::launch_zero(s->adam_m.p, M * s->p_stride, nullptr)) != hipSuccess ||
        (e = sur::launch_zero(s->adam_v.p, M * s->p_stride, nullptr)) != hipSuccess ||
        hipMemset(s->step.p, 0, sizeof(unsigned long long)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        sur_destroy(s);
        return IRE_E_DEVICE;
    }
    *out = s;
    return IRE_OK;
}

void sur_destroy(sur_net *s) {
    if (!s) return;
    (void)hipSetDevice(s->device);
    (void)hipDeviceSynchronize();
    for (auto *bf : {&s->WT, &s->Wf, &s->x16, &s->h, &s->delta}) bf->release();
    for (auto *bf : {&s->b, &s->wout, &s->bout, &s->master, &s->grad, &s->adam_m, &s->adam_v, &s->xb, &s->yb, &s->ds,
                     &s->out, &s->g, &s->loss, &s->data_x, &s->data_y})
        bf->release();
    s->step.release();
    if (s->cap) (void)hipStreamDestroy(s->cap);
    delete s;
}

const char *sur_last_error(const sur_net *s) { return s ? s->err.c_str() : "null handle"; }

int sur_set_normalization(sur_net *s, const float *x_mean, const float *x_std, float y_mean, float y_std) {
    if (!s) return IRE_E_INVALID;
    if (!x_mean || !x_std || !finite_f(x_mean, sur::kFeatures) || !finite_f(x_std, sur::kFeatures) ||
        !std::isfinite(y_mean) || !(y_std > 0.0f))
        return s->fail(IRE_E_INVALID, "need finite means and positive standard deviations");
    for (int c = 0; c < sur::kFeatures; ++c) {
        if (!(x_std[c] > 0.0f)) return s->fail(IRE_E_INVALID, "x_std[%d] must be > 0", c);
        s->x_mean[c] = x_mean[c];
        s->x_std[c] = x_std[c];
    }
    s->y_mean = y_mean;
    s->y_std = y_std;
    s->norm_set = true;
    return IRE_OK;
}

int64_t sur_param_count(const sur_net *s) { return s ? (int64_t)s->p_stride : 0; }

int sur_get_params(sur_net *s, float *params) {
    if (!s || !params) return IRE_E_INVALID;
    hipError_t e;
    if ((e = hipSetDevice(s->device)) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess ||
        (e = hipMemcpy(params, s->master.p, (size_t)s->members * s->p_stride * sizeof(float), hipMemcpyDeviceToHost)) !=
            hipSuccess)
        return s->hip_fail(e, "parameter copy");
    return IRE_OK;
}

int sur_set_params(sur_net *s, const float *params) {
    if (!s || !params) return IRE_E_INVALID;
    const size_t n = (size_t)s->members * s->p_stride;
    if (!finite_f(params, n)) return s->fail(IRE_E_INVALID, "non-finite parameters");
    if (hipSetDevice(s->device) != hipSuccess) return s->fail(IRE_E_DEVICE, "hipSetDevice");
    std::vector<float> p(params, params + n);
    // the padding inputs carry no weight
    for (int m = 0; m < s->members; ++m)
        for (int o = 0; o < sur::kWidth; ++o)
            for (int i = sur::kNetInputs; i < sur::kIn; ++i) p[(size_t)m * s->p_stride + (size_t)o * sur::kIn + i] = 0.0f;
    return upload_params(s, p);
}

int sur_train(sur_net *s, const float *X, const float *y, int64_t n, const sur_train_opts *o, void *hip_stream,
              float *final_loss) {
    if (!s) return IRE_E_INVALID;
    sur_train_opts opt;
    sur_default_train_opts(&opt);
    if (o) opt = *o;
    if (!X || !y || n < 1) return s->fail(IRE_E_INVALID, "need rows");
    if (opt.batch < 128 || opt.batch % 128 || opt.batch > (1 << 20)) return s->fail(IRE_E_INVALID, "batch must be a multiple of 128 in [128, 2^20]");
    if (opt.steps < 1 || !(opt.lr > 0.0) || !(opt.lr_min >= 0.0) || !(opt.beta1 >= 0.0 && opt.beta1 < 1.0) ||
        !(opt.beta2 >= 0.0 && opt.beta2 < 1.0) || !(opt.eps > 0.0))
        return s->fail(IRE_E_INVALID, "invalid optimizer options");
    if (!finite_f(X, (size_t)n * sur::kFeatures) || !finite_f(y, (size_t)n)) return s->fail(IRE_E_INVALID, "non-finite data");
    hipError_t e;
    if ((e = hipSetDevice(s->device)) != hipSuccess) return s->hip_fail(e, "hipSetDevice");
    if (!s->norm_set) {
        // standardise with the data's own moments
        double mx[sur::kFeatures] = {0}, sx[sur::kFeatures] = {0}, my = 0.0, sy = 0.0;
        for (int64_t r = 0; r < n; ++r) {
            for (int c = 0; c < sur::kFeatures; ++c) mx[c] += X[r * sur::kFeatures + c];
            my += y[r];
        }
        for (int c = 0; c < sur::kFeatures; ++c) mx[c] /= (double)n;
        my /= (double)n;
        for (int64_t r = 0; r < n; ++r) {
            for (int c = 0; c < sur::kFeatures; ++c) {
                const double d = X[r * sur::kFeatures + c] - mx[c];
                sx[c] += d * d;
            }
            sy += (y[r] - my) * (y[r] - my);
        }
        for (int c = 0; c < sur::kFeatures; ++c) {
            s->x_mean[c] = (float)mx[c];
            const double sd = std::sqrt(sx[c] / (double)n);
            s->x_std[c] = sd > 1e-12 ? (float)sd : 1.0f;
        }
        s->y_mean = (float)my;
        const double sdy = std::sqrt(sy / (double)n);
        s->y_std = sdy > 1e-12 ? (float)sdy : 1.0f;
        s->norm_set = true;
    }
    int rc = ensure_workspace(s, opt.batch);
    if (rc) return rc;
    if ((e = s->data_x.ensure((size_t)n * sur::kFeatures)) != hipSuccess || (e = s->data_y.ensure((size_t)n)) != hipSuccess)
        return s->fail(IRE_E_NOMEM, "training data: %s", hipGetErrorString(e));
    if ((e = hipMemcpy(s->data_x.p, X, (size_t)n * sur::kFeatures * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(s->data_y.p, y, (size_t)n * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemset(s->step.p, 0, sizeof(unsigned long long))) != hipSuccess ||
        (e = hipDeviceSynchronize()) != hipSuccess)
        return s->hip_fail(e, "training data upload");
    const sur::NetView v = s->view();
    const sur::TrainView t = s->tview(opt.batch);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    auto step = [&](hipStream_t q) {
        return sur::launch_train_step(v, t, s->data_x.p, s->data_y.p, n, opt.seed, s->step.p, (float)opt.lr,
                                      (float)opt.lr_min, (unsigned long long)opt.steps, (float)opt.beta1,
                                      (float)opt.beta2, (float)opt.eps, 1, q);
    };
    if (opt.use_graph) {
        hipGraph_t g = nullptr;
        hipGraphExec_t x = nullptr;
        if ((e = hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return s->hip_fail(e, "begin capture");
        hipError_t e1 = step(s->cap);
        hipError_t e2 = hipStreamEndCapture(s->cap, &g);
        if (e1 != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return s->hip_fail(e1 != hipSuccess ? e1 : e2, "capture");
        }
        if ((e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0)) != hipSuccess) {
            (void)hipGraphDestroy(g);
            return s->hip_fail(e, "graph instantiate");
        }
        for (int64_t k = 0; k < opt.steps && e == hipSuccess; ++k) e = hipGraphLaunch(x, st);
        hipError_t e3 = hipStreamSynchronize(st);
        (void)hipGraphExecDestroy(x);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess || e3 != hipSuccess) return s->hip_fail(e != hipSuccess ? e : e3, "training");
    } else {
        for (int64_t k = 0; k < opt.steps; ++k)
            if ((e = step(st)) != hipSuccess) return s->hip_fail(e, "training step");
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return s->hip_fail(e, "training");
    }
    if (final_loss && (e = hipMemcpy(final_loss, s->loss.p, (size_t)s->members * sizeof(float), hipMemcpyDeviceToHost)) != hipSuccess)
        return s->hip_fail(e, "loss copy");
    return IRE_OK;
}

int sur_gradients(sur_net *s, const float *X, const float *y, int64_t n, float *grads, float *loss) {
    if (!s) return IRE_E_INVALID;
    if (!X || !y || n < 1 || n > 65536) return s->fail(IRE_E_INVALID, "need 1 <= n <= 65536 rows");
    hipError_t e;
    if ((e = hipSetDevice(s->device)) != hipSuccess) return s->hip_fail(e, "hipSetDevice");
    const int64_t cap = (n + 127) / 128 * 128;
    int rc = ensure_workspace(s, cap);
    if (rc) return rc;
    // the same rows for every member
    std::vector<float> xb((size_t)s->members * n * sur::kFeatures), yb((size_t)s->members * n);
    for (int m = 0; m < s->members; ++m) {
        std::memcpy(xb.data() + (size_t)m * n * sur::kFeatures, X, (size_t)n * sur::kFeatures * sizeof(float));
        std::memcpy(yb.data() + (size_t)m * n, y, (size_t)n * sizeof(float));
    }
    if ((e = hipMemcpy(s->xb.p, xb.data(), xb.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(s->yb.p, yb.data(), yb.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = sur::launch_zero(s->grad.p, (size_t)s->members * s->p_stride, nullptr)) != hipSuccess)
        return s->hip_fail(e, "upload");
    sur::TrainView t = s->tview(n);
    if ((e = sur::launch_train_step(s->view(), t, nullptr, nullptr, n, 0, s->step.p, 0.0f, 0.0f, 1, 0.9f, 0.999f,
                                    1e-8f, 0, nullptr)) != hipSuccess ||
        (e = hipDeviceSynchronize()) != hipSuccess)
        return s->hip_fail(e, "gradient pass");
    if (grads && (e = hipMemcpy(grads, s->grad.p, (size_t)s->members * s->p_stride * sizeof(float), hipMemcpyDeviceToHost)) != hipSuccess)
        return s->hip_fail(e, "gradient copy");
    if (loss && (e = hipMemcpy(loss, s->loss.p, (size_t)s->members * sizeof(float), hipMemcpyDeviceToHost)) != hipSuccess)
        return s->hip_fail(e, "loss copy");
    if ((e = sur::launch_zero(s->grad.p, (size_t)s->members * s->p_stride, nullptr)) != hipSuccess)
        return s->hip_fail(e, "zero");
    return IRE_OK;
}

int sur_predict_dev(sur_net *s, const float *X_dev, int64_t n, float *mean_dev, float *spread_dev, void *hip_stream) {
    if (!s) return IRE_E_INVALID;
    if (!X_dev || !mean_dev || !spread_dev || n < 0) return s->fail(IRE_E_INVALID, "null pointer or negative n");
    if (n == 0) return IRE_OK;
    hipError_t e;
    if ((e = hipSetDevice(s->device)) != hipSuccess) return s->hip_fail(e, "hipSetDevice");
    if ((e = sur::launch_predict(s->view(), X_dev, n, mean_dev, spread_dev, reinterpret_cast<hipStream_t>(hip_stream))) != hipSuccess)
        return s->hip_fail(e, "predict");
    return IRE_OK;
}

int sur_predict(sur_net *s, const float *X, int64_t n, float *mean_logT, float *spread) {
    if (!s) return IRE_E_INVALID;
    if (!X || !mean_logT || !spread || n < 0) return s->fail(IRE_E_INVALID, "null pointer or negative n");
    hipError_t e;
    if ((e = hipSetDevice(s->device)) != hipSuccess) return s->hip_fail(e, "hipSetDevice");
    const int64_t chunk = 1 << 22;
    DevBuf<float> dx, dm, ds;
    if ((e = dx.ensure((size_t)std::min(n, chunk) * sur::kFeatures)) != hipSuccess ||
        (e = dm.ensure((size_t)std::min(n, chunk))) != hipSuccess || (e = ds.ensure((size_t)std::min(n, chunk))) != hipSuccess)
        return s->fail(IRE_E_NOMEM, "prediction buffers");
    int rc = IRE_OK;
    for (int64_t r0 = 0; r0 < n && rc == IRE_OK; r0 += chunk) {
        const int64_t c = std::min(chunk, n - r0);
        if ((e = hipMemcpy(dx.p, X + r0 * sur::kFeatures, (size_t)c * sur::kFeatures * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) {
            rc = s->hip_fail(e, "upload");
            break;
        }
        if ((e = sur::launch_predict(s->view(), dx.p, c, dm.p, ds.p, nullptr)) != hipSuccess ||
            (e = hipMemcpy(mean_logT + r0, dm.p, (size_t)c * sizeof(float), hipMemcpyDeviceToHost)) != hipSuccess ||
            (e = hipMemcpy(spread + r0, ds.p, (size_t)c * sizeof(float), hipMemcpyDeviceToHost)) != hipSuccess)
            rc = s->hip_fail(e, "predict");
    }
    dx.release();
    dm.release();
    ds.release();
    return rc;
}

int sur_predict_models_dev(sur_net *s, int64_t n_models, int64_t n_rows, const float *model_x_dev,
                           const int64_t *row_off_dev, const int64_t *radius_off_dev, const float *radius_dev,
                           int64_t n_radius, float *mean_dev, float *spread_dev, float *model_spread_dev,
                           void *hip_stream) {
    if (!s) return IRE_E_INVALID;
    if (n_models < 0 || n_rows < 0 || n_radius < 0) return s->fail(IRE_E_INVALID, "negative size");
    if (n_models == 0) return IRE_OK;
    if (!model_x_dev || !row_off_dev || !radius_off_dev || (!radius_dev && n_radius > 0) ||
        (n_rows > 0 && (!mean_dev || !spread_dev)))
        return s->fail(IRE_E_INVALID, "null pointer");
    hipError_t e;
    if ((e = hipSetDevice(s->device)) != hipSuccess) return s->hip_fail(e, "hipSetDevice");
    const sur::ModelRows q{n_models, n_radius, model_x_dev, row_off_dev, radius_off_dev, radius_dev};
    if ((e = sur::launch_predict_models(s->view(), q, n_rows, mean_dev, spread_dev, model_spread_dev,
                                        reinterpret_cast<hipStream_t>(hip_stream))) != hipSuccess)
        return s->hip_fail(e, "predict models");
    return IRE_OK;
}

int sur_predict_models(sur_net *s, int64_t n_models, const float *model_x, const int64_t *row_off,
                       const int64_t *radius_off, const float *radius, int64_t n_radius, float *mean_logT,
                       float *spread, float *model_spread) {
    if (!s) return IRE_E_INVALID;
    if (n_models < 0 || n_radius < 0) return s->fail(IRE_E_INVALID, "negative size");
    if (n_models == 0) return IRE_OK;
    if (!model_x || !row_off || !radius_off || (!radius && n_radius > 0)) return s->fail(IRE_E_INVALID, "null pointer");
    if (row_off[0] != 0) return s->fail(IRE_E_INVALID, "row_off[0] must be 0");
    for (int64_t m = 0; m < n_models; ++m) {
        const int64_t nm = row_off[m + 1] - row_off[m];
        if (nm < 0) return s->fail(IRE_E_INVALID, "row offsets must not decrease");
        if (nm > 0 && (radius_off[m] < 0 || radius_off[m] + nm > n_radius))
            return s->fail(IRE_E_INVALID, "radius range of a model outside the radius table");
    }
    for (int64_t j = 0; j < n_models * (sur::kFeatures - 1); ++j)
        if (!std::isfinite(model_x[j])) return s->fail(IRE_E_INVALID, "non-finite model parameter");
    for (int64_t j = 0; j < n_radius; ++j)
        if (!std::isfinite(radius[j])) return s->fail(IRE_E_INVALID, "non-finite radius");
    const int64_t n_rows = row_off[n_models];
    if (n_rows > 0 && (!mean_logT || !spread)) return s->fail(IRE_E_INVALID, "null output");
    hipError_t e;
    if ((e = hipSetDevice(s->device)) != hipSuccess) return s->hip_fail(e, "hipSetDevice");
    DevBuf<float> dx, dr, dm, ds, dms;
    DevBuf<int64_t> dro, dra;
    int rc = IRE_OK;
    if ((e = dx.ensure((size_t)n_models * (sur::kFeatures - 1))) != hipSuccess ||
        (e = dr.ensure((size_t)n_radius)) != hipSuccess || (e = dm.ensure((size_t)n_rows)) != hipSuccess ||
        (e = ds.ensure((size_t)n_rows)) != hipSuccess || (e = dms.ensure((size_t)n_models)) != hipSuccess ||
        (e = dro.ensure((size_t)n_models + 1)) != hipSuccess || (e = dra.ensure((size_t)n_models)) != hipSuccess) {
        rc = s->fail(IRE_E_NOMEM, "prediction buffers");
    } else if ((e = hipMemcpy(dx.p, model_x, (size_t)n_models * (sur::kFeatures - 1) * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
               (n_radius > 0 && (e = hipMemcpy(dr.p, radius, (size_t)n_radius * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) ||
               (e = hipMemcpy(dro.p, row_off, ((size_t)n_models + 1) * sizeof(int64_t), hipMemcpyHostToDevice)) != hipSuccess ||
               (e = hipMemcpy(dra.p, radius_off, (size_t)n_models * sizeof(int64_t), hipMemcpyHostToDevice)) != hipSuccess) {
        rc = s->hip_fail(e, "upload");
    } else {
        const sur::ModelRows q{n_models, n_radius, dx.p, dro.p, dra.p, dr.p};
        if ((e = sur::launch_predict_models(s->view(), q, n_rows, dm.p, ds.p, dms.p, nullptr)) != hipSuccess ||
            (e = hipDeviceSynchronize()) != hipSuccess)
            rc = s->hip_fail(e, "predict models");
        else if ((n_rows > 0 && ((e = hipMemcpy(mean_logT, dm.p, (size_t)n_rows * sizeof(float), hipMemcpyDeviceToHost)) != hipSuccess ||
                                 (e = hipMemcpy(spread, ds.p, (size_t)n_rows * sizeof(float), hipMemcpyDeviceToHost)) != hipSuccess)) ||
                 (model_spread && (e = hipMemcpy(model_spread, dms.p, (size_t)n_models * sizeof(float), hipMemcpyDeviceToHost)) != hipSuccess))
            rc = s->hip_fail(e, "download");
    }
    dx.release(); dr.release(); dm.release(); ds.release(); dms.release(); dro.release(); dra.release();
    return rc;
}

int sur_save(sur_net *s, const char *path) {
    if (!s || !path) return IRE_E_INVALID;
    std::vector<float> p((size_t)s->members * s->p_stride);
    int rc = sur_get_params(s, p.data());
    if (rc) return rc;
    std::ofstream f(path, std::ios::binary);
    if (!f) return s->fail(IRE_E_INVALID, "cannot write %s", path);
    const int32_t hdr[4] = {0x53555231, s->members, sur::kWidth, s->depth};  // "SUR1"
    f.write(reinterpret_cast<const char *>(hdr), sizeof(hdr));
    f.write(reinterpret_cast<const char *>(s->x_mean), sizeof(s->x_mean));
    f.write(reinterpret_cast<const char *>(s->x_std), sizeof(s->x_std));
    f.write(reinterpret_cast<const char *>(&s->y_mean), sizeof(float));
    f.write(reinterpret_cast<const char *>(&s->y_std), sizeof(float));
    f.write(reinterpret_cast<const char *>(p.data()), p.size() * sizeof(float));
    return f ? IRE_OK : s->fail(IRE_E_INVALID, "write failed");
}

int sur_load(sur_net *s, const char *path) {
    if (!s || !path) return IRE_E_INVALID;
    std::ifstream f(path, std::ios::binary);
    if (!f) return s->fail(IRE_E_INVALID, "cannot read %s", path);
    int32_t hdr[4];
    f.read(reinterpret_cast<char *>(hdr), sizeof(hdr));
    if (!f || hdr[0] != 0x53555231 || hdr[1] != s->members || hdr[2] != sur::kWidth || hdr[3] != s->depth)
        return s->fail(IRE_E_INVALID, "%s does not hold a network of this shape", path);
    float xm[sur::kFeatures], xs[sur::kFeatures], ym, ys;
    f.read(reinterpret_cast<char *>(xm), sizeof(xm));
    f.read(reinterpret_cast<char *>(xs), sizeof(xs));
    f.read(reinterpret_cast<char *>(&ym), sizeof(float));
    f.read(reinterpret_cast<char *>(&ys), sizeof(float));
    std::vector<float> p((size_t)s->members * s->p_stride);
    f.read(reinterpret_cast<char *>(p.data()), p.size() * sizeof(float));
    if (!f) return s->fail(IRE_E_INVALID, "%s is truncated", path);
    int rc = sur_set_normalization(s, xm, xs, ym, ys);
    if (rc) return rc;
    return sur_set_params(s, p.data());
}

}  // extern "C"
