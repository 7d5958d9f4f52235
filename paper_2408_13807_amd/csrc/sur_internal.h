// Internal layouts of the MLP surrogate (shared by sur_kernels.hip and sur_api.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sur {

constexpr int kWidth = 256;    // hidden width
constexpr int kFeatures = 6;   // cloud/shell parameters per row
constexpr int kLogRadius = kFeatures;  // one input derived from the six: log10(max(r/R_out, 1e-4)) + 1.5
constexpr int kNetInputs = kFeatures + 1;
constexpr int kIn = 32;        // inputs padded to the MFMA k granularity

// Parameter layout per ensemble member (FP32 master, flat):
//   [0, kWidth*kIn)                 W_0 (row-major [out][in], inputs beyond kNetInputs stay zero)
//   (depth-1) blocks of kWidth^2    W_1 .. W_{depth-1}
//   off_b:    depth*kWidth          hidden biases
//   off_wout: kWidth                output weights
//   off_bout: 1                     output bias
// The BF16 weights share the weight part of that layout: Wf holds each block in the order
// in which the forward passes read their MFMA fragments (frag_index), WT each block transposed.
struct NetView {
    int members, depth;
    __bf16 *WT, *Wf;
    float *b, *wout, *bout;
    size_t w_stride, b_stride, p_stride;
    size_t off_b, off_wout, off_bout;
    float x_mean[kFeatures], x_inv_std[kFeatures];
    float y_mean, y_std, y_inv_std;
};

// Whole-model prediction inputs (device pointers): model m owns output rows
// [row_off[m], row_off[m+1]); its cloud parameters (feature columns 0..4) are
// model_x[m*5 .. m*5+4]; the shells' relative mid-radii (column 5) are
// radius[radius_off[m] + j], j < row_off[m+1] - row_off[m].
struct ModelRows {
    int64_t n_models, n_radius;
    const float *model_x;
    const int64_t *row_off, *radius_off;
    const float *radius;
};

struct TrainView {
    int64_t batch;              // rows per member and step
    int64_t ld;                 // row stride of the feature-major arrays: batch rounded up to 16
    float *xb, *yb;             // [M][batch][kFeatures], [M][batch] gathered mini-batch
    // feature-major (rows contiguous per feature) so that the weight gradient
    // reads its MFMA fragments straight from them; rows [batch, ld) hold zero deltas
    __bf16 *x16;                // [M][kIn][ld] normalised inputs
    __bf16 *h;                  // [M][depth][kWidth][ld] activations
    float *ds;                  // [M][depth][batch][kWidth] SiLU'(z) (row-major)
    __bf16 *delta;              // [M][depth][kWidth][ld] d loss / d z
    float *out, *g;             // [M][batch] outputs and d loss / d output
    float *loss;                // [M] mean squared error of the step (normalised target)
    float *grad, *master, *adam_m, *adam_v;  // [M][p_stride]
};

// Position in a Wf block of the weight of output o and input i (K inputs): the block
// holds, for each 32-output group and each k step of 16 inputs, one MFMA A fragment
// of 64 lanes x 8 inputs (lane = 32 * ((i >> 3) & 1) + o % 32, input i % 8 in the
// lane's 8), so that a wave reads a fragment as 1 KB of contiguous memory.
__host__ __device__ inline size_t frag_index(size_t o, size_t i, size_t K) {
    return ((((o >> 5) * (K >> 4) + (i >> 4)) * 64 + ((i >> 3) & 1) * 32 + (o & 31)) << 3) + (i & 7);
}

// Write one master parameter (member m, flat index q) into the BF16/FP32 copies the kernels read.
__device__ __forceinline__ void scatter_param(const NetView &v, int m, size_t q, float p) {
    if (q < v.off_b) {
        size_t blk, K;
        if (q < (size_t)kWidth * kIn) {
            blk = 0;
            K = kIn;
        } else {
            blk = (size_t)kWidth * kIn + ((q - (size_t)kWidth * kIn) / ((size_t)kWidth * kWidth)) * kWidth * kWidth;
            K = kWidth;
        }
        const size_t e = q - blk;
        const size_t o = e / K, i = e % K;
        v.WT[(size_t)m * v.w_stride + blk + i * kWidth + o] = (__bf16)p;
        v.Wf[(size_t)m * v.w_stride + blk + frag_index(o, i, K)] = (__bf16)p;
    } else if (q < v.off_wout) {
        v.b[(size_t)m * v.b_stride + (q - v.off_b)] = p;
    } else if (q < v.off_bout) {
        v.wout[(size_t)m * kWidth + (q - v.off_wout)] = p;
    } else {
        v.bout[m] = p;
    }
}

size_t predict_lds();
hipError_t configure();
hipError_t launch_predict(const NetView &v, const float *X, int64_t n, float *mean_logT, float *spread, hipStream_t s);
hipError_t launch_predict_models(const NetView &v, const ModelRows &q, int64_t n_rows, float *mean_logT,
                                 float *spread, float *model_spread, hipStream_t s);
// One training step on the batch in t (gathered from X, y when X is not null);
// with `update`, an Adam step and the step counter increment follow.
hipError_t launch_train_step(const NetView &v, const TrainView &t, const float *X, const float *y, int64_t n_data,
                             unsigned long long seed, unsigned long long *step, float lr_max, float lr_min,
                             unsigned long long total_steps, float beta1, float beta2, float eps, int update,
                             hipStream_t s);
hipError_t launch_sync_params(const NetView &v, const float *master, hipStream_t s);
hipError_t launch_zero(float *a, size_t n, hipStream_t s);

}  // namespace sur
