// MLP surrogate of the IRE temperature profile: BF16 MFMA kernels for gfx950.
//
// The network maps 6 cloud/shell parameters (padded to 32 inputs) through
// `depth` hidden layers of width 256 with SiLU activations to log10 T.
// Weights are BF16 (FP32 master copies for Adam), accumulation is FP32 in the
// matrix cores (v_mfma_f32_32x32x16_bf16).  Every layer is computed as
// D = W . H^T: the weights (row-major [out][in], read from L2) are the MFMA A
// operand and the activations (row-major [row][feature], staged in LDS) the B
// operand, so each lane's accumulators hold 4 consecutive output features of
// one row and the epilogue stores 8 bytes at a time.
//
// MFMA 32x32x16 bf16 lane layout (wave64): A fragment of lane l = A[l&31][8(l>>5) .. +7],
// B fragment = B[8(l>>5) .. +7][l&31] (given as B^T rows), accumulator r of lane l =
// D[8(r>>2) + 4(l>>5) + (r&3)][l&31].
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sur_internal.h"

namespace sur {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kW = kWidth;         // 256
constexpr int kR = 128;            // rows per workgroup tile
constexpr int kLd = kW + 8;        // LDS row stride (bf16) of activation tiles
constexpr int kLdX = kIn + 8;      // LDS row stride of the input tile
constexpr int kThreads = 256;      // 4 waves

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

__device__ __forceinline__ f32x16 mfma(const bf16x8 &a, const bf16x8 &b, const f32x16 &c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// The network sees one input derived from the six (kLogRadius): log10 of the
// relative radius (floored at 1e-4) shifted by 1.5, which spreads the inner
// shells of log-spaced grids that r / R_out alone packs near zero.
__device__ __forceinline__ float log_radius_input(float r) { return log10f(fmaxf(r, 1e-4f)) + 1.5f; }

// Normalised inputs of rows [row0, row0 + kR) into the LDS input tile (zero padded).
__device__ __forceinline__ void load_inputs(const float *X, int64_t n, int64_t row0, const NetView &v, __bf16 *xs) {
    for (int j = threadIdx.x; j < kR * kIn; j += blockDim.x) {
        const int r = j / kIn, c = j % kIn;
        const int64_t row = row0 + r;
        float x = 0.0f;
        if (row < n) {
            if (c < kFeatures) x = (X[row * kFeatures + c] - v.x_mean[c]) * v.x_inv_std[c];
            else if (c == kLogRadius) x = log_radius_input(X[row * kFeatures + kFeatures - 1]);
        }
        xs[r * kLdX + c] = (__bf16)x;
    }
}

// One hidden layer for the kR rows in LDS: hout = SiLU(W hin + b).  Wave w
// computes output features [64w, 64w + 64) for all rows.  With TRAIN the
// activation and SiLU'(z) are also stored to global memory (rows < n).
template <bool TRAIN>
__device__ __forceinline__ void layer_fwd(const __bf16 *W, const float *bias, int K, const __bf16 *hin, int ldin, __bf16 *hout,
                          __bf16 *h_g, float *ds_g, int64_t row0, int64_t n, int64_t ld) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    f32x16 acc[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f32x16{};
    // W is the layer's block of the fragment-ordered weights (frag_index)
    const int nst = K >> 4;
    const __bf16 *wf = W + ((size_t)(wave * 2) * nst * 64 + lane) * 8;
    for (int kk = 0; kk < K; kk += 16) {
        bf16x8 wa[2], hb[4];
#pragma unroll
        for (int a = 0; a < 2; ++a) wa[a] = *reinterpret_cast<const bf16x8 *>(wf + ((size_t)a * nst + (kk >> 4)) * 512);
#pragma unroll
        for (int b = 0; b < 4; ++b) hb[b] = *reinterpret_cast<const bf16x8 *>(hin + (b * 32 + l32) * ldin + kk + 8 * half);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = mfma(wa[a], hb[b], acc[a][b]);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int row = b * 32 + l32;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int o = wave * 64 + a * 32 + 8 * g + 4 * half;
                bf16x4 hv;
                float dv[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float z = acc[a][b][4 * g + q] + bias[o + q];
                    hv[q] = (__bf16)silu(z);
                    dv[q] = dsilu(z);
                }
                *reinterpret_cast<bf16x4 *>(hout + row * kLd + o) = hv;
                if (TRAIN && row0 + row < ld) {
                    // feature-major activations (rows of 32 lanes contiguous per feature)
#pragma unroll
                    for (int q = 0; q < 4; ++q) h_g[(size_t)(o + q) * ld + row0 + row] = hv[q];
                }
                if (TRAIN && row0 + row < n)
                    *reinterpret_cast<float4 *>(ds_g + (row0 + row) * kW + o) = float4{dv[0], dv[1], dv[2], dv[3]};
            }
        }
}

// Output layer: y = w_out . h + b_out for the kR rows (two threads per row).
__device__ __forceinline__ float out_row(const __bf16 *h, const float *wout, float bout) {
    const int r = threadIdx.x >> 1, part = threadIdx.x & 1;
    float s = 0.0f;
    for (int c = part * 128; c < part * 128 + 128; ++c) s += (float)h[r * kLd + c] * wout[c];
    s += __shfl_xor(s, 1, 64);
    return s + bout;
}

// ---------------------------------------------------------------------------
// Inference: every member on every row; mean log10 T and relative spread of T.

// Inference keeps every activation, and the inputs, multiplied by
// kActScale = -log2(e): the pre-activations are then -log2(e) z, the argument
// of the exp2 in SiLU(z) = z / (1 + e^-z), and the scaled SiLU is t / (1 +
// 2^t) for t = -log2(e) z.  The weights are unchanged; the biases are scaled
// as they are loaded and the output layer divides by kActScale.
constexpr float kActScale = -1.44269504088896341f;
constexpr float kInvActScale = -0.693147180559945309f;

__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    const bf16x2 v = __builtin_convertvector(f32x2{a, b}, bf16x2);
    return __builtin_bit_cast(uint32_t, v);
}

// One row of the inference input tile: the network's inputs from the six
// features (normalised; the derived log-radius input), times kActScale, as
// BF16, zero padded to kIn; rows at or beyond n are zero.
__device__ __forceinline__ void stage_row(const float (&f)[kFeatures], bool valid, const NetView &v, __bf16 *xrow) {
    float x[kNetInputs];
#pragma unroll
    for (int c = 0; c < kFeatures; ++c) x[c] = (f[c] - v.x_mean[c]) * v.x_inv_std[c];
    x[kLogRadius] = log_radius_input(f[kFeatures - 1]);
    uint32_t p[kIn / 2];
#pragma unroll
    for (int c = 0; c < kIn / 2; ++c) {
        const float a = 2 * c < kNetInputs && valid ? x[2 * c] * kActScale : 0.0f;
        const float b = 2 * c + 1 < kNetInputs && valid ? x[2 * c + 1] * kActScale : 0.0f;
        p[c] = pack_bf16x2(a, b);
    }
#pragma unroll
    for (int c = 0; c < kIn / 8; ++c)
        *reinterpret_cast<uint4 *>(xrow + 8 * c) = uint4{p[4 * c], p[4 * c + 1], p[4 * c + 2], p[4 * c + 3]};
}

// Row inputs for prediction: a row-major [n][kFeatures] matrix (one thread
// per row, its loads in flight together) ...
struct RowInputs {
    const float *X;
    __device__ __forceinline__ void operator()(int64_t n, int64_t row0, const NetView &v, __bf16 *xs) const {
        if (threadIdx.x < kR) {
            const int64_t row = row0 + threadIdx.x;
            const bool valid = row < n;
            float f[kFeatures];
#pragma unroll
            for (int c = 0; c < kFeatures; ++c) f[c] = valid ? X[row * kFeatures + c] : 0.0f;
            stage_row(f, valid, v, xs + threadIdx.x * kLdX);
        }
    }
};

// ... or whole models: the cloud parameters once per model (feature columns
// 0..4) and the shells' relative mid-radii (column 5) from a radius table in
// which models with the same shell grid may share their values.  The first
// wave finds the model holding row0 by a 64-way search and stages the next 64
// model boundaries in LDS, where each row finds its model.
struct ModelInputs {
    ModelRows q;
    __device__ __forceinline__ void operator()(int64_t n, int64_t row0, const NetView &v, __bf16 *xs) const {
        __shared__ int64_t s_bnd[64];
        __shared__ int64_t s_first;
        const int lane = threadIdx.x & 63;
        if (threadIdx.x < 64) {
            // last m with row_off[m] <= row0 (row_off[0] = 0 <= row0); it lies in [lo, hi]
            int64_t lo = 0, hi = q.n_models - 1;
            while (hi > lo) {
                const int64_t step = (hi - lo + 63) / 64;
                const int64_t c = lo + (lane + 1) * step;
                const bool ok = c <= hi && q.row_off[c] <= row0;
                lo += step * __popcll(__ballot(ok));
                hi = min(hi, lo + step - 1);
            }
            const int64_t b = lo + 1 + lane;
            s_bnd[lane] = b < q.n_models ? q.row_off[b] : INT64_MAX;
            if (lane == 0) s_first = lo;
        }
        __syncthreads();
        if (threadIdx.x < kR) {
            const int64_t row = row0 + threadIdx.x;
            const bool valid = row < n;
            int64_t m = s_first;
            if (valid) {
                // boundaries s_bnd[i] = row_off[s_first + 1 + i] <= row, counted by bisection
                int c = 0;
                if (s_bnd[63] <= row) {
                    c = 64;
                } else {
#pragma unroll
                    for (int step = 32; step > 0; step >>= 1)
                        if (s_bnd[c + step - 1] <= row) c += step;
                }
                m += c;
                if (c == 64)        // a tile over more than 64 models
                    while (m + 1 < q.n_models && q.row_off[m + 1] <= row) ++m;
            }
            float f[kFeatures];
            const int64_t k = valid ? q.radius_off[m] + (row - q.row_off[m]) : -1;
#pragma unroll
            for (int c = 0; c < kFeatures - 1; ++c) f[c] = valid ? q.model_x[m * (kFeatures - 1) + c] : 0.0f;
            f[kFeatures - 1] = (k >= 0 && k < q.n_radius) ? q.radius[k] : 0.0f;
            stage_row(f, valid, v, xs + threadIdx.x * kLdX);
        }
    }
};

// Inference kernel.  One workgroup (4 waves) per tile of kR = 128 rows; the
// activations of the tile live in ONE LDS buffer that every hidden layer
// overwrites in place (the layer's products are complete in registers before
// the buffer is rewritten), so a workgroup takes ~80 KB of LDS and two run on
// a CU.  Wave w computes output features [64w, 64w + 64) of every layer:
// accumulators start at the (scaled) bias; the weights are read in fragment
// order (frag_index), one contiguous 1 KB load per fragment, and the fragments
// of the next kAhead k steps are in flight in a register ring; the activation
// fragments of the next step are requested right after the current step's
// first MFMA (the order within a step is pinned: left to itself the compiler
// moves the loads next to their use).  SiLU costs one exp2 and one
// reciprocal, and pairs of results are converted to BF16 together.  The output
// layer w_out . h is folded into the last hidden layer's epilogue (FP32
// activations): each lane sums its 32 features of 4 rows, the two half-waves
// and then the 4 waves are added, and the thread of each row accumulates the
// moments of T over the members.
constexpr int kPredictWaves = kThreads / 64;

// kActScale * SiLU(z) from t = kActScale * z, with the hardware exp2 and reciprocal
__device__ __forceinline__ float silu_scaled(float t) {
    return t * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(t));
}

// acc[a][b] = kActScale (bias + W . h^T) for this wave's 64 output features
// and the kR rows, from W in fragment order and hin = kActScale h; lane l holds in entry r of acc[a][b] feature 64 w + 32 a + 8 (r >> 2)
// + 4 (l >> 5) + (r & 3) of row 32 b + (l & 31).
template <int K>
__device__ __forceinline__ void predict_layer(const __bf16 *W, const float *bias, const __bf16 *hin, int ldin,
                                              f32x16 (&acc)[2][4]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int half = lane >> 5, l32 = lane & 31;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const float *bb = bias + wave * 64 + a * 32 + 4 * half;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const float4 bv = *reinterpret_cast<const float4 *>(bb + 8 * g);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                acc[a][b][4 * g + 0] = bv.x * kActScale;
                acc[a][b][4 * g + 1] = bv.y * kActScale;
                acc[a][b][4 * g + 2] = bv.z * kActScale;
                acc[a][b][4 * g + 3] = bv.w * kActScale;
            }
        }
    }
    constexpr int kSteps = K / 16;
    // fragment-ordered weights: the fragment of 32-output group q and k step st is
    // 512 contiguous values, this lane's 8 at offset 8 * lane
    const __bf16 *wrow0 = W + ((size_t)(wave * 2) * kSteps * 64 + lane) * 8;
    const __bf16 *wrow1 = wrow0 + (size_t)kSteps * 512;
    const __bf16 *hrow = hin + l32 * ldin + 8 * half;
    constexpr int kAhead = kSteps < 4 ? kSteps : 4;
    bf16x8 wa[kAhead][2], hb[2][4];
#pragma unroll
    for (int s = 0; s < kAhead; ++s) {
        wa[s][0] = *reinterpret_cast<const bf16x8 *>(wrow0 + 512 * s);
        wa[s][1] = *reinterpret_cast<const bf16x8 *>(wrow1 + 512 * s);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) hb[0][b] = *reinterpret_cast<const bf16x8 *>(hrow + b * 32 * ldin);
#pragma unroll
    for (int st = 0; st < kSteps; ++st) {
        const int k = 16 * st;
        const bf16x8 c0 = wa[st % kAhead][0], c1 = wa[st % kAhead][1];
        if (st + kAhead < kSteps) {
            wa[st % kAhead][0] = *reinterpret_cast<const bf16x8 *>(wrow0 + 512 * (st + kAhead));
            wa[st % kAhead][1] = *reinterpret_cast<const bf16x8 *>(wrow1 + 512 * (st + kAhead));
        }
        if (st + 1 < kSteps) {
#pragma unroll
            for (int b = 0; b < 4; ++b)
                hb[(st + 1) & 1][b] = *reinterpret_cast<const bf16x8 *>(hrow + b * 32 * ldin + k + 16);
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            acc[0][b] = mfma(c0, hb[st & 1][b], acc[0][b]);
            acc[1][b] = mfma(c1, hb[st & 1][b], acc[1][b]);
        }
        // one MFMA, the next step's 4 LDS reads, the 2 weight loads, the other 7 MFMAs
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
        __builtin_amdgcn_sched_group_barrier(0x020, 2, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 7, 0);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Epilogue of a hidden layer: the scaled SiLU of the accumulators.  Hidden
// layers store the values, rounded to BF16, into the tile buffer; the last
// hidden layer instead folds the output layer in (FP32 values): this wave's
// part of w_out . (kActScale h) for the 4 rows b * 32 + l32, summed over the
// two half-waves into ysum[wave][row].
template <bool kLast>
__device__ __forceinline__ void predict_epilogue(const f32x16 (&acc)[2][4], __bf16 *hout, const float *wout,
                                                 float *ysum) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    float y[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int o = wave * 64 + a * 32 + 8 * g + 4 * half;
            float4 w = float4{0.0f, 0.0f, 0.0f, 0.0f};
            if constexpr (kLast) w = *reinterpret_cast<const float4 *>(wout + o);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const float s0 = silu_scaled(acc[a][b][4 * g]), s1 = silu_scaled(acc[a][b][4 * g + 1]);
                const float s2 = silu_scaled(acc[a][b][4 * g + 2]), s3 = silu_scaled(acc[a][b][4 * g + 3]);
                if constexpr (kLast)
                    y[b] += w.x * s0 + w.y * s1 + w.z * s2 + w.w * s3;
                else
                    *reinterpret_cast<uint2 *>(hout + (b * 32 + l32) * kLd + o) =
                        uint2{pack_bf16x2(s0, s1), pack_bf16x2(s2, s3)};
            }
        }
        // one scheduling region per 64 values (measured: 4, 16, 32, 64 values or
        // none per region are within 1 %, 64 and none the fastest)
        __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (kLast) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            y[b] += __shfl_xor(y[b], 32, 64);
            if (half == 0) ysum[wave * kR + b * 32 + l32] = y[b];
        }
    }
}

template <typename Inputs>
__global__ __launch_bounds__(kThreads, 2) void sur_predict_kernel(NetView v, Inputs in, int64_t n, float *mean_logT,
                                                                  float *spread) {
    extern __shared__ __align__(16) unsigned char smem[];
    __bf16 *xs = reinterpret_cast<__bf16 *>(smem);
    __bf16 *h = xs + kR * kLdX;
    float *ysum = reinterpret_cast<float *>(h + kR * kLd);
    const int64_t row0 = (int64_t)blockIdx.x * kR;
    in(n, row0, v, xs);
    float s_log = 0.0f, s_T = 0.0f, s_T2 = 0.0f;
    f32x16 acc[2][4];
    for (int m = 0; m < v.members; ++m) {
        const __bf16 *W = v.Wf + (size_t)m * v.w_stride;
        const float *b = v.b + (size_t)m * v.b_stride;
        __syncthreads();                    // inputs staged / the previous member's sums read
        for (int l = 0; l < v.depth; ++l) {
            if (l == 0) {
                predict_layer<kIn>(W, b, xs, kLdX, acc);
            } else {
                __syncthreads();            // every wave's features of layer l - 1 stored
                predict_layer<kW>(W + (size_t)kW * kIn + (size_t)(l - 1) * kW * kW, b + l * kW, h, kLd, acc);
                if (l + 1 < v.depth) __syncthreads();   // every wave has read layer l - 1: overwrite in place
            }
            // (layer 0 reads the input tile, and the previous member's last layer only read h)
            if (l + 1 == v.depth)
                predict_epilogue<true>(acc, h, v.wout + (size_t)m * kW, ysum);
            else
                predict_epilogue<false>(acc, h, v.wout + (size_t)m * kW, ysum);
        }
        __syncthreads();                    // the waves' output sums
        if (threadIdx.x < kR) {
            float y = 0.0f;
#pragma unroll
            for (int w = 0; w < kPredictWaves; ++w) y += ysum[w * kR + threadIdx.x];
            y = y * kInvActScale + v.bout[m];
            const float lt = y * v.y_std + v.y_mean;       // log10 T of this member
            const float T = exp10f(lt);
            s_log += lt;
            s_T += T;
            s_T2 += T * T;
        }
    }
    if (threadIdx.x < kR) {
        const int64_t row = row0 + threadIdx.x;
        if (row < n) {
            const float M = (float)v.members;
            const float mT = s_T / M;
            const float var = fmaxf(s_T2 / M - mT * mT, 0.0f) * (v.members > 1 ? M / (M - 1.0f) : 0.0f);
            mean_logT[row] = s_log / M;
            spread[row] = sqrtf(var) / mT;
        }
    }
}

// Largest row spread of every model (one wave per model).
__global__ __launch_bounds__(256) void sur_model_max(const float *spread, int64_t n_rows, ModelRows q,
                                                     float *model_spread) {
    const int lane = threadIdx.x & 63;
    const int64_t m = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (m >= q.n_models) return;
    const int64_t a = q.row_off[m] > 0 ? q.row_off[m] : 0;
    const int64_t b = q.row_off[m + 1] < n_rows ? q.row_off[m + 1] : n_rows;
    float mx = 0.0f;
    for (int64_t r = a + lane; r < b; r += 64) mx = fmaxf(mx, spread[r]);
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    if (lane == 0) model_spread[m] = mx;
}

// ---------------------------------------------------------------------------
// Training, one launch per stage; blockIdx.y selects the ensemble member.

// Forward of a batch: stores every hidden activation and SiLU'(z), the output,
// and the output-layer gradient g = d loss / d y of the mean squared error.
__global__ __launch_bounds__(kThreads) void sur_train_fwd(NetView v, TrainView t) {
    extern __shared__ __align__(16) unsigned char smem[];
    __bf16 *xs = reinterpret_cast<__bf16 *>(smem);
    __bf16 *h0 = xs + kR * kLdX;
    __bf16 *h1 = h0 + kR * kLd;
    const int m = blockIdx.y;
    const int64_t n = t.batch;
    const int64_t row0 = (int64_t)blockIdx.x * kR;
    const __bf16 *W = v.Wf + (size_t)m * v.w_stride;
    const float *b = v.b + (size_t)m * v.b_stride;
    const float *X = t.xb + (size_t)m * n * kFeatures;
    const int64_t ld = t.ld;
    load_inputs(X, n, row0, v, xs);
    __syncthreads();
    // keep the normalised input tile (feature-major) for the first layer's weight gradient
    for (int j = threadIdx.x; j < kR * kIn; j += blockDim.x) {
        const int c = j / kR, r = j % kR;
        if (row0 + r < ld) t.x16[(size_t)m * kIn * ld + (size_t)c * ld + row0 + r] = xs[r * kLdX + c];
    }
    const size_t act = (size_t)m * v.depth * n * kW;   // SiLU': per member depth x [n][256]
    const size_t hact = (size_t)m * v.depth * kW * ld; // activations: per member depth x [256][ld]
    layer_fwd<true>(W, b, kIn, xs, kLdX, h0, t.h + hact, t.ds + act, row0, n, ld);
    __bf16 *hin = h0, *hout = h1;
    for (int l = 1; l < v.depth; ++l) {
        __syncthreads();
        layer_fwd<true>(W + (size_t)kW * kIn + (size_t)(l - 1) * kW * kW, b + l * kW, kW, hin, kLd, hout,
                        t.h + hact + (size_t)l * kW * ld, t.ds + act + (size_t)l * n * kW, row0, n, ld);
        __bf16 *tmp = hin; hin = hout; hout = tmp;
    }
    __syncthreads();
    const float y = out_row(hin, v.wout + (size_t)m * kW, v.bout[m]);
    if ((threadIdx.x & 1) == 0) {
        const int64_t row = row0 + (threadIdx.x >> 1);
        if (row < n) {
            const float target = (t.yb[(size_t)m * n + row] - v.y_mean) * v.y_inv_std;
            const float d = y - target;
            t.out[(size_t)m * n + row] = y;
            t.g[(size_t)m * n + row] = 2.0f * d / (float)n;
            atomicAdd(&t.loss[m], d * d / (float)n);
        }
    }
}

// Backward through the hidden layers: delta_top = g w_out (.) SiLU'(z_top), then
// delta_{l-1} = (W_l^T delta_l) (.) SiLU'(z_{l-1}); every delta is stored (BF16).
__global__ __launch_bounds__(kThreads) void sur_train_bwd(NetView v, TrainView t) {
    extern __shared__ __align__(16) unsigned char smem[];
    __bf16 *d0 = reinterpret_cast<__bf16 *>(smem);
    __bf16 *d1 = d0 + kR * kLd;
    const int m = blockIdx.y;
    const int64_t n = t.batch;
    const int64_t row0 = (int64_t)blockIdx.x * kR;
    const int L = v.depth;
    const int64_t ld = t.ld;
    const size_t act = (size_t)m * L * n * kW;      // SiLU' (row-major)
    const size_t dact = (size_t)m * L * kW * ld;    // deltas (feature-major)
    const float *wout = v.wout + (size_t)m * kW;
    // top delta
    {
        const float *ds = t.ds + act + (size_t)(L - 1) * n * kW;
        __bf16 *dg = t.delta + dact + (size_t)(L - 1) * kW * ld;
        for (int j = threadIdx.x; j < kR * kW; j += blockDim.x) {
            const int r = j / kW, c = j % kW;
            const int64_t row = row0 + r;
            float d = 0.0f;
            if (row < n) d = t.g[(size_t)m * n + row] * wout[c] * ds[row * kW + c];
            d0[r * kLd + c] = (__bf16)d;
        }
        __syncthreads();
        // feature-major copy for the weight gradient (rows [n, ld) are zero)
        for (int j = threadIdx.x; j < kR * kW; j += blockDim.x) {
            const int c = j / kR, r = j % kR;
            if (row0 + r < ld) dg[(size_t)c * ld + row0 + r] = d0[r * kLd + c];
        }
    }
    const __bf16 *WT = v.WT + (size_t)m * v.w_stride;
    __bf16 *din = d0, *dout = d1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    for (int l = L - 1; l >= 1; --l) {
        __syncthreads();
        // delta_{l-1}[row][k] = sum_o W_l[o][k] delta_l[row][o]: A = W_l^T ([in][out]), B = delta_l
        const __bf16 *A = WT + (size_t)kW * kIn + (size_t)(l - 1) * kW * kW;
        f32x16 acc[2][4];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int bb = 0; bb < 4; ++bb) acc[a][bb] = f32x16{};
        for (int kk = 0; kk < kW; kk += 16) {
            bf16x8 wa[2], hb[4];
#pragma unroll
            for (int a = 0; a < 2; ++a)
                wa[a] = *reinterpret_cast<const bf16x8 *>(A + (size_t)(wave * 64 + a * 32 + l32) * kW + kk + 8 * half);
#pragma unroll
            for (int bb = 0; bb < 4; ++bb)
                hb[bb] = *reinterpret_cast<const bf16x8 *>(din + (bb * 32 + l32) * kLd + kk + 8 * half);
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int bb = 0; bb < 4; ++bb) acc[a][bb] = mfma(wa[a], hb[bb], acc[a][bb]);
        }
        const float *ds = t.ds + act + (size_t)(l - 1) * n * kW;
        __bf16 *dg = t.delta + dact + (size_t)(l - 1) * kW * ld;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int bb = 0; bb < 4; ++bb) {
                const int r = bb * 32 + l32;
                const int64_t row = row0 + r;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int k = wave * 64 + a * 32 + 8 * g + 4 * half;
                    float4 dsv = row < n ? *reinterpret_cast<const float4 *>(ds + row * kW + k) : float4{0, 0, 0, 0};
                    bf16x4 dv;
                    dv[0] = (__bf16)(acc[a][bb][4 * g + 0] * dsv.x);
                    dv[1] = (__bf16)(acc[a][bb][4 * g + 1] * dsv.y);
                    dv[2] = (__bf16)(acc[a][bb][4 * g + 2] * dsv.z);
                    dv[3] = (__bf16)(acc[a][bb][4 * g + 3] * dsv.w);
                    *reinterpret_cast<bf16x4 *>(dout + r * kLd + k) = dv;
                    if (row < ld) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) dg[(size_t)(k + q) * ld + row] = dv[q];
                    }
                }
            }
        __bf16 *tmp = din; din = dout; dout = tmp;
    }
}

// Weight and bias gradients of the hidden layers: dW_l[o][i] = sum over rows
// of delta_l[row][o] x_l[row][i] (x_0 the inputs, x_l = h_{l-1}), db_l[o] =
// sum over rows of delta_l[row][o].  One workgroup per 64 x 64 block (o, i) of
// one layer of one member (layer 0 has 32 inputs); its 4 waves split the rows,
// each accumulating the block with MFMAs whose fragments are 16-byte reads of
// the feature-major deltas and activations (rows contiguous, so no transpose),
// the next step's fragments in flight; the waves' partial blocks are added
// through LDS and stored by one wave (each gradient entry has one writer).
constexpr int kWgBlock = 64;
__global__ __launch_bounds__(kThreads) void sur_train_wgrad(NetView v, TrainView t) {
    extern __shared__ __align__(16) unsigned char smem[];
    float *part = reinterpret_cast<float *>(smem);     // [3 waves][64 entries][64 lanes]
    const int m = blockIdx.y / v.depth, l = blockIdx.y % v.depth;
    const int Kin = l == 0 ? kIn : kW;
    const int nib = (Kin + kWgBlock - 1) / kWgBlock;
    const int tile = blockIdx.x;
    if (tile >= (kW / kWgBlock) * nib) return;        // the grid is sized for the widest layer
    const int o0 = (tile / nib) * kWgBlock, i0 = (tile % nib) * kWgBlock;
    const int nsub = (Kin - i0 < kWgBlock ? Kin - i0 : kWgBlock) / 32;   // 32-wide input blocks: 2, or 1
    const int64_t ld = t.ld;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    const __bf16 *dT = t.delta + ((size_t)m * v.depth + l) * kW * ld;
    const __bf16 *xT = l == 0 ? t.x16 + (size_t)m * kIn * ld : t.h + ((size_t)m * v.depth + (l - 1)) * kW * ld;
    const __bf16 *a0p = dT + (size_t)(o0 + l32) * ld + 8 * half;
    const __bf16 *a1p = a0p + (size_t)32 * ld;
    const __bf16 *b0p = xT + (size_t)(i0 + l32) * ld + 8 * half;
    const __bf16 *b1p = nsub == 2 ? b0p + (size_t)32 * ld : b0p;
    // this wave's rows: a contiguous quarter of the 16-row steps
    const int64_t steps = ld / 16, per = (steps + kPredictWaves - 1) / kPredictWaves;
    const int64_t s0 = wave * per, s1 = s0 + per < steps ? s0 + per : steps;
    f32x16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x16{};
    if (s0 < s1) {
        bf16x8 fa0 = *reinterpret_cast<const bf16x8 *>(a0p + s0 * 16), fa1 = *reinterpret_cast<const bf16x8 *>(a1p + s0 * 16);
        bf16x8 fb0 = *reinterpret_cast<const bf16x8 *>(b0p + s0 * 16), fb1 = *reinterpret_cast<const bf16x8 *>(b1p + s0 * 16);
        for (int64_t st = s0; st < s1; ++st) {
            const int64_t nx = (st + 1 < s1 ? st + 1 : st) * 16;
            const bf16x8 na0 = *reinterpret_cast<const bf16x8 *>(a0p + nx), na1 = *reinterpret_cast<const bf16x8 *>(a1p + nx);
            const bf16x8 nb0 = *reinterpret_cast<const bf16x8 *>(b0p + nx), nb1 = *reinterpret_cast<const bf16x8 *>(b1p + nx);
            acc[0][0] = mfma(fa0, fb0, acc[0][0]);
            acc[1][0] = mfma(fa1, fb0, acc[1][0]);
            acc[0][1] = mfma(fa0, fb1, acc[0][1]);
            acc[1][1] = mfma(fa1, fb1, acc[1][1]);
            fa0 = na0; fa1 = na1; fb0 = nb0; fb1 = nb1;
        }
    }
    // add the waves' blocks: waves 1..3 through LDS into wave 0
    if (wave > 0) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r) part[((wave - 1) * 64 + (a * 2 + b) * 16 + r) * 64 + lane] = acc[a][b][r];
    }
    __syncthreads();
    if (wave == 0) {
        float *gW = t.grad + (size_t)m * v.p_stride + (l == 0 ? 0 : (size_t)kW * kIn + (size_t)(l - 1) * kW * kW);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                if (b >= nsub) continue;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    float sum = acc[a][b][r];
#pragma unroll
                    for (int w = 0; w < kPredictWaves - 1; ++w) sum += part[(w * 64 + (a * 2 + b) * 16 + r) * 64 + lane];
                    const int o = o0 + a * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                    gW[(size_t)o * Kin + i0 + b * 32 + l32] = sum;
                }
            }
    }
    // bias gradient of this o block (the i0 = 0 workgroup): thread = (feature, quarter of the rows)
    if (i0 == 0) {
        __syncthreads();
        const int o = o0 + (threadIdx.x & 63), q = threadIdx.x >> 6;
        const int64_t r0 = (ld / 8) * q / kPredictWaves * 8, r1 = (ld / 8) * (q + 1) / kPredictWaves * 8;
        float sum = 0.0f;
        for (int64_t r = r0; r < r1; r += 8) {
            const bf16x8 d = *reinterpret_cast<const bf16x8 *>(dT + (size_t)o * ld + r);
#pragma unroll
            for (int e = 0; e < 8; ++e) sum += (float)d[e];
        }
        part[threadIdx.x] = sum;
        __syncthreads();
        if (threadIdx.x < 64)
            t.grad[(size_t)m * v.p_stride + v.off_b + (size_t)l * kW + o] =
                part[threadIdx.x] + part[threadIdx.x + 64] + part[threadIdx.x + 128] + part[threadIdx.x + 192];
    }
}

// Output-layer gradients: dw_out[c] = sum_rows g h_top[c], db_out = sum_rows g.
__global__ void sur_train_outgrad(NetView v, TrainView t) {
    const int m = blockIdx.y;
    const int64_t n = t.batch;
    const int c = threadIdx.x;
    const size_t hact = ((size_t)m * v.depth + (v.depth - 1)) * kW * t.ld + (size_t)c * t.ld;  // feature c, top layer
    const int64_t r0 = (int64_t)blockIdx.x * 256, r1 = r0 + 256 < n ? r0 + 256 : n;
    float s = 0.0f, sg = 0.0f;
    for (int64_t r = r0; r < r1; ++r) {
        const float g = t.g[(size_t)m * n + r];
        s += g * (float)t.h[hact + r];
        sg += g;
    }
    float *gp = t.grad + (size_t)m * v.p_stride;
    atomicAdd(&gp[v.off_wout + c], s);
    if (c == 0) atomicAdd(&gp[v.off_bout], sg);
}

// Adam on the FP32 master parameters with a cosine learning-rate schedule over
// total_steps; refreshes the BF16 weights and their transposes and clears the gradients.
__global__ void sur_adam(NetView v, TrainView t, const unsigned long long *step, float lr_max, float lr_min,
                         unsigned long long total_steps, float beta1, float beta2, float eps) {
    const unsigned long long s = *step;
    const float frac = total_steps > 0 ? fminf((float)s / (float)total_steps, 1.0f) : 0.0f;
    const float lr = lr_min + 0.5f * (lr_max - lr_min) * (1.0f + cospif(frac));
    const float bc1 = 1.0f - powf(beta1, (float)(s + 1));
    const float bc2 = 1.0f - powf(beta2, (float)(s + 1));
    const size_t total = (size_t)v.members * v.p_stride;
    for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < total; j += (size_t)gridDim.x * blockDim.x) {
        const float g = t.grad[j];
        const float mo = beta1 * t.adam_m[j] + (1.0f - beta1) * g;
        const float ve = beta2 * t.adam_v[j] + (1.0f - beta2) * g * g;
        t.adam_m[j] = mo;
        t.adam_v[j] = ve;
        const float p = t.master[j] - lr * (mo / bc1) / (sqrtf(ve / bc2) + eps);
        t.master[j] = p;
        t.grad[j] = 0.0f;
        scatter_param(v, (int)(j / v.p_stride), j % v.p_stride, p);
    }
}

// Copy master parameters (all members) into the BF16 weights and FP32 biases.
__global__ void sur_sync_params(NetView v, const float *master) {
    const size_t total = (size_t)v.members * v.p_stride;
    for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < total; j += (size_t)gridDim.x * blockDim.x)
        scatter_param(v, (int)(j / v.p_stride), j % v.p_stride, master[j]);
}

// Gather a random mini-batch per member (rows drawn with replacement by hashing\n// seed, step and slot with splitmix64).
__global__ void sur_gather(const float *X, const float *y, int64_t n_data, TrainView t, const unsigned long long *step,
                           unsigned long long seed, int members) {
    const int64_t B = t.batch;
    const unsigned long long s = *step;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < B * members;
         j += (int64_t)gridDim.x * blockDim.x) {
        // splitmix64 of (seed, step, slot) picks the row
        unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (s * (unsigned long long)(B * members) + (unsigned long long)j + 1);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const int64_t row = (int64_t)(z % (unsigned long long)n_data);
        for (int c = 0; c < kFeatures; ++c) t.xb[j * kFeatures + c] = X[row * kFeatures + c];
        t.yb[j] = y[row];
    }
}

__global__ void sur_zero(float *a, size_t n) {
    for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (size_t)gridDim.x * blockDim.x) a[j] = 0.0f;
}

__global__ void sur_step_inc(unsigned long long *step) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *step += 1;
}

}  // namespace

size_t predict_lds() { return (size_t)kR * kLdX * 2 + (size_t)kR * kLd * 2 + (size_t)kPredictWaves * kR * sizeof(float); }
size_t train_fwd_lds() { return (size_t)kR * kLdX * 2 + (size_t)2 * kR * kLd * 2; }
size_t bwd_lds() { return (size_t)2 * kR * kLd * 2; }
size_t wgrad_lds() { return (size_t)(kPredictWaves - 1) * 64 * 64 * sizeof(float); }

hipError_t configure() {
    hipError_t e;
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void *>(&sur_predict_kernel<RowInputs>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)predict_lds())) != hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void *>(&sur_predict_kernel<ModelInputs>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)predict_lds())) != hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void *>(&sur_train_fwd),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)train_fwd_lds())) != hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void *>(&sur_train_bwd),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)bwd_lds())) != hipSuccess)
        return e;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&sur_train_wgrad),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)wgrad_lds());
}

hipError_t launch_predict(const NetView &v, const float *X, int64_t n, float *mean_logT, float *spread, hipStream_t s) {
    const int64_t blocks = (n + kR - 1) / kR;
    hipLaunchKernelGGL(sur_predict_kernel<RowInputs>, dim3((unsigned)blocks), dim3(kThreads), predict_lds(), s, v,
                       RowInputs{X}, n, mean_logT, spread);
    return hipGetLastError();
}

hipError_t launch_predict_models(const NetView &v, const ModelRows &q, int64_t n_rows, float *mean_logT,
                                 float *spread, float *model_spread, hipStream_t s) {
    if (n_rows > 0) {
        const int64_t blocks = (n_rows + kR - 1) / kR;
        hipLaunchKernelGGL(sur_predict_kernel<ModelInputs>, dim3((unsigned)blocks), dim3(kThreads), predict_lds(), s,
                           v, ModelInputs{q}, n_rows, mean_logT, spread);
    }
    if (model_spread && q.n_models > 0)
        hipLaunchKernelGGL(sur_model_max, dim3((unsigned)((q.n_models + 3) / 4)), dim3(256), 0, s, spread, n_rows, q,
                           model_spread);
    return hipGetLastError();
}

hipError_t launch_train_step(const NetView &v, const TrainView &t, const float *X, const float *y, int64_t n_data,
                             unsigned long long seed, unsigned long long *step, float lr_max, float lr_min,
                             unsigned long long total_steps, float beta1, float beta2, float eps, int update,
                             hipStream_t s) {
    const int M = v.members;
    const bool gather = X != nullptr;
    const unsigned blocks = (unsigned)((t.batch + kR - 1) / kR);
    const unsigned groups = (unsigned)((kW / kWgBlock) * (kW / kWgBlock));   // blocks of the widest layer
    if (gather) hipLaunchKernelGGL(sur_gather, dim3(256), dim3(256), 0, s, X, y, n_data, t, step, seed, M);
    hipLaunchKernelGGL(sur_zero, dim3(1), dim3(64), 0, s, t.loss, (size_t)M);
    hipLaunchKernelGGL(sur_train_fwd, dim3(blocks, M), dim3(kThreads), train_fwd_lds(), s, v, t);
    hipLaunchKernelGGL(sur_train_bwd, dim3(blocks, M), dim3(kThreads), bwd_lds(), s, v, t);
    hipLaunchKernelGGL(sur_train_wgrad, dim3(groups, M * v.depth), dim3(kThreads), wgrad_lds(), s, v, t);
    hipLaunchKernelGGL(sur_train_outgrad, dim3((unsigned)((t.batch + 255) / 256), M), dim3(kW), 0, s, v, t);
    if (update) {
        hipLaunchKernelGGL(sur_adam, dim3(512), dim3(256), 0, s, v, t, step, lr_max, lr_min, total_steps, beta1,
                           beta2, eps);
        hipLaunchKernelGGL(sur_step_inc, dim3(1), dim3(64), 0, s, step);
    }
    return hipGetLastError();
}

hipError_t launch_sync_params(const NetView &v, const float *master, hipStream_t s) {
    hipLaunchKernelGGL(sur_sync_params, dim3(512), dim3(256), 0, s, v, master);
    return hipGetLastError();
}

hipError_t launch_zero(float *a, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(sur_zero, dim3(512), dim3(256), 0, s, a, n);
    return hipGetLastError();
}


}  // namespace sur
