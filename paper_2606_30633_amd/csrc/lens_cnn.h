// Internal declarations of the learned initializer (lens_cnn.hip, lens_cnn_api.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lens_api.h"

namespace lens {

constexpr int CNN_IN = 64;       // input side
constexpr int CNN_CONV = 6;      // 3x3 convolutions, ReLU after each
constexpr int CNN_C6 = 128;      // channels of the last convolution
constexpr int CNN_H1 = 256;      // hidden width of the MLP
constexpr int CNN_NT = 14;       // regressed parameters
constexpr int CNN_OUT = 2 * CNN_NT;   // means + log-variances
constexpr int CNN_MAXD = 64;

// K-splits of a weight-gradient GEMM over K output positions: about 64 K steps
// of 32 per split (so that small outputs still fill the GPU), at most 1024.
inline int wgrad_splits(long long K) {
    const long long s = K / 2048;
    return (int)(s < 1 ? 1 : (s > 1024 ? 1024 : s));
}

struct CnnLayer {
    int cin, cout, stride;
    long long w_off, b_off;   // offsets into the flat parameter vector
};

// Bias gradients are column sums over row chunks (fixed order): rows per
// chunk for a matrix of `rows` rows, and the chunk-partial buffer size that
// covers every layer at a batch limit (chunks <= max(batch, 288), columns <= 256).
inline int colsum_rows_per_chunk(int rows) {
    if (rows >= 262144) return 1024;
    const int r = rows / 256;
    return r < 8 ? 8 : r;
}
inline long long colpart_capacity(int max_batch) {
    return ((long long)(max_batch > 288 ? max_batch : 288) + 1) * CNN_H1;
}

// Where the network's outputs go in a parameter vector, and the prior of the rest.
struct CnnTargetMap {
    int d;
    int prior_kind[CNN_MAXD];
    double prior[CNN_MAXD][4];   // (a, b, lo, hi) as in lens_plan_set_prior
    int cnn_slot[CNN_MAXD];      // network output index, or -1: drawn from the prior
    double mean[CNN_NT], stdv[CNN_NT];
};

struct CnnNet {
    int max_batch;
    long long nparams;
    CnnLayer conv[CNN_CONV];
    CnnLayer fc1, fc2;
    float* params;      // fp32 master copy
    float* grads;
    float* adam_m;
    float* adam_v;
    __bf16* wbf;        // bf16 copy used by the GEMMs
    __bf16* act[CNN_CONV];
    __bf16* dact[CNN_CONV];
    __bf16* pooled;
    float* dpooled;
    __bf16* hidden;
    __bf16* dhidden;
    float* out;
    __bf16* dout;
    float* wpart;
    double* colpart;
    double* losspart;
    double* c0part;       // [max_batch][32][10] first-layer weight and bias gradient per image
    CnnTargetMap* tmap;   // device copy
    __bf16* prep;         // prepared images for init_propose
    __bf16* img_stage;    // [max_batch][64][64] the training batch (captured step)
    float* tgt_stage;     // [max_batch][CNN_NT]
    float* hyper;         // [2] learning rate, Adam step (device)
    float* loss_dev;      // [1]
    hipGraphExec_t train_graph;   // one captured training step (forward, backward, Adam)
    int graph_batch;
    hipStream_t cap_stream;
    int step;
    float sigma;
    bool has_map;
};

hipError_t cnn_forward(CnnNet& net, int B, const __bf16* img, hipStream_t st);
hipError_t cnn_backward(CnnNet& net, int B, const __bf16* img, const float* target, float* loss, hipStream_t st);
// Adam with the learning rate and step of net.hyper (cnn_set_hyper).
hipError_t cnn_adam(CnnNet& net, hipStream_t st);
hipError_t cnn_set_hyper(CnnNet& net, float lr, int step, hipStream_t st);
hipError_t cnn_init(CnnNet& net, uint64_t seed, hipStream_t st);
hipError_t cnn_params_to_bf16(CnnNet& net, hipStream_t st);
hipError_t cnn_prepare(long long n, const float* img, float sigma, int add_noise, uint64_t seed, uint64_t counter0,
                       __bf16* out, hipStream_t st);
hipError_t cnn_propose(int S, int s0, int n, int d, const float* net_out, const CnnTargetMap* tm, uint64_t seed,
                       float* theta, int* flags, hipStream_t st);

}  // namespace lens
