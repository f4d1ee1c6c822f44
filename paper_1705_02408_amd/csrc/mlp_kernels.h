// Learned per-edge drift surrogate: 16 -> 64 -> 64 -> 1 ReLU network with
// bfloat16 inputs, weights and first hidden activations and float32
// accumulation on the gfx950 matrix cores.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

constexpr int kMlpIn = 16;
constexpr int kMlpH = 64;
// float32 parameter block: W1[16][64] b1[64] W2[64][64] b2[64] w3[64] b3[1]
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpIn * kMlpH;
constexpr int kOffW2 = kOffB1 + kMlpH;
constexpr int kOffB2 = kOffW2 + kMlpH * kMlpH;
constexpr int kOffW3 = kOffB2 + kMlpH;
constexpr int kOffB3 = kOffW3 + kMlpH;
constexpr int kMlpParams = kOffB3 + 1;  // 5313
// bfloat16 copies: W1[16][64], W2[64][64], w3[64]
constexpr int kBfW1 = 0;
constexpr int kBfW2 = kBfW1 + kMlpIn * kMlpH;
constexpr int kBfW3 = kBfW2 + kMlpH * kMlpH;
constexpr int kMlpBf = kBfW3 + kMlpH;
// partial sums written by one training wave (gradient of every parameter)
constexpr int kGradWords = kMlpParams;

struct MlpDev {
    const float *p;        // float32 masters [kMlpParams]
    const uint16_t *pb;    // bfloat16 copies [kMlpBf]
};

// Training scratch for one batch of B rows.
struct MlpTrain {
    const uint16_t *X;      // features of the training set [n][16] (bf16 bits)
    const float *t;         // targets [n]
    const long long *idx;   // batch rows (indices into X / t), [B]
    int B;                  // batch size, a multiple of 32
    uint16_t *XT;           // [16][B] batch features, transposed
    uint16_t *H1T;          // [64][B] bf16(relu(z1)), transposed
    uint64_t *mask1;        // [B] bit h: z1[h] > 0
    uint16_t *dZ2;          // [B][64] bf16(dL/dz2)
    uint16_t *dZ2T;         // [64][B]
    uint16_t *dZ1T;         // [64][B] bf16(dL/dz1)
    float *y;               // [B] outputs
    float *part;            // [nparts][kGradWords] per-wave gradient partial sums
    int nparts;
};

struct MlpAdam {
    float *p;       // masters
    uint16_t *pb;   // bf16 copies
    float *m, *v;   // moments
    const float *part;
    int nparts;
    float lr, beta1, beta2, eps;
    float c1, c2;   // bias corrections 1 - beta1^step, 1 - beta2^step
    float *grad_out;  // optional: the summed gradient (for checks), may be null
    int apply;        // 0: only sum the gradient
};

// The network predicts the correction to the 8-point base in units of
// 1/kResidualScale (a power of two, so the rescaling is exact).
constexpr float kResidualScale = 256.0f;

// y = network(X[i]) (nullable) and
// drift = len * clamp(base + y / kResidualScale, 0, 1) (nullable; base nullable = 0)
__global__ void k_mlp_infer(MlpDev d, const uint16_t *X, long long n, const float *len,
                            const float *base, float *y, float *drift);
__global__ void k_mlp_train_fwd(MlpDev d, MlpTrain t);
__global__ void k_mlp_train_bwd_h(MlpDev d, MlpTrain t);
__global__ void k_mlp_train_bwd_w(MlpDev d, MlpTrain t);
__global__ void k_mlp_adam(MlpAdam a);
__global__ void k_mlp_to_bf16(const float *p, uint16_t *pb);
