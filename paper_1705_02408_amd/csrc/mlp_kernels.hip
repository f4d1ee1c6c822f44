// Learned per-edge drift surrogate on the gfx950 matrix cores.
//
// Network: y = w3 . relu(W2^T h1 + b2) + b3,  h1 = bf16(relu(W1^T x + b1)),
// 16 -> 64 -> 64 -> 1, x and the weights in bfloat16, float32 accumulation
// (v_mfma_f32_32x32x16_bf16).  The prediction is the edge's mean
// "1 - quality" along its length; the drift increment is length * clamp(y, 0, 1).
//
// Layout.  One wave computes 32 edges at a time as transposed products
// (hidden x edges), so every lane owns one edge (lane % 32) and the
// accumulator registers of one layer can feed the B operand of the next
// directly.  For the 32x32 MFMA, accumulator register v of lane l holds row
// 8*(v/4) + 4*(l/32) + v%4 and column l%32; operand slot e of lane l holds
// K index 8*(l/32) + e.  Hidden units reach layer 2 in that row order, and the
// layer-2 weight fragments are loaded in the same permuted order.
//
// Training: forward over a batch (also writing bfloat16 transposed copies of
// the inputs, first activations and output gradients), backward through layer
// 2 on the matrix cores, and weight gradients as matrix products with the
// batch as the K dimension.  Every wave writes its partial sums; one kernel
// sums them in a fixed order (deterministic) and applies Adam.
#include "device_common.h"
#include "mlp_kernels.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short short8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {

__device__ __forceinline__ bf16x8 load8(const uint16_t *p) {
    const uint4 q = *reinterpret_cast<const uint4 *>(p);
    return __builtin_bit_cast(bf16x8, q);
}
__device__ __forceinline__ bf16x8 zero8() {
    const uint4 q = make_uint4(0u, 0u, 0u, 0u);
    return __builtin_bit_cast(bf16x8, q);
}
__device__ __forceinline__ bf16x8 pack8(const uint16_t *v) {
    short8 s;
#pragma unroll
    for (int e = 0; e < 8; ++e) s[e] = (short)v[e];
    return __builtin_bit_cast(bf16x8, s);
}
__device__ __forceinline__ f32x16 mfma(const bf16x8 &a, const bf16x8 &b, const f32x16 &c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
// accumulator register v of a lane in half h holds tile row rowmap(v, h)
__device__ __forceinline__ int rowmap(int v, int h) { return 8 * (v >> 2) + 4 * h + (v & 3); }

struct Frags {
    bf16x8 a1[2];        // W1^T, hidden tile t
    bf16x8 a2[2][2][2];  // W2^T, output tile, input tile, K half
};

__device__ __forceinline__ void load_frags(const MlpDev &d, int h, int c, Frags &f) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        uint16_t v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = d.pb[kBfW1 + (8 * h + e) * kMlpH + 32 * t + c];
        f.a1[t] = pack8(v);
    }
#pragma unroll
    for (int to = 0; to < 2; ++to)
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int hs = 0; hs < 2; ++hs) {
                uint16_t v[8];
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    v[e] = d.pb[kBfW2 + (32 * ti + rowmap(8 * hs + e, h)) * kMlpH + 32 * to + c];
                f.a2[to][ti][hs] = pack8(v);
            }
}

// Forward of the 32 edges whose features the lane pair holds in bx.  Returns
// the output (both halves), the layer-1 accumulators (pre-bias) and the
// layer-2 pre-activations z2.
__device__ __forceinline__ float forward32(const Frags &f, const bf16x8 &bx, const float *sb1,
                                           const float *sb2, const float *sw3, float sb3,
                                           int h, f32x16 (&d1)[2], uint16_t (&h1)[2][16],
                                           f32x16 (&z2)[2]) {
    const f32x16 zero = {};
    d1[0] = mfma(f.a1[0], bx, zero);
    d1[1] = mfma(f.a1[1], bx, zero);
    bf16x8 bh[2][2];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti) {
#pragma unroll
        for (int v = 0; v < 16; ++v)
            h1[ti][v] = f2bf(fmaxf(d1[ti][v] + sb1[32 * ti + rowmap(v, h)], 0.0f));
        bh[ti][0] = pack8(&h1[ti][0]);
        bh[ti][1] = pack8(&h1[ti][8]);
    }
    float y = 0.0f;
#pragma unroll
    for (int to = 0; to < 2; ++to) {
        f32x16 acc = {};
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int hs = 0; hs < 2; ++hs) acc = mfma(f.a2[to][ti][hs], bh[ti][hs], acc);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int o = 32 * to + rowmap(v, h);
            const float z = acc[v] + sb2[o];
            z2[to][v] = z;
            y += sw3[o] * fmaxf(z, 0.0f);
        }
    }
    y += __shfl_xor(y, 32, 64);
    return y + sb3;
}

__device__ __forceinline__ void load_small(const MlpDev &d, float *sb1, float *sb2, float *sw3,
                                           float *sb3) {
    for (int i = threadIdx.x; i < kMlpH; i += blockDim.x) {
        sb1[i] = d.p[kOffB1 + i];
        sb2[i] = d.p[kOffB2 + i];
        sw3[i] = bf2f(d.pb[kBfW3 + i]);
    }
    if (threadIdx.x == 0) *sb3 = d.p[kOffB3];
    __syncthreads();
}

// sum over the 32 lanes of each half (the 32 edges of a tile)
__device__ __forceinline__ float half_sum(float v) {
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace

// y = network(X[i]) and drift = len * clamp(base + y / kResidualScale, 0, 1).
__global__ void __launch_bounds__(256) k_mlp_infer(MlpDev d, const uint16_t *X, long long n,
                                                   const float *len, const float *base, float *y,
                                                   float *drift) {
    __shared__ float sb1[kMlpH], sb2[kMlpH], sw3[kMlpH], sb3;
    load_small(d, sb1, sb2, sw3, &sb3);
    const int l = lane_id(), h = l >> 5, c = l & 31;
    Frags f;
    load_frags(d, h, c, f);
    const long long waves = (long long)gridDim.x * (blockDim.x >> 6);
    for (long long tile = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
         tile * 32 < n; tile += waves) {
        const long long i = tile * 32 + c;
        const bool valid = i < n;
        const bf16x8 bx = valid ? load8(X + i * kMlpIn + 8 * h) : zero8();
        f32x16 d1[2], z2[2];
        uint16_t h1[2][16];
        const float out = forward32(f, bx, sb1, sb2, sw3, sb3, h, d1, h1, z2);
        if (h == 0 && valid) {
            if (y) y[i] = out;
            if (drift) {
                const float r = (base ? base[i] : 0.0f) + out * (1.0f / kResidualScale);
                drift[i] = len[i] * fminf(fmaxf(r, 0.0f), 1.0f);
            }
        }
    }
}

// Training forward over the batch rows t.idx[0..B): outputs, transposed bf16
// copies for the weight gradients, the layer-2 output gradient dZ2 and the
// partial sums of the w3, b2, b3 gradients.  Launch exactly t.nparts waves.
__global__ void __launch_bounds__(256) k_mlp_train_fwd(MlpDev d, MlpTrain t) {
    __shared__ float sb1[kMlpH], sb2[kMlpH], sw3[kMlpH], sb3;
    load_small(d, sb1, sb2, sw3, &sb3);
    const int l = lane_id(), h = l >> 5, c = l & 31;
    Frags f;
    load_frags(d, h, c, f);
    const int g = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    float gw3[2][16], gb2[2][16], gb3 = 0.0f;
#pragma unroll
    for (int to = 0; to < 2; ++to)
#pragma unroll
        for (int v = 0; v < 16; ++v) gw3[to][v] = gb2[to][v] = 0.0f;
    const float inv = 2.0f / (float)t.B;
    for (int tile = g; tile * 32 < t.B; tile += t.nparts) {
        const int b = tile * 32 + c;
        const long long row = t.idx[b];
        const bf16x8 bx = load8(t.X + row * kMlpIn + 8 * h);
        {
            const uint4 raw = __builtin_bit_cast(uint4, bx);
            const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
            for (int e = 0; e < 8; ++e)
                t.XT[(8 * h + e) * t.B + b] = (uint16_t)(w[e >> 1] >> (16 * (e & 1)));
        }
        f32x16 d1[2], z2[2];
        uint16_t h1[2][16];
        const float y = forward32(f, bx, sb1, sb2, sw3, sb3, h, d1, h1, z2);
        uint64_t msk = 0;
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int hid = 32 * ti + rowmap(v, h);
                t.H1T[hid * t.B + b] = h1[ti][v];
                if (d1[ti][v] + sb1[hid] > 0.0f) msk |= 1ull << hid;
            }
        msk |= __shfl_xor(msk, 32, 64);
        const float dy = inv * (y - t.t[row]);
        if (h == 0) {
            t.y[b] = y;
            t.mask1[b] = msk;
            gb3 += dy;
        }
#pragma unroll
        for (int to = 0; to < 2; ++to)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int o = 32 * to + rowmap(v, h);
                const float z = z2[to][v];
                const float dz = z > 0.0f ? dy * sw3[o] : 0.0f;
                const uint16_t dzb = f2bf(dz);
                t.dZ2[b * kMlpH + o] = dzb;
                t.dZ2T[o * t.B + b] = dzb;
                gw3[to][v] += dy * fmaxf(z, 0.0f);
                gb2[to][v] += dz;
            }
    }
    float *part = t.part + (size_t)g * kGradWords;
#pragma unroll
    for (int to = 0; to < 2; ++to)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const float s3 = half_sum(gw3[to][v]);
            const float s2 = half_sum(gb2[to][v]);
            if (c == 0) {
                const int o = 32 * to + rowmap(v, h);
                part[kOffW3 + o] = s3;
                part[kOffB2 + o] = s2;
            }
        }
    gb3 = half_sum(gb3);
    if (l == 0) part[kOffB3] = gb3;
}

// dZ1 = mask1 * (W2 dZ2) on the matrix cores, stored transposed in bfloat16,
// and the partial sums of the b1 gradient.  Launch exactly t.nparts waves.
__global__ void __launch_bounds__(256) k_mlp_train_bwd_h(MlpDev d, MlpTrain t) {
    const int l = lane_id(), h = l >> 5, c = l & 31;
    const int g = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    // A fragments of W2 (rows hidden, K over outputs in natural order)
    bf16x8 aw[2][4];
#pragma unroll
    for (int th = 0; th < 2; ++th)
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) aw[th][ks] = load8(d.pb + kBfW2 + (32 * th + c) * kMlpH + 16 * ks + 8 * h);
    float gb1[2][16];
#pragma unroll
    for (int th = 0; th < 2; ++th)
#pragma unroll
        for (int v = 0; v < 16; ++v) gb1[th][v] = 0.0f;
    for (int tile = g; tile * 32 < t.B; tile += t.nparts) {
        const int b = tile * 32 + c;
        const uint64_t msk = t.mask1[b];
#pragma unroll
        for (int th = 0; th < 2; ++th) {
            f32x16 acc = {};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
                acc = mfma(aw[th][ks], load8(t.dZ2 + b * kMlpH + 16 * ks + 8 * h), acc);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int hid = 32 * th + rowmap(v, h);
                const float dz = ((msk >> hid) & 1ull) ? acc[v] : 0.0f;
                t.dZ1T[hid * t.B + b] = f2bf(dz);
                gb1[th][v] += dz;
            }
        }
    }
    float *part = t.part + (size_t)g * kGradWords;
#pragma unroll
    for (int th = 0; th < 2; ++th)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const float s = half_sum(gb1[th][v]);
            if (c == 0) part[kOffB1 + 32 * th + rowmap(v, h)] = s;
        }
}

// Weight gradients with the batch as the K dimension: wave g sums the rows
// [g*K, (g+1)*K) of the batch, K = B / nparts (a multiple of 16).
//   dW2^T[o][j] = sum_b dZ2T[o][b] H1T[j][b],   dW1^T[j][f] = sum_b dZ1T[j][b] XT[f][b]
__global__ void __launch_bounds__(256) k_mlp_train_bwd_w(MlpDev d, MlpTrain t) {
    const int l = lane_id(), h = l >> 5, c = l & 31;
    const int g = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int K = t.B / t.nparts;
    const int b0 = g * K;
    f32x16 a2[2][2] = {};  // [output tile][hidden tile]
    f32x16 a1[2] = {};     // [hidden tile], columns = features
    for (int k0 = b0; k0 < b0 + K; k0 += 16) {
        const int kk = k0 + 8 * h;
        bf16x8 dz2[2], h1[2], dz1[2];
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            dz2[tt] = load8(t.dZ2T + (32 * tt + c) * t.B + kk);
            h1[tt] = load8(t.H1T + (32 * tt + c) * t.B + kk);
            dz1[tt] = load8(t.dZ1T + (32 * tt + c) * t.B + kk);
        }
        const bf16x8 xt = (c < kMlpIn) ? load8(t.XT + c * t.B + kk) : zero8();
#pragma unroll
        for (int to = 0; to < 2; ++to)
#pragma unroll
            for (int th = 0; th < 2; ++th) a2[to][th] = mfma(dz2[to], h1[th], a2[to][th]);
#pragma unroll
        for (int th = 0; th < 2; ++th) a1[th] = mfma(dz1[th], xt, a1[th]);
    }
    float *part = t.part + (size_t)g * kGradWords;
#pragma unroll
    for (int to = 0; to < 2; ++to)
#pragma unroll
        for (int th = 0; th < 2; ++th)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int o = 32 * to + rowmap(v, h);
                const int j = 32 * th + c;
                part[kOffW2 + j * kMlpH + o] = a2[to][th][v];
            }
    if (c < kMlpIn)
#pragma unroll
        for (int th = 0; th < 2; ++th)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int j = 32 * th + rowmap(v, h);
                part[kOffW1 + c * kMlpH + j] = a1[th][v];
            }
}

// Sum the per-wave partials in a fixed order, then (optionally) one Adam step
// on the float32 masters and a refresh of the bfloat16 copies.
__global__ void __launch_bounds__(256) k_mlp_adam(MlpAdam a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kMlpParams) return;
    float gs = 0.0f;
    for (int g = 0; g < a.nparts; ++g) gs += a.part[(size_t)g * kGradWords + i];
    if (a.grad_out) a.grad_out[i] = gs;
    if (!a.apply) return;
    const float m = a.beta1 * a.m[i] + (1.0f - a.beta1) * gs;
    const float v = a.beta2 * a.v[i] + (1.0f - a.beta2) * gs * gs;
    a.m[i] = m;
    a.v[i] = v;
    const float p = a.p[i] - a.lr * (m / a.c1) / (sqrtf(v / a.c2) + a.eps);
    a.p[i] = p;
    if (i < kOffB1) a.pb[kBfW1 + (i - kOffW1)] = f2bf(p);
    else if (i >= kOffW2 && i < kOffB2) a.pb[kBfW2 + (i - kOffW2)] = f2bf(p);
    else if (i >= kOffW3 && i < kOffB3) a.pb[kBfW3 + (i - kOffW3)] = f2bf(p);
}

__global__ void __launch_bounds__(256) k_mlp_to_bf16(const float *p, uint16_t *pb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kMlpIn * kMlpH) pb[kBfW1 + i] = f2bf(p[kOffW1 + i]);
    if (i < kMlpH * kMlpH) pb[kBfW2 + i] = f2bf(p[kOffW2 + i]);
    if (i < kMlpH) pb[kBfW3 + i] = f2bf(p[kOffW3 + i]);
}
