// C ABI of the learned per-edge drift surrogate (see include/mpap.h): inputs,
// training, scoring of a roadmap's edges, and the analytic re-walk that
// judges a search run on the surrogate's drift.
#include "device_common.h"
#include "mlp_kernels.h"
#include "runtime_internal.h"
#include "steer_kernels.h"

// out[i] = in[perm[i]]
__global__ void k_gather_f32(long long n, const int *perm, const float *in, float *out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[perm[i]];
}

struct mpap_surrogate {
    int dev = -1;
    float *p = nullptr;      // float32 masters [kMlpParams]
    uint16_t *pb = nullptr;  // bfloat16 copies [kMlpBf]
    float *m = nullptr, *v = nullptr;
    int step = 0;
    // training scratch (grown on demand)
    int B = 0, nparts = 0;
    uint16_t *XT = nullptr, *H1T = nullptr, *dZ2 = nullptr, *dZ2T = nullptr, *dZ1T = nullptr;
    uint64_t *mask1 = nullptr;
    float *y = nullptr, *part = nullptr, *grad = nullptr;
    long long *idx = nullptr;
    long long idx_cap = 0;
    float *t_all = nullptr;  // targets of the graph trained on
    long long t_cap = 0;
    float *sq = nullptr;     // loss accumulator
};

namespace {

void sur_free_scratch(mpap_surrogate *s) {
    dfree(s->XT); dfree(s->H1T); dfree(s->dZ2); dfree(s->dZ2T); dfree(s->dZ1T);
    dfree(s->mask1); dfree(s->y); dfree(s->part); dfree(s->grad);
    s->B = 0;
}

// batch sizes are powers of two >= 64; nparts waves each sum B/nparts rows
int sur_scratch(mpap_surrogate *s, int B) {
    if (B < 64 || (B & (B - 1))) return fail(MPAP_ERR_INVAL, "batch must be a power of two >= 64");
    if (B == s->B) return MPAP_OK;
    sur_free_scratch(s);
    const int nparts = std::min(64, B / 64);
    int r;
    if ((r = dalloc(&s->XT, (size_t)kMlpIn * B)) || (r = dalloc(&s->H1T, (size_t)kMlpH * B)) ||
        (r = dalloc(&s->dZ2, (size_t)kMlpH * B)) || (r = dalloc(&s->dZ2T, (size_t)kMlpH * B)) ||
        (r = dalloc(&s->dZ1T, (size_t)kMlpH * B)) || (r = dalloc(&s->mask1, B)) ||
        (r = dalloc(&s->y, B)) || (r = dalloc(&s->part, (size_t)nparts * kGradWords)) ||
        (r = dalloc(&s->grad, kMlpParams)))
        return r;
    s->B = B;
    s->nparts = nparts;
    return MPAP_OK;
}

MlpDev dev_view(const mpap_surrogate *s) {
    MlpDev d;
    d.p = s->p;
    d.pb = s->pb;
    return d;
}

MlpTrain train_view(mpap_surrogate *s, const uint16_t *X, const float *t, const long long *idx) {
    MlpTrain tr{};
    tr.X = X; tr.t = t; tr.idx = idx; tr.B = s->B;
    tr.XT = s->XT; tr.H1T = s->H1T; tr.mask1 = s->mask1; tr.dZ2 = s->dZ2; tr.dZ2T = s->dZ2T;
    tr.dZ1T = s->dZ1T; tr.y = s->y; tr.part = s->part; tr.nparts = s->nparts;
    return tr;
}

// one batch: forward, backward, and (apply) an Adam step; grad_out optional
int sur_batch(mpap_surrogate *s, const uint16_t *X, const float *t, const long long *idx,
              float lr, bool apply, float *grad_out, hipStream_t st) {
    const MlpDev d = dev_view(s);
    const MlpTrain tr = train_view(s, X, t, idx);
    const int blocks = s->nparts / 4 > 0 ? s->nparts / 4 : 1;
    const int threads = (s->nparts >= 4 ? 4 : s->nparts) * 64;
    k_mlp_train_fwd<<<blocks, threads, 0, st>>>(d, tr);
    k_mlp_train_bwd_h<<<blocks, threads, 0, st>>>(d, tr);
    k_mlp_train_bwd_w<<<blocks, threads, 0, st>>>(d, tr);
    MlpAdam ad{};
    ad.p = s->p; ad.pb = s->pb; ad.m = s->m; ad.v = s->v; ad.part = s->part;
    ad.nparts = s->nparts; ad.lr = lr; ad.beta1 = 0.9f; ad.beta2 = 0.999f; ad.eps = 1e-8f;
    ad.grad_out = grad_out; ad.apply = apply ? 1 : 0;
    if (apply) {
        s->step += 1;
        ad.c1 = (float)(1.0 - std::pow(0.9, (double)s->step));
        ad.c2 = (float)(1.0 - std::pow(0.999, (double)s->step));
    }
    k_mlp_adam<<<div_up(kMlpParams, 256), 256, 0, st>>>(ad);
    HIP_TRY(hipGetLastError());
    return MPAP_OK;
}

// acc += sum over i < n of (y[idx[i]] - t[idx[i]])^2
__global__ void k_sq_err(const float *y, const float *t, const long long *idx, long long n,
                         float *acc) {
    float s = 0.f;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const long long k = idx[i];
        const float d = y[k] - t[k];
        s += d * d;
    }
    s = wave_sum(s);
    if (lane_id() == 0) atomicAdd(acc, s);
}

__global__ void k_zero_f32(float *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

SteerArgs steer_view(const mpap_graph *g) {
    SteerArgs a{};
    a.n = g->n; a.pos = g->pos; a.vel = g->vel; a.nbox = 0; a.nblob = g->nblob; a.mu = g->bmu;
    a.sig = g->bsig; a.amp = g->bamp; a.T = g->horizon; a.K = g->traj_steps; a.k_out = g->k_out;
    return a;
}

// edge lengths the drift is proportional to (trajectory length for dim 6)
const float *drift_length(const mpap_graph *g) { return g->elen ? g->elen : g->ocost; }

// surrogate inputs and 8-point base of every edge, enqueued on st
int enqueue_features(mpap_graph *g, hipStream_t st) {
    if (!g->pos) return fail(MPAP_ERR_INVAL, "graph has no environment (build it with mpap_build_graph)");
    int r;
    if (!g->feat && (r = dalloc(&g->feat, (size_t)std::max<long long>(g->e, 1) * kMlpIn))) return r;
    if (!g->sbase && (r = dalloc(&g->sbase, std::max<long long>(g->e, 1)))) return r;
    if (g->n == 0) return MPAP_OK;
    if (g->dim == 6) {
        if (g->e > 0)
            k_traj_features<<<div_up(g->e, 256), 256, sizeof(float) * 5 * (size_t)g->nblob,
                              st>>>(steer_view(g), g->optr, g->ocol, g->elen, g->feat, g->sbase);
    } else {
        BuildArgs a{};
        a.n = g->n; a.dim = g->dim; a.pos = g->pos; a.nblob = g->nblob; a.mu = g->bmu;
        a.sig = g->bsig; a.amp = g->bamp; a.r = g->radius; a.step = g->check_step;
        a.reset_q = g->reset_q;
        const size_t lds = sizeof(float) * ((size_t)g->nblob * g->dim + 2 * (size_t)g->nblob);
        if (g->e > 0 && g->uptr)
            k_edge_features_pairs<<<div_up(g->e / 2 + 1, 256), 256, lds, st>>>(
                a, g->n, g->optr, g->ocol, g->ocost, g->uptr, g->feat, g->sbase);
        else if (g->e > 0)
            k_edge_features<<<div_up(g->e, 256), 256, lds, st>>>(a, g->n, g->optr, g->ocol,
                                                                 g->ocost, g->feat, g->sbase);
    }
    HIP_TRY(hipGetLastError());
    return MPAP_OK;
}

// graph features on demand (roadmaps built by mpap_build_graph only)
int ensure_features(mpap_graph *g, hipStream_t st) {
    if (g->feat) return MPAP_OK;
    int r = enqueue_features(g, st);
    if (r) return r;
    HIP_TRY(hipStreamSynchronize(st));
    return MPAP_OK;
}

// counter-based SplitMix64 and Box-Muller for the He-normal initialisation
uint64_t sm64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
double unit(uint64_t key, uint64_t i) {
    return ((double)(sm64(key + (i + 1) * 0x9E3779B97F4A7C15ull) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

// 32-bit FNV-1a of a byte range (the check word of saved parameters)
uint32_t fnv1a(const void *data, size_t n) {
    const unsigned char *b = static_cast<const unsigned char *>(data);
    uint32_t h = 2166136261u;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 16777619u;
    }
    return h;
}
constexpr char kSurMagic[8] = {'M', 'P', 'A', 'P', 'S', 'U', 'R', '1'};

}  // namespace

extern "C" {

int mpap_surrogate_create(mpap_surrogate **out) {
    if (!out) return fail(MPAP_ERR_INVAL, "out is null");
    *out = nullptr;
    DeviceInfo di;
    int r = device_info(&di);
    if (r) return r;
    mpap_surrogate *s = new mpap_surrogate();
    s->dev = di.dev;
    if ((r = dalloc(&s->p, kMlpParams)) || (r = dalloc(&s->pb, kMlpBf)) ||
        (r = dalloc(&s->m, kMlpParams)) || (r = dalloc(&s->v, kMlpParams)) ||
        (r = dalloc(&s->sq, 1))) {
        mpap_surrogate_free(s);
        return r;
    }
    std::vector<float> z(kMlpParams, 0.f);
    HIP_TRY(hipMemcpy(s->p, z.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(s->m, z.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(s->v, z.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    k_mlp_to_bf16<<<div_up(kMlpH * kMlpH, 256), 256>>>(s->p, s->pb);
    HIP_TRY(hipDeviceSynchronize());
    *out = s;
    return MPAP_OK;
}

void mpap_surrogate_free(mpap_surrogate *s) {
    if (!s) return;
    sur_free_scratch(s);
    dfree(s->p); dfree(s->pb); dfree(s->m); dfree(s->v); dfree(s->idx); dfree(s->t_all);
    dfree(s->sq);
    delete s;
}

int mpap_surrogate_set_params(mpap_surrogate *s, const float *params, int32_t count) {
    if (!s || !params) return fail(MPAP_ERR_INVAL, "null argument");
    if (count != kMlpParams) return fail(MPAP_ERR_INVAL, "expected 5313 parameters");
    for (int i = 0; i < count; ++i)
        if (!std::isfinite(params[i])) return fail(MPAP_ERR_INVAL, "non-finite parameter");
    HIP_TRY(hipMemcpy(s->p, params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    std::vector<float> z(kMlpParams, 0.f);
    HIP_TRY(hipMemcpy(s->m, z.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(s->v, z.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    s->step = 0;
    k_mlp_to_bf16<<<div_up(kMlpH * kMlpH, 256), 256>>>(s->p, s->pb);
    HIP_TRY(hipDeviceSynchronize());
    return MPAP_OK;
}

int mpap_surrogate_get_params(const mpap_surrogate *s, float *params, int32_t capacity,
                              int32_t *count) {
    if (!s || !count) return fail(MPAP_ERR_INVAL, "null argument");
    *count = kMlpParams;
    if (capacity < kMlpParams) return fail(MPAP_ERR_CAPACITY, "capacity below 5313");
    HIP_TRY(hipMemcpy(params, s->p, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
    return MPAP_OK;
}

int mpap_surrogate_init(mpap_surrogate *s, uint64_t seed) {
    if (!s) return fail(MPAP_ERR_INVAL, "null surrogate");
    std::vector<float> p(kMlpParams, 0.f);
    const uint64_t key = sm64(seed * 0x9E3779B97F4A7C15ull ^ 11ull);
    uint64_t k = 0;
    auto normal = [&]() {
        const double u1 = unit(key, k++), u2 = unit(key, k++);
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    };
    for (int i = 0; i < kMlpIn * kMlpH; ++i) p[kOffW1 + i] = (float)(normal() * std::sqrt(2.0 / kMlpIn));
    for (int i = 0; i < kMlpH * kMlpH; ++i) p[kOffW2 + i] = (float)(normal() * std::sqrt(2.0 / kMlpH));
    // output layer zero: an untrained network predicts exactly the 8-point base
    return mpap_surrogate_set_params(s, p.data(), kMlpParams);
}

int mpap_surrogate_save(const mpap_surrogate *s, const char *path) {
    if (!s || !path) return fail(MPAP_ERR_INVAL, "null argument");
    std::vector<float> p(kMlpParams);
    HIP_TRY(hipMemcpy(p.data(), s->p, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
    const uint32_t h = fnv1a(p.data(), sizeof(float) * kMlpParams);
    const int32_t cnt = kMlpParams;
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(MPAP_ERR_INVAL, std::string("cannot open ") + path + " for writing");
    bool ok = std::fwrite(kSurMagic, 1, 8, f) == 8 && std::fwrite(&cnt, 4, 1, f) == 1 &&
              std::fwrite(p.data(), sizeof(float), kMlpParams, f) == (size_t)kMlpParams &&
              std::fwrite(&h, 4, 1, f) == 1;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return fail(MPAP_ERR_INVAL, std::string("cannot write ") + path);
    return MPAP_OK;
}

int mpap_surrogate_load(mpap_surrogate *s, const char *path) {
    if (!s || !path) return fail(MPAP_ERR_INVAL, "null argument");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(MPAP_ERR_INVAL, std::string("cannot open ") + path);
    char magic[8] = {};
    int32_t cnt = 0;
    uint32_t h = 0;
    std::vector<float> p(kMlpParams);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kSurMagic, 8) == 0 &&
              std::fread(&cnt, 4, 1, f) == 1 && cnt == kMlpParams &&
              std::fread(p.data(), sizeof(float), kMlpParams, f) == (size_t)kMlpParams &&
              std::fread(&h, 4, 1, f) == 1;
    char extra;
    ok = ok && std::fread(&extra, 1, 1, f) == 0;  // nothing after the hash
    std::fclose(f);
    if (!ok) return fail(MPAP_ERR_INVAL, std::string("not a surrogate parameter file: ") + path);
    if (h != fnv1a(p.data(), sizeof(float) * kMlpParams))
        return fail(MPAP_ERR_INVAL, std::string("parameter hash mismatch in ") + path);
    return mpap_surrogate_set_params(s, p.data(), kMlpParams);
}

int mpap_edge_features(const mpap_graph *gc, void *stream, uint16_t *out, int64_t capacity,
                       float *base) {
    if (!gc) return fail(MPAP_ERR_INVAL, "null graph");
    mpap_graph *g = const_cast<mpap_graph *>(gc);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int r;
    if ((r = ensure_features(g, st))) return r;
    if (out) {
        if (capacity < g->e * kMlpIn) return fail(MPAP_ERR_CAPACITY, "capacity below 16 * edges");
        HIP_TRY(hipMemcpy(out, g->feat, sizeof(uint16_t) * kMlpIn * g->e, hipMemcpyDeviceToHost));
    }
    if (base && g->e > 0)
        HIP_TRY(hipMemcpy(base, g->sbase, sizeof(float) * g->e, hipMemcpyDeviceToHost));
    return MPAP_OK;
}

int mpap_surrogate_forward(const mpap_surrogate *s, const uint16_t *X, int64_t n, float *y) {
    if (!s || (n > 0 && (!X || !y)) || n < 0) return fail(MPAP_ERR_INVAL, "null argument");
    if (n == 0) return MPAP_OK;
    uint16_t *dX = nullptr;
    float *dy = nullptr;
    int r;
    if ((r = dalloc(&dX, (size_t)n * kMlpIn)) || (r = dalloc(&dy, n))) {
        dfree(dX);
        return r;
    }
    hipError_t he = hipMemcpy(dX, X, sizeof(uint16_t) * kMlpIn * n, hipMemcpyHostToDevice);
    if (he == hipSuccess) {
        const int blocks = std::max(1, std::min(div_up(n, 128), 1024));
        k_mlp_infer<<<blocks, 256>>>(dev_view(s), dX, n, nullptr, nullptr, dy, nullptr);
        he = hipGetLastError();
    }
    if (he == hipSuccess) he = hipMemcpy(y, dy, sizeof(float) * n, hipMemcpyDeviceToHost);
    dfree(dX);
    dfree(dy);
    if (he != hipSuccess) return fail(MPAP_ERR_HIP, hipGetErrorString(he));
    return MPAP_OK;
}

int mpap_surrogate_gradient(mpap_surrogate *s, const uint16_t *X, const float *t, int32_t n,
                            float *grad, float *y_out) {
    if (!s || !X || !t || !grad) return fail(MPAP_ERR_INVAL, "null argument");
    int r;
    if ((r = sur_scratch(s, n))) return r;
    uint16_t *dX = nullptr;
    float *dt = nullptr;
    long long *di = nullptr;
    if ((r = dalloc(&dX, (size_t)n * kMlpIn)) || (r = dalloc(&dt, n)) || (r = dalloc(&di, n))) {
        dfree(dX); dfree(dt);
        return r;
    }
    std::vector<long long> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    hipError_t he = hipMemcpy(dX, X, sizeof(uint16_t) * kMlpIn * n, hipMemcpyHostToDevice);
    if (he == hipSuccess) he = hipMemcpy(dt, t, sizeof(float) * n, hipMemcpyHostToDevice);
    if (he == hipSuccess) he = hipMemcpy(di, idx.data(), sizeof(long long) * n, hipMemcpyHostToDevice);
    if (he == hipSuccess) {
        r = sur_batch(s, dX, dt, di, 0.f, false, s->grad, nullptr);
        if (r == MPAP_OK) {
            he = hipMemcpy(grad, s->grad, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost);
            if (he == hipSuccess && y_out) he = hipMemcpy(y_out, s->y, sizeof(float) * n, hipMemcpyDeviceToHost);
        }
    }
    dfree(dX); dfree(dt); dfree(di);
    if (r) return r;
    if (he != hipSuccess) return fail(MPAP_ERR_HIP, hipGetErrorString(he));
    return MPAP_OK;
}

int mpap_surrogate_train(mpap_surrogate *s, const mpap_graph *gc, const int64_t *edges,
                         int64_t n_train, int32_t epochs, int32_t batch, float lr, void *stream,
                         float *epoch_loss) {
    if (!s || !gc || !edges || n_train < 1 || epochs < 0 || !(lr > 0.f))
        return fail(MPAP_ERR_INVAL, "bad argument");
    mpap_graph *g = const_cast<mpap_graph *>(gc);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    for (int64_t i = 0; i < n_train; ++i)
        if (edges[i] < 0 || edges[i] >= g->e) return fail(MPAP_ERR_INVAL, "edge index out of range");
    int r;
    if ((r = sur_scratch(s, batch))) return r;
    if (n_train < batch) return fail(MPAP_ERR_INVAL, "fewer training edges than one batch");
    if ((r = ensure_features(g, st))) return r;
    if (g->e > s->t_cap) {
        dfree(s->t_all);
        if ((r = dalloc(&s->t_all, g->e))) return r;
        s->t_cap = g->e;
    }
    if (n_train > s->idx_cap) {
        dfree(s->idx);
        if ((r = dalloc(&s->idx, n_train))) return r;
        s->idx_cap = n_train;
    }
    k_drift_ratio<<<div_up(g->e, 256), 256, 0, st>>>(g->e, g->odrift, drift_length(g), g->sbase,
                                                     kResidualScale, s->t_all);
    HIP_TRY(hipMemcpyAsync(s->idx, edges, sizeof(long long) * n_train, hipMemcpyHostToDevice, st));
    const long long steps = n_train / batch;
    const double total = std::max<double>(1.0, (double)steps * epochs);
    for (int ep = 0; ep < epochs; ++ep) {
        for (long long k = 0; k < steps; ++k) {
            // cosine decay from lr to lr/100 over the whole run
            const double f = ((double)ep * steps + k) / total;
            const float lr_k = (float)(lr * (0.01 + 0.99 * 0.5 * (1.0 + std::cos(3.141592653589793 * f))));
            if ((r = sur_batch(s, g->feat, s->t_all, s->idx + k * batch, lr_k, true, nullptr, st)))
                return r;
        }
        if (epoch_loss) {
            // mean squared error of the updated network over the training edges
            float *yall = nullptr;
            if ((r = dalloc(&yall, g->e))) return r;
            const int blocks = std::max(1, std::min(div_up(g->e, 128), 2048));
            k_mlp_infer<<<blocks, 256, 0, st>>>(dev_view(s), g->feat, g->e, nullptr, nullptr,
                                                yall, nullptr);
            k_zero_f32<<<1, 64, 0, st>>>(s->sq, 1);
            k_sq_err<<<std::max(1, std::min(div_up(n_train, 256), 1024)), 256, 0, st>>>(
                yall, s->t_all, s->idx, n_train, s->sq);
            float sum = 0.f;
            HIP_TRY(hipMemcpyAsync(&sum, s->sq, sizeof(float), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            epoch_loss[ep] = sum / (float)n_train;
            dfree(yall);
        }
    }
    HIP_TRY(hipStreamSynchronize(st));
    return MPAP_OK;
}

int mpap_surrogate_score(const mpap_surrogate *s, mpap_graph *g, void *stream, float *ms) {
    if (!s || !g) return fail(MPAP_ERR_INVAL, "null argument");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int r;
    if (!g->sdrift && (r = dalloc(&g->sdrift, std::max<long long>(g->e, 1)))) return r;
    if (!g->symmetric_alias && !g->srdrift && (r = dalloc(&g->srdrift, std::max<long long>(g->e, 1))))
        return r;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, st));
    r = sur_enqueue_score(s, g, g->sdrift, st);
    if (r == MPAP_OK) {
        HIP_TRY(hipEventRecord(e1, st));
        HIP_TRY(hipEventSynchronize(e1));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, e0, e1));
        if (ms) *ms = t;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return r;
}

int mpap_analytic_drift(mpap_graph *g, void *stream, float *ms) {
    if (!g) return fail(MPAP_ERR_INVAL, "null graph");
    if (!g->pos) return fail(MPAP_ERR_INVAL, "graph has no environment (build it with mpap_build_graph)");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, st));
    int r = enqueue_analytic_drift(g, g->odrift, st);
    if (r == MPAP_OK) {
        HIP_TRY(hipEventRecord(e1, st));
        HIP_TRY(hipEventSynchronize(e1));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, e0, e1));
        if (ms) *ms = t;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return r;
}

int mpap_graph_drift(const mpap_graph *g, int32_t which, float *out) {
    if (!g || !out || (which != 0 && which != 1)) return fail(MPAP_ERR_INVAL, "bad argument");
    const float *src = which == 0 ? g->odrift : g->sdrift;
    if (!src) return fail(MPAP_ERR_INVAL, "no surrogate drift on this graph");
    if (g->e > 0) HIP_TRY(hipMemcpy(out, src, sizeof(float) * g->e, hipMemcpyDeviceToHost));
    return MPAP_OK;
}

}  // extern "C"

int sur_enqueue_score(const mpap_surrogate *s, mpap_graph *g, float *out, hipStream_t st) {
    if (!s || !g) return fail(MPAP_ERR_INVAL, "null argument");
    if (!out) return fail(MPAP_ERR_INVAL, "no drift array to score into");
    // the inputs are part of the cost of scoring a roadmap: recompute them
    int r = enqueue_features(g, st);
    if (r) return r;
    if (g->e > 0) {
        const int blocks = std::max(1, std::min(div_up(g->e, 128), 2048));
        k_mlp_infer<<<blocks, 256, 0, st>>>(dev_view(s), g->feat, g->e, drift_length(g), g->sbase,
                                            nullptr, out);
        if (!g->symmetric_alias && out == g->sdrift) {
            // in-edge order for the search of a directed roadmap
            k_gather_f32<<<div_up(g->e, 256), 256, 0, st>>>(g->e, g->rperm, g->sdrift, g->srdrift);
        }
    }
    HIP_TRY(hipGetLastError());
    return MPAP_OK;
}

int enqueue_analytic_drift(const mpap_graph *g, float *out, hipStream_t st) {
    if (!g || !out) return fail(MPAP_ERR_INVAL, "null argument");
    if (!g->pos) return fail(MPAP_ERR_INVAL, "graph has no environment (build it with mpap_build_graph)");
    if (g->n > 0 && g->dim == 6) {
        k_traj_drift<<<g->n, 64, sizeof(float) * 5 * (size_t)g->nblob, st>>>(
            steer_view(g), g->optr, g->ocol, out, nullptr);
    } else if (g->n > 0 && g->e > 0) {
        BuildArgs a{};
        a.n = g->n; a.dim = g->dim; a.pos = g->pos; a.nblob = g->nblob; a.mu = g->bmu;
        a.sig = g->bsig; a.amp = g->bamp; a.r = g->radius; a.step = g->check_step;
        a.reset_q = g->reset_q;
        const size_t lds = sizeof(float) * ((size_t)g->nblob * g->dim + 2 * (size_t)g->nblob);
        if (g->uptr)
            k_edge_drift_pairs<<<div_up(g->e / 2 + 1, 256), 256, lds, st>>>(
                a, g->n, g->optr, g->ocol, g->ocost, g->uptr, out);
        else
            k_edge_drift<<<div_up(g->e, 256), 256, lds, st>>>(a, g->n, g->optr, g->ocol,
                                                              g->ocost, out);
    }
    HIP_TRY(hipGetLastError());
    return MPAP_OK;
}
