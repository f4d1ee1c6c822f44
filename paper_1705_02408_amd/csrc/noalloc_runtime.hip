// mpap_search_noalloc: the search of one roadmap (Alg. 3 until no plan is
// open, goal front of Alg. 3's P_candidates) with every piece of device state
// in one fixed, file-scope scratch array instead of memory from hipMalloc.
//
// For callers that cannot allocate device memory.  The scratch array is
// kNoAllocScratchBytes per device, held from the first load of the library on
// that device until the process ends; every call on a device reuses it and
// leaves the last call's contents behind, so everything a search reads before
// writing is cleared on the stream first (k_search_init, the goal counters).
// Two calls that overlap on one device (other streams, other threads) race on
// the same memory: callers serialise them.
#include "runtime_internal.h"

namespace {

constexpr size_t kNoAllocScratchBytes = 64ull << 20;  // 64 MiB per device
constexpr int kNoAllocMaxDevices = 64;

}  // namespace

// Device state of mpap_search_noalloc.  Host code never passes this name to a
// kernel or a copy: it uses the address hipGetSymbolAddress gives per device.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

std::mutex g_scratch_mu;
unsigned char *g_scratch_dev[kNoAllocMaxDevices];  // device address of scratch per device

// The scratch array's address on the current device (looked up once per
// device, with that device current).
int scratch_address(int dev, unsigned char **out) {
    *out = nullptr;
    if (dev < 0 || dev >= kNoAllocMaxDevices)
        return fail(MPAP_ERR_DEVICE, "device index beyond the no-allocation table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(MPAP_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                          hipGetErrorString(e));
        g_scratch_dev[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_dev[dev];
    return MPAP_OK;
}

// Bump carving of the scratch array (256-byte aligned pieces).  A piece that
// does not fit marks the carving failed for good (every later piece is null).
struct Carver {
    unsigned char *base;
    size_t off, cap;
    bool bad = false;
    template <typename T>
    T *take(size_t count) {
        const size_t o = (off + 255) & ~size_t(255);
        const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        if (bad || o > cap || bytes > cap - o) {
            bad = true;
            return nullptr;
        }
        off = o + bytes;
        return reinterpret_cast<T *>(base + o);
    }
    size_t left() const {
        const size_t o = (off + 255) & ~size_t(255);
        return (!bad && o < cap) ? cap - o : 0;
    }
};

// The one query's parameters, written on the device (no host staging copy).
__global__ void k_noalloc_query(float *qbeta, int *qnobj, int *qroot, int *qheur,
                                float *qdelta, int *qlast, int *qearly, float beta, int nobj,
                                int root, int heur, float delta, int early) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        qbeta[0] = beta;
        qnobj[0] = nobj;
        qroot[0] = root;
        qheur[0] = heur;
        qdelta[0] = delta;
        qlast[0] = 0;
        qearly[0] = early;
    }
}

// The goal front (query 0, region at offset 0) split into per-objective
// arrays for the copies to the caller.
__global__ void k_noalloc_unpack(const float4 *lab, const int *node, const int *count,
                                 float *c, float *d, float *m, int *gn) {
    const int k = *count;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
        const float4 L = lab[i];
        c[i] = L.x;
        d[i] = L.y;
        m[i] = L.z;
        gn[i] = node[i];
    }
}

}  // namespace

extern "C" int mpap_search_noalloc(const mpap_graph *gc, const mpap_search_params *sp,
                                   void *stream, float *cost, float *drift, float *maxdrift,
                                   int32_t *goal_node, int32_t capacity, int32_t *count) {
    if (!gc || !sp || !count) return fail(MPAP_ERR_INVAL, "null graph, params or count");
    *count = 0;
    if (capacity < 0) return fail(MPAP_ERR_INVAL, "capacity < 0");
    mpap_graph *g = const_cast<mpap_graph *>(gc);
    if (g->nq != 1)
        return fail(MPAP_ERR_INVAL, "mpap_search_noalloc takes a single-query roadmap");
    const mpap_search_params &x = *sp;
    if (x.n_obj != 2 && x.n_obj != 3) return fail(MPAP_ERR_INVAL, "n_obj must be 2 or 3");
    if (x.init_node < 0 || x.init_node >= g->n) return fail(MPAP_ERR_INVAL, "init_node out of range");
    if (!(x.lambda > 0.0f) || !(x.radius > 0.0f) || std::isnan(x.beta))
        return fail(MPAP_ERR_INVAL, "lambda and radius must be > 0, beta not NaN");
    const float delta = x.lambda * x.radius;
    if (!(delta > 0.0f) || !std::isfinite(delta))
        return fail(MPAP_ERR_INVAL, "lambda * radius must be finite and > 0");
    if (x.heuristic != 0 && x.heuristic != 1)
        return fail(MPAP_ERR_INVAL, "heuristic must be 0 (analytic) or 1 (surrogate)");
    if (x.heuristic == 1 && !(g->symmetric_alias ? g->sdrift : g->srdrift))
        return fail(MPAP_ERR_INVAL, "no surrogate drift on this graph (mpap_surrogate_score)");
    if (x.block_threads != 0 && x.block_threads != 256 && x.block_threads != 512 &&
        x.block_threads != 1024)
        return fail(MPAP_ERR_INVAL, "block_threads must be 0, 256, 512 or 1024");
    if (x.skip != 0) return fail(MPAP_ERR_INVAL, "skip must be 0 for a single search");
    if (x.early_stop != 0 && x.early_stop != 1)
        return fail(MPAP_ERR_INVAL, "early_stop must be 0 or 1");

    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != g->dev) return fail(MPAP_ERR_INVAL, "the graph lives on another device");
    unsigned char *base = nullptr;
    int r = scratch_address(dev, &base);
    if (r) return r;
    SearchShape L;
    if ((r = search_shape(x.stage_cap > 0 ? x.stage_cap : 0,
                          x.block_threads ? x.block_threads : 1024, x.wave_min_targets, L,
                          x.merge_halves)))
        return r;
    L.obj = x.n_obj == 2 || x.n_obj == 3 ? x.n_obj : 0;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    // carve: per-node state, fixed words, then the label stores.  No spill
    // space: a front beyond the LDS stage is reported as an overflow.
    const int32_t n = g->n;
    Carver cv{base, 0, kNoAllocScratchBytes};
    Workspace w;  // pointers into the scratch array only (never freed)
    w.n = n;
    w.nblocks = L.nblocks;
    w.nb = cv.take<int4>(n);
    w.fo = cv.take<int4>(n);
    w.minopen = cv.take<float>(n);
    w.gcnt = cv.take<int>(n);
    w.mark = cv.take<int>(n);
    w.wt = cv.take<int>(n);
    w.alist = cv.take<int>((size_t)kListRegions * n);
    w.acnt = cv.take<int>(2 * kListRegions);
    w.mcur = cv.take<int>(2 * kListRegions);
    w.part_cnt = cv.take<long long>(2 * (size_t)L.nblocks);
    w.part_open = cv.take<long long>(2 * (size_t)L.nblocks);
    w.part_step = cv.take<long long>(2 * (size_t)L.nblocks);
    w.pool_top = cv.take<unsigned>(1);
    w.bar = cv.take<unsigned>(1);
    w.err = cv.take<int>(1);
    w.out = cv.take<long long>(kOutWords);
    w.wstat = cv.take<long long>((size_t)kTraceCap * kTraceWords);
    w.qbeta = cv.take<float>(1);
    w.qnobj = cv.take<int>(1);
    w.qroot = cv.take<int>(1);
    w.qlast = cv.take<int>(1);
    w.qheur = cv.take<int>(1);
    w.qdelta = cv.take<float>(1);
    w.qearly = cv.take<int>(1);
    w.qstop = cv.take<int>(1);
    w.g_laboff = cv.take<long long>(1);
    w.g_labcap = cv.take<int>(1);
    w.g_count = cv.take<int>(1);
    w.g_overflow = cv.take<int>(1);
    w.g_total = cv.take<long long>(1);
    w.nq_cap = 1;
    if (cv.bad || cv.left() < (size_t)4 << 20)
        return fail(MPAP_ERR_INVAL,
                    "roadmap too large for the no-allocation search: " + std::to_string(n) +
                        " nodes leave less than 4 MiB of the " +
                        std::to_string(kNoAllocScratchBytes >> 20) +
                        " MiB scratch for labels (use mpap_search)");
    // the rest: bucket pool 55 %, arena 15 %, frontier 15 %, goal front 15 %
    const size_t rest = cv.left() - 8 * 256;
    const size_t pool_n = (rest * 55 / 100) / sizeof(float4);
    const size_t arena_n = (rest * 15 / 100) / sizeof(int2);
    const size_t F_n = (rest * 15 / 100) / sizeof(float4);
    const size_t goal_n = (rest * 15 / 100) / (2 * sizeof(float4) + 2 * sizeof(int));
    w.pool = cv.take<float4>(pool_n);
    w.arena = cv.take<int2>(arena_n);
    w.F = cv.take<float4>(F_n);
    w.g_out = cv.take<float4>(goal_n);
    w.g_out_node = cv.take<int>(goal_n);
    // the caller's copy: cost, drift, max drift, goal node per label
    float *u_c = cv.take<float>(goal_n);
    float *u_d = cv.take<float>(goal_n);
    float *u_m = cv.take<float>(goal_n);
    int *u_n = cv.take<int>(goal_n);
    if (cv.bad) return fail(MPAP_ERR_HIP, "internal error: scratch carving");
    w.pool_cap = std::min<unsigned long long>(pool_n, (1ull << 31) - 1);
    w.arena_cap = (long long)arena_n;
    w.F_cap = (long long)F_n;
    w.goal_cap = (long long)goal_n;
    w.spill = nullptr;
    w.spill_flags = nullptr;
    w.spill_cap = 0;

    SearchPrep p;  // scalar fields only (search_args reads nq, max_waves, near_scan)
    p.nq = 1;
    p.max_waves = x.max_waves > 0 ? x.max_waves : 1 << 18;
    p.near_scan = x.near_scan > 0 ? x.near_scan : 16;
    p.early_any = x.early_stop != 0;
    SearchArgs a = search_args(g, &w, p, L);

    k_noalloc_query<<<1, 64, 0, s>>>(w.qbeta, w.qnobj, w.qroot, w.qheur, w.qdelta, w.qlast,
                                     w.qearly, x.beta, x.n_obj, g->qoff_h[0] + x.init_node,
                                     x.heuristic, delta, x.early_stop);
    k_search_init<<<div_up(n, 256), 256, 0, s>>>(a);
    k_search_roots<<<1, 256, 0, s>>>(a);
    HIP_TRY(hipGetLastError());
    void *kargs[] = {&a};
    HIP_TRY(hipLaunchCooperativeKernel(search_kernel_for(L, n), dim3(L.nblocks), dim3(L.threads),
                                       kargs, L.lds, s));
    if (x.early_stop) k_close_stopped<<<1, 1024, 0, s>>>(a);
    long long dev_out[kOutWords];
    int dev_err = 0;
    HIP_TRY(hipMemcpyAsync(dev_out, w.out, sizeof(dev_out), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&dev_err, w.err, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int status = (int)dev_out[kOutStatus];
    if (dev_err & kErrTimeout)
        return fail(MPAP_ERR_HIP, "a grid or half-workgroup barrier wait timed out");
    if (dev_err & kErrTarget)
        return fail(MPAP_ERR_HIP, "internal error: a queued merge target is not a node");
    if (status == kStatusNoConverge)
        return fail(MPAP_ERR_NOCONVERGE, "max_waves reached with open plans");
    if (dev_err & kErrBucket)
        return fail(MPAP_ERR_OVERFLOW, "a front outgrew the LDS stage of " +
                                           std::to_string(L.capB) +
                                           " labels (no spill space without allocation; "
                                           "use mpap_search)");
    if (dev_err & kErrPool)
        return fail(MPAP_ERR_OVERFLOW, "label pool of the no-allocation scratch exhausted "
                                       "(use mpap_search)");
    if (status == kStatusArena)
        return fail(MPAP_ERR_OVERFLOW, "label arena or group of the no-allocation scratch "
                                       "exhausted (use mpap_search)");
    if (status != kStatusOk || dev_err != 0)
        return fail(MPAP_ERR_HIP, "search reported status " + std::to_string(status));

    // goal front (a7) into the scratch, then to the caller
    GoalArgs ga = goal_args(g, &w);
    long long total = 0;
    int k = 0, ovf = 0;
    k_zero_i32<<<1, 64, 0, s>>>(w.g_count, 1);
    k_zero_i32<<<1, 64, 0, s>>>(w.g_overflow, 1);
    k_goal_bound<<<1, 1024, 0, s>>>(a, ga, (long long)goal_n, w.g_total);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(&total, w.g_total, sizeof(long long), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (total > (long long)goal_n)
        return fail(MPAP_ERR_OVERFLOW, "goal labels beyond the no-allocation scratch "
                                       "(use mpap_search)");
    if (total > 0) {
        k_goal_front<<<1, L.threads, L.lds, s>>>(a, ga);
        k_noalloc_unpack<<<std::max(1, std::min(div_up(total, 256), 64)), 256, 0, s>>>(
            w.g_out, w.g_out_node, w.g_count, u_c, u_d, u_m, u_n);
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipMemcpyAsync(&k, w.g_count, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&ovf, w.g_overflow, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&dev_err, w.err, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (ovf || dev_err) return fail(MPAP_ERR_OVERFLOW, "goal front overflow");
    *count = k;
    if (capacity < k) return fail(MPAP_ERR_CAPACITY, "capacity below the front size");
    if (k > 0) {
        if (cost) HIP_TRY(hipMemcpyAsync(cost, u_c, sizeof(float) * k, hipMemcpyDeviceToHost, s));
        if (drift) HIP_TRY(hipMemcpyAsync(drift, u_d, sizeof(float) * k, hipMemcpyDeviceToHost, s));
        if (maxdrift)
            HIP_TRY(hipMemcpyAsync(maxdrift, u_m, sizeof(float) * k, hipMemcpyDeviceToHost, s));
        if (goal_node)
            HIP_TRY(hipMemcpyAsync(goal_node, u_n, sizeof(int) * k, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    return MPAP_OK;
}
