// Internal host-runtime state shared by the C ABI implementation files.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "graph_kernels.h"
#include "mpap.h"
#include "search_kernels.h"

// ------------------------------------------------------------- error state
extern thread_local std::string g_last_error;

inline int fail(int status, const std::string &msg) {
    g_last_error = msg;
    return status;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(e_ == hipErrorOutOfMemory ? MPAP_ERR_NOMEM : MPAP_ERR_HIP,      \
                        std::string(#expr) + ": " + hipGetErrorString(e_));             \
    } while (0)

struct DeviceInfo {
    int dev = -1;
    int cus = 0;
    int coop = 0;
    size_t max_lds = 0;
};

inline int device_info(DeviceInfo *out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(MPAP_ERR_DEVICE, std::string("libmpap is built for gfx950, device is ") +
                                         prop.gcnArchName);
    out->dev = dev;
    out->cus = prop.multiProcessorCount;
    int coop = 0;
    HIP_TRY(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    out->coop = coop;
    out->max_lds = prop.sharedMemPerBlock;
    if (!coop) return fail(MPAP_ERR_DEVICE, "device does not support cooperative launches");
    return MPAP_OK;
}

template <typename T>
inline int dalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    HIP_TRY(hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T)));
    return MPAP_OK;
}

template <typename T>
inline void dfree(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

inline int div_up(long long a, long long b) { return (int)((a + b - 1) / b); }

constexpr int kTraceCap = 4096;  // waves recorded in the per-wave trace

// exclusive scan of n int32 (device); tmp holds >= div_up(n, kScanTile) ints
inline int scan_i32(const int *in, int *out, long long n, int *tmp, hipStream_t s) {
    if (n <= 0) return MPAP_OK;
    const int nb = div_up(n, kScanTile);
    k_scan_block_sums<<<nb, 256, 0, s>>>(in, n, tmp);
    k_scan_sums<<<1, 1024, 0, s>>>(tmp, nb);
    k_scan_apply<<<nb, 256, 0, s>>>(in, n, tmp, out);
    HIP_TRY(hipGetLastError());
    return MPAP_OK;
}


// ------------------------------------------------------------------ graph
struct Workspace;

struct mpap_graph {
    int dev = -1;
    int32_t n = 0;
    int64_t e = 0;
    int32_t n_goal = 0;
    bool symmetric_alias = false;  // in-edge arrays alias the out-edge ones
    // forward CSR
    int32_t *optr = nullptr, *ocol = nullptr;
    float *ocost = nullptr, *odrift = nullptr;
    // reverse CSR (in-edges)
    int32_t *rptr = nullptr, *rsrc = nullptr;
    float *rcost = nullptr, *rdrift = nullptr;
    uint8_t *nflag = nullptr;
    int32_t *goal_list = nullptr;
    // query partition: query q owns nodes [qoff[q], qoff[q+1]) and goal list
    // entries [qgoff[q], qgoff[q+1]); a plain roadmap is one query
    int32_t nq = 1;
    std::vector<int32_t> qoff_h, qgoff_h;
    int32_t *qoff = nullptr, *qgoff = nullptr;
    // environment of a roadmap built by mpap_build_graph (inputs of the
    // surrogate's features); absent for imported and concatenated graphs
    int dim = 0, nbox = 0, nblob = 0;
    float check_step = 0.f, reset_q = 0.f, radius = 0.f;
    float *pos = nullptr, *bmu = nullptr, *bsig = nullptr, *bamp = nullptr;
    float *blo = nullptr, *bhi = nullptr;  // obstacle boxes [nbox][w] (closed), w = 3 for dim 6
    // double integrator (dim 6): velocities, steering time, check steps, and
    // the trajectory length of every edge (the drift's length)
    float *vel = nullptr, *elen = nullptr;
    float horizon = 0.f;
    int traj_steps = 0, k_out = 0;
    // directed roadmaps: reverse slot -> forward edge index, and the
    // surrogate drift in reverse order
    int32_t *rperm = nullptr;
    float *srdrift = nullptr;
    uint16_t *feat = nullptr;  // [E][16] bf16 surrogate inputs, computed on demand
    float *sbase = nullptr;    // [E] 8-point estimate of the mean of (1 - q) per edge
    float *sdrift = nullptr;   // [E] surrogate drift (forward edge order)
    // symmetric roadmaps with an environment: uptr[u] = entries v > u in the
    // rows before u ([n+1]; uptr[n] id-ordered pairs), so the per-edge inputs
    // and drifts are evaluated once per pair
    int32_t *uptr = nullptr;
    std::vector<Workspace *> spare;
    std::mutex mu;
};

// g->uptr of a symmetric roadmap (rows sorted by target id); synchronises s
int build_pair_index(mpap_graph *g, hipStream_t s);

inline int graph_set_single_query(mpap_graph *g) {
    g->nq = 1;
    g->qoff_h = {0, g->n};
    g->qgoff_h = {0, g->n_goal};
    int r;
    if ((r = dalloc(&g->qoff, 2)) || (r = dalloc(&g->qgoff, 2))) return r;
    HIP_TRY(hipMemcpy(g->qoff, g->qoff_h.data(), 2 * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(g->qgoff, g->qgoff_h.data(), 2 * sizeof(int32_t), hipMemcpyHostToDevice));
    return MPAP_OK;
}

void graph_release(mpap_graph *g);

// ------------------------------------------------------------- workspace
struct Workspace {
    int32_t n = 0;
    unsigned long long pool_cap = 0;
    long long arena_cap = 0, F_cap = 0;
    int nblocks = 0;
    long long goal_cap = 0;
    float4 *pool = nullptr;
    unsigned *pool_top = nullptr;
    int4 *nb = nullptr;
    float *minopen = nullptr;
    int *gcnt = nullptr;
    int4 *fo = nullptr;
    int *mark = nullptr;
    int *wt = nullptr;
    int *alist = nullptr;
    int *acnt = nullptr;
    int *mcur = nullptr;
    float4 *F = nullptr;
    int2 *arena = nullptr;
    long long *part_cnt = nullptr, *part_open = nullptr;
    long long *part_step = nullptr;
    unsigned *bar = nullptr;
    int *err = nullptr;
    long long *out = nullptr;
    long long *wstat = nullptr;
    float4 *spill = nullptr;
    uint8_t *spill_flags = nullptr;
    long long spill_cap = 0;  // capG the spill space was sized for
    // per query
    int nq_cap = 0;
    float *qbeta = nullptr;
    int *qnobj = nullptr, *qroot = nullptr, *qlast = nullptr, *qheur = nullptr;
    int *qearly = nullptr, *qstop = nullptr;
    float *qdelta = nullptr;
    long long *g_laboff = nullptr;
    int *g_labcap = nullptr;
    int *g_overflow = nullptr;
    // goal front: per-query regions, then packed densely in query order
    float4 *g_out = nullptr;
    int *g_out_node = nullptr, *g_n = nullptr, *g_count = nullptr;
    long long *g_total = nullptr;
    float4 *p_lab = nullptr;
    int *p_node = nullptr;
    long long p_cap = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // pinned host staging of the small uploads and read-backs of a search
    // (asynchronous copies without the runtime's pageable bounce); its bytes
    // are in use until the stream has passed the copies that name them
    unsigned char *hpin = nullptr;
    size_t hpin_cap = 0;

    void free_all() {
        dfree(pool); dfree(pool_top); dfree(nb); dfree(minopen); dfree(gcnt); dfree(fo);
        dfree(mark); dfree(wt); dfree(alist); dfree(acnt); dfree(mcur); dfree(F); dfree(arena); dfree(part_cnt);
        dfree(part_open); dfree(part_step); dfree(bar); dfree(err); dfree(out); dfree(wstat);
        dfree(spill); dfree(spill_flags);
        dfree(g_out); dfree(g_out_node); dfree(g_n); dfree(g_count); dfree(g_total);
        dfree(p_lab); dfree(p_node);
        dfree(qbeta); dfree(qnobj); dfree(qroot); dfree(qlast); dfree(qheur); dfree(qdelta);
        dfree(qearly); dfree(qstop);
        dfree(g_laboff);
        dfree(g_labcap); dfree(g_overflow);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        ev0 = ev1 = nullptr;
        if (hpin) (void)hipHostFree(hpin);
        hpin = nullptr;
        hpin_cap = 0;
    }
};

// At least `bytes` of pinned staging (the stream must have passed every copy
// that uses the old buffer).
inline int ws_pinned(Workspace *w, size_t bytes) {
    if (bytes <= w->hpin_cap) return MPAP_OK;
    size_t cap = std::max<size_t>(bytes, 64 * 1024);
    if (w->hpin) (void)hipHostFree(w->hpin);
    w->hpin = nullptr;
    w->hpin_cap = 0;
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&w->hpin), cap, hipHostMallocDefault));
    w->hpin_cap = cap;
    return MPAP_OK;
}

inline int ws_alloc_nodes(Workspace *w, int32_t n, int nblocks) {
    int r;
    w->n = n;
    w->nblocks = nblocks;
    if ((r = dalloc(&w->pool_top, 1))) return r;
    if ((r = dalloc(&w->nb, n))) return r;
    if ((r = dalloc(&w->minopen, n))) return r;
    if ((r = dalloc(&w->gcnt, n))) return r;
    if ((r = dalloc(&w->fo, n))) return r;
    if ((r = dalloc(&w->mark, n))) return r;
    if ((r = dalloc(&w->wt, n))) return r;
    if ((r = dalloc(&w->alist, (size_t)kListRegions * n))) return r;
    if ((r = dalloc(&w->acnt, 2 * kListRegions))) return r;
    if ((r = dalloc(&w->mcur, 2 * kListRegions))) return r;
    if ((r = dalloc(&w->part_cnt, 2 * (size_t)nblocks))) return r;
    if ((r = dalloc(&w->part_open, 2 * (size_t)nblocks))) return r;
    if ((r = dalloc(&w->part_step, 2 * (size_t)nblocks))) return r;
    if ((r = dalloc(&w->bar, 1))) return r;
    if ((r = dalloc(&w->err, 1))) return r;
    if ((r = dalloc(&w->out, kOutWords))) return r;
    if ((r = dalloc(&w->wstat, (size_t)kTraceCap * kTraceWords))) return r;
    if ((r = dalloc(&w->g_total, 1))) return r;
    HIP_TRY(hipEventCreate(&w->ev0));
    HIP_TRY(hipEventCreate(&w->ev1));
    return MPAP_OK;
}

inline int ws_queries(Workspace *w, int nq) {
    if (nq <= w->nq_cap) return MPAP_OK;
    int r;
    dfree(w->qbeta); dfree(w->qnobj); dfree(w->qroot); dfree(w->qlast); dfree(w->g_laboff);
    dfree(w->g_labcap); dfree(w->g_n); dfree(w->g_count); dfree(w->qheur); dfree(w->qdelta);
    dfree(w->qearly); dfree(w->qstop);
    if ((r = dalloc(&w->qbeta, nq)) || (r = dalloc(&w->qnobj, nq)) || (r = dalloc(&w->qheur, nq)) ||
        (r = dalloc(&w->qearly, nq)) || (r = dalloc(&w->qstop, nq)) ||
        (r = dalloc(&w->qdelta, nq)) ||
        (r = dalloc(&w->qroot, nq)) || (r = dalloc(&w->qlast, nq)) ||
        (r = dalloc(&w->g_laboff, nq)) || (r = dalloc(&w->g_labcap, nq)) ||
        (r = dalloc(&w->g_n, nq)) || (r = dalloc(&w->g_count, nq)))
        return r;
    if (!w->g_overflow && (r = dalloc(&w->g_overflow, 1))) return r;
    w->nq_cap = nq;
    return MPAP_OK;
}

inline int ws_spill(Workspace *w, long long capG) {
    if (capG <= w->spill_cap) return MPAP_OK;
    int r;
    dfree(w->spill);
    dfree(w->spill_flags);
    w->spill_cap = 0;
    if ((r = dalloc(&w->spill, (size_t)w->nblocks * 2 * capG)) ||
        (r = dalloc(&w->spill_flags, (size_t)w->nblocks * capG)))
        return r;
    w->spill_cap = capG;
    return MPAP_OK;
}

inline int ws_grow(Workspace *w, unsigned long long pool_cap, long long arena_cap,
                   long long F_cap, long long goal_cap) {
    int r;
    if (pool_cap > w->pool_cap) {
        dfree(w->pool);
        if ((r = dalloc(&w->pool, pool_cap))) return r;
        w->pool_cap = pool_cap;
    }
    if (arena_cap > w->arena_cap) {
        dfree(w->arena);
        if ((r = dalloc(&w->arena, arena_cap))) return r;
        w->arena_cap = arena_cap;
    }
    if (F_cap > w->F_cap) {
        dfree(w->F);
        if ((r = dalloc(&w->F, F_cap))) return r;
        w->F_cap = F_cap;
    }
    if (goal_cap > w->goal_cap) {
        dfree(w->g_out); dfree(w->g_out_node);
        if ((r = dalloc(&w->g_out, goal_cap))) return r;
        if ((r = dalloc(&w->g_out_node, goal_cap))) return r;
        w->goal_cap = goal_cap;
    }
    return MPAP_OK;
}

inline int ws_pack(Workspace *w, long long cap) {
    if (cap <= w->p_cap) return MPAP_OK;
    int r;
    dfree(w->p_lab);
    dfree(w->p_node);
    w->p_cap = 0;
    if ((r = dalloc(&w->p_lab, cap)) || (r = dalloc(&w->p_node, cap))) return r;
    w->p_cap = cap;
    return MPAP_OK;
}

// ------------------------------------------------------------------ result
struct mpap_result {
    mpap_graph *g = nullptr;
    Workspace *ws = nullptr;
    int n_obj = 2;
    std::vector<float> qbeta;   // per-query bound
    std::vector<int> qnobj;     // per-query objective count
    std::vector<int> qheur;     // per-query heuristic (0 analytic, 1 surrogate)
    std::vector<int> qearly;    // per-query early stop of Alg. 3's loop condition (0/1)
    std::vector<int> qstop;     // per query: groups expanded before the early stop, -1 none
    // goal fronts of all queries, query q at [front_off[q], front_off[q+1])
    std::vector<float4> front;
    std::vector<int32_t> front_node;
    std::vector<int64_t> front_off;
    std::vector<int32_t> qlast;      // last wave that expanded a label of the query
    std::vector<float> qlatency_ms;  // device time from launch start to that wave's end
    std::vector<int64_t> trace;
    mpap_stats stats{};
    long long arena_labels = 0;  // arena size: expanded labels + goal plans closed at a stop
    unsigned long long pool_used = 0;  // bucket pool slots in use when the search ended
    long long reused_arena = 0;  // an update: arena ids taken over from the earlier result
    // an update: arena id where each expanded group starts (earlier results'
    // groups first), and the arena size last; empty for a plain search (its
    // trace has the group sizes)
    std::vector<long long> group_start;
    std::vector<int2> arena_host;  // filled on first mpap_label_path
    bool arena_loaded = false;
    bool ws_borrowed = false;  // ws belongs to a plan (valid until its next run)
    // the parameters the search ran with (the judge's fallback re-search uses them)
    std::vector<float> qdelta;
    std::vector<int> qroot;
    int max_waves = 0, near_scan = 16, stage_cap = 0, block_threads = 1024;
    int wave_min_targets = 0, merge_halves = 0;
    // judge of a search on the learned drift: queries whose front it rejected
    // are answered by an analytic re-search (fallback), whose label ids are
    // reported shifted by id_offset
    bool judged = false;
    mpap_result *fallback = nullptr;
    std::vector<uint8_t> qfall;
    long long id_offset = 0;
};

// ------------------------------------------------------ search preparation
// Validated per-query parameters of one batched search.
struct SearchPrep {
    int nq = 0;
    std::vector<float> delta;  // per query lambda * radius
    int max_waves = 0, near_scan = 16, stage_cap = 0, block_threads = 1024;
    int wave_min_targets = 0;  // 0: default; < 0: never merge by single waves
    int merge_halves = 0;      // 0: by halves on large roadmaps; > 0: always (the children
                               // threshold of whole-workgroup targets); < 0: never
    std::vector<float> beta;
    std::vector<int> nobj, root, heur;
    std::vector<int> skip;  // 1: the query is not searched (its root is not seeded)
    std::vector<int> early; // 1: Alg. 3's early stop (loop ends at a group with a goal plan)
    bool early_any = false;
};
// Launch shape of the persistent search kernel.
struct SearchShape {
    int threads = 1024, capC = 1024, capB = 0, nblocks = 0;
    int wcap = 0, wslice = 0;  // single-wave merges: front capacity, LDS slice bytes
    int wmin = 0;              // and the least small-target count that uses them
    bool explicit_wmin = false;
    // merges by halves (1024-thread workgroups, workgroup-only build): each
    // half's LDS bytes, front stage and chunk; fronts above big_front labels
    // or targets with more than big_children children go to the whole workgroup
    int halves = 0, half_lds = 0, capBh = 0, capCh = 0, big_front = 0, big_children = 0;
    int halves_min = 0;  // least targets of an iteration that merges by halves
    bool halves_forced = false;  // the halves build whatever the roadmap's size
    int obj = 0;  // 2 or 3: every query has that many objectives (a build for it); 0: mixed
    size_t lds = 0;
};
int search_prep(const mpap_graph *g, const mpap_search_params *sp, int32_t nsp, SearchPrep &p);
int search_shape(int stage_cap, int block_threads, int wave_min_targets, SearchShape &L,
                 int merge_halves = 0);
// Uploads the per-query parameters into w (synchronous).
int search_upload(Workspace *w, const SearchPrep &p, hipStream_t s);
// The search with capacity growth and retries, goal fronts and statistics,
// eagerly on stream s into res (whose ws is w).
int search_eager(mpap_graph *g, const SearchPrep &p, const SearchShape &L, Workspace *w,
                 hipStream_t s, mpap_result *res);
SearchArgs search_args(const mpap_graph *g, Workspace *w, const SearchPrep &p,
                       const SearchShape &L);
// After a successful search launch with arguments a (device status words in
// dev_out): goal fronts, host copies and statistics into res.
// total: the goal-front bound k_goal_bound already wrote to w->g_total (read
// back by the caller), or -1 (this function runs k_goal_bound).
int search_goal_finish(mpap_graph *g, const SearchPrep &p, const SearchShape &L, Workspace *w,
                       hipStream_t s, mpap_result *res, const SearchArgs &a,
                       const long long *dev_out, float ms, int retries, long long total = -1);
// A search workspace of g for launch shape L (a spare one when it fits).
int acquire_workspace(mpap_graph *g, const SearchShape &L, Workspace **out);
GoalArgs goal_args(const mpap_graph *g, Workspace *w);
// The search kernel build for a launch on g: with single-wave merges only
// when some iteration can have wmin targets (or the caller asked for them).
// The build with merges by halves runs on roadmaps of at least 16 nodes per
// workgroup (smaller ones rarely have iterations with enough targets), or
// when the caller asked for it.
inline bool halves_build(const SearchShape &L, int n) {
    return L.halves && (L.halves_forced || n >= 16 * (long long)L.nblocks);
}
inline bool wave_build(const SearchShape &L, int n) {
    return L.wcap > 0 && (L.explicit_wmin || n >= 4 * (long long)L.wmin);
}
// The search build for a launch on g (see search_kernels.h).
inline const void *search_kernel_for(const SearchShape &L, int n) {
    const void *k;
    if (wave_build(L, n))
        k = L.obj == 2 ? reinterpret_cast<const void *>(k_search_wave_o2)
                       : reinterpret_cast<const void *>(k_search_wave);
    else if (halves_build(L, n))
        k = L.obj == 2   ? reinterpret_cast<const void *>(k_search_halves_o2)
            : L.obj == 3 ? reinterpret_cast<const void *>(k_search_halves_o3)
                         : reinterpret_cast<const void *>(k_search_halves);
    else
        k = L.obj == 2   ? reinterpret_cast<const void *>(k_search_o2)
            : L.obj == 3 ? reinterpret_cast<const void *>(k_search_o3)
                         : reinterpret_cast<const void *>(k_search);
    return k;
}
// 2 or 3 when every searched query of p has that many objectives, else 0
inline int uniform_objectives(const SearchPrep &p) {
    int o = -1;
    for (int q = 0; q < p.nq; ++q) {
        if (q < (int)p.skip.size() && p.skip[q]) continue;
        if (o < 0) o = p.nobj[q];
        else if (o != p.nobj[q]) return 0;
    }
    return o == 2 || o == 3 ? o : 0;
}

// Fills res's fronts, statistics, trace and latencies from host copies.
void search_finish(mpap_result *res, const SearchPrep &p, const long long *dev_out,
                   const int *counts, const float4 *plab, const int *pnode, const int *qlast,
                   const int *qstop, const long long *trace, float ms, int retries,
                   const SearchShape &L);

// Surrogate scoring of one roadmap (features, then inference) enqueued on a
// stream, writing the drift to out[e]; used by plans and mpap_surrogate_score.
struct mpap_surrogate;
int sur_enqueue_score(const mpap_surrogate *s, mpap_graph *g, float *out, hipStream_t st);
// The analytic drift of every edge of g (built by mpap_build_graph) enqueued
// on a stream, written to out[e] (forward edge order).
int enqueue_analytic_drift(const mpap_graph *g, float *out, hipStream_t st);

