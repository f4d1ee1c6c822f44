// Captured batches (include/mpap.h, mpap_plan_*): the surrogate scoring of
// every roadmap, the persistent search and the goal-front extraction of a
// fixed set of queries recorded once as a HIP graph and launched again with
// one call.
//
// Graph layout (all nodes in one chain):
//   [scoring: features + inference per roadmap] -> k_search_init ->
//   k_search_roots -> event -> k_search (cooperative kernel node) -> event ->
//   [k_close_stopped, with early stops] -> k_count_front -> clears ->
//   k_goal_bound -> k_goal_front -> k_goal_pack ->
//   copies of the status words, counts, packed fronts, last waves and the
//   wave trace into pinned host buffers.
// The two kernel segments are recorded by stream capture; the search kernel
// is added as an explicit node carrying the cooperative launch attribute.
// Clears inside the graph are kernels (no memset nodes).
//
// Capacities come from an eager sizing search at creation.  A launch whose
// device status reports an overflow falls back to the eager search on the
// plan's workspace (which grows it) and records the graph again.
#include "runtime_internal.h"

struct mpap_plan {
    mpap_graph *g = nullptr;
    SearchPrep prep;
    SearchShape shape;
    Workspace *w = nullptr;
    std::vector<mpap_graph *> parts;
    std::vector<const mpap_surrogate *> models;
    std::vector<long long> eoff;  // first edge of each part in the batch graph
    bool analytic = false;        // parts without a model: analytic drift recomputed
    SearchArgs args{};
    GoalArgs gargs{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // pinned host copies written by the graph
    long long *h_out = nullptr;
    int *h_err = nullptr;
    int *h_ovf = nullptr;
    int *h_count = nullptr;
    int *h_qlast = nullptr;
    int *h_qstop = nullptr;
    float4 *h_plab = nullptr;
    int *h_pnode = nullptr;
    long long *h_trace = nullptr;
    long long h_pcap = 0;
    int launches = 0, rebuilds = 0, fallbacks = 0;
};

namespace {

void host_free(void *p) {
    if (p) (void)hipHostFree(p);
}

void plan_drop_graph(mpap_plan *p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    host_free(p->h_out); host_free(p->h_err); host_free(p->h_ovf); host_free(p->h_count);
    host_free(p->h_qlast); host_free(p->h_plab); host_free(p->h_pnode); host_free(p->h_trace);
    host_free(p->h_qstop);
    p->h_qstop = nullptr;
    p->h_out = nullptr; p->h_err = nullptr; p->h_ovf = nullptr; p->h_count = nullptr;
    p->h_qlast = nullptr; p->h_plab = nullptr; p->h_pnode = nullptr; p->h_trace = nullptr;
    p->h_pcap = 0;
}

template <typename T>
int host_alloc(T **ptr, size_t count) {
    *ptr = nullptr;
    void *q = nullptr;
    HIP_TRY(hipHostMalloc(&q, sizeof(T) * std::max<size_t>(count, 1), hipHostMallocDefault));
    *ptr = static_cast<T *>(q);
    return MPAP_OK;
}

// Ends a capture on cs into *child (also on an error inside the capture).
int end_capture(hipStream_t cs, hipGraph_t *child, int status) {
    hipGraph_t gph = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &gph);
    if (status) {
        if (gph) (void)hipGraphDestroy(gph);
        return status;
    }
    if (e != hipSuccess) {
        if (gph) (void)hipGraphDestroy(gph);
        return fail(MPAP_ERR_HIP, std::string("stream capture: ") + hipGetErrorString(e));
    }
    *child = gph;
    return MPAP_OK;
}

// Records the graph for the plan's current workspace capacities.
int plan_record(mpap_plan *p) {
    plan_drop_graph(p);
    Workspace *w = p->w;
    mpap_graph *g = p->g;
    const int nq = p->prep.nq;
    int r;
    p->args = search_args(g, w, p->prep, p->shape);
    p->gargs = goal_args(g, w);
    p->h_pcap = w->p_cap;
    if ((r = host_alloc(&p->h_out, kOutWords)) || (r = host_alloc(&p->h_err, 1)) ||
        (r = host_alloc(&p->h_ovf, 1)) || (r = host_alloc(&p->h_count, nq)) ||
        (r = host_alloc(&p->h_qlast, nq)) || (r = host_alloc(&p->h_qstop, nq)) ||
        (r = host_alloc(&p->h_plab, w->p_cap)) ||
        (r = host_alloc(&p->h_pnode, w->p_cap)) ||
        (r = host_alloc(&p->h_trace, (size_t)kTraceCap * kTraceWords)))
        return r;

    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t pre = nullptr, post = nullptr;
    const SearchArgs &a = p->args;
    const GoalArgs &ga = p->gargs;
    // segment 1: scoring, state initialisation, roots
    r = MPAP_OK;
    hipError_t he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (he != hipSuccess) r = fail(MPAP_ERR_HIP, hipGetErrorString(he));
    if (!r) {
        for (size_t q = 0; q < p->models.size() && !r; ++q) {
            if (p->models[q])
                r = sur_enqueue_score(p->models[q], p->parts[q], g->sdrift + p->eoff[q], cs);
            else if (p->analytic)
                r = enqueue_analytic_drift(p->parts[q], g->odrift + p->eoff[q], cs);
        }
        if (!r) {
            k_search_init<<<div_up(g->n, 256), 256, 0, cs>>>(a);
            k_search_roots<<<div_up(nq, 256), 256, 0, cs>>>(a);
            he = hipGetLastError();
            if (he != hipSuccess) r = fail(MPAP_ERR_HIP, hipGetErrorString(he));
        }
        r = end_capture(cs, &pre, r);
    }
    // segment 2: counts, goal fronts, packing, copies to the host
    if (!r) {
        he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (he != hipSuccess) r = fail(MPAP_ERR_HIP, hipGetErrorString(he));
    }
    if (!r) {
        if (p->prep.early_any) k_close_stopped<<<1, 1024, 0, cs>>>(a);
        k_count_front<<<std::max(1, std::min(div_up(g->n, 256), 1024)), 256, 0, cs>>>(a);
        k_zero_i32<<<div_up(nq, 256), 256, 0, cs>>>(w->g_count, nq);
        k_zero_i32<<<1, 32, 0, cs>>>(w->g_overflow, 1);
        k_goal_bound<<<1, 1024, 0, cs>>>(a, ga, w->goal_cap, w->g_total);
        k_goal_front<<<std::min(nq, p->shape.nblocks), p->shape.threads, p->shape.lds, cs>>>(a, ga);
        k_goal_pack<<<std::min(nq, 1024), 256, 0, cs>>>(ga, w->p_lab, w->p_node, w->p_cap);
        he = hipGetLastError();
        const hipMemcpyKind d2h = hipMemcpyDeviceToHost;
        if (he == hipSuccess) he = hipMemcpyAsync(p->h_out, w->out, sizeof(long long) * kOutWords, d2h, cs);
        if (he == hipSuccess) he = hipMemcpyAsync(p->h_err, w->err, sizeof(int), d2h, cs);
        if (he == hipSuccess) he = hipMemcpyAsync(p->h_ovf, w->g_overflow, sizeof(int), d2h, cs);
        if (he == hipSuccess) he = hipMemcpyAsync(p->h_count, w->g_count, sizeof(int) * nq, d2h, cs);
        if (he == hipSuccess) he = hipMemcpyAsync(p->h_qlast, w->qlast, sizeof(int) * nq, d2h, cs);
        if (he == hipSuccess) he = hipMemcpyAsync(p->h_qstop, w->qstop, sizeof(int) * nq, d2h, cs);
        if (he == hipSuccess)
            he = hipMemcpyAsync(p->h_plab, w->p_lab, sizeof(float4) * w->p_cap, d2h, cs);
        if (he == hipSuccess)
            he = hipMemcpyAsync(p->h_pnode, w->p_node, sizeof(int) * w->p_cap, d2h, cs);
        if (he == hipSuccess)
            he = hipMemcpyAsync(p->h_trace, w->wstat, sizeof(long long) * kTraceCap * kTraceWords,
                                d2h, cs);
        if (he != hipSuccess) r = fail(MPAP_ERR_HIP, hipGetErrorString(he));
        r = end_capture(cs, &post, r);
    }
    (void)hipStreamDestroy(cs);
    if (r) {
        if (pre) (void)hipGraphDestroy(pre);
        return r;
    }

    // the chain: pre -> ev0 -> search -> ev1 -> post
    hipGraph_t gph = nullptr;
    he = hipGraphCreate(&gph, 0);
    hipGraphNode_t n_pre = nullptr, n_e0 = nullptr, n_s = nullptr, n_e1 = nullptr, n_post = nullptr;
    void *kargs[] = {&p->args};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void *>(search_kernel_for(p->shape, g->n));
    kp.gridDim = dim3(p->shape.nblocks);
    kp.blockDim = dim3(p->shape.threads);
    kp.sharedMemBytes = (unsigned)p->shape.lds;
    kp.kernelParams = kargs;
    kp.extra = nullptr;
    hipLaunchAttributeValue coop{};
    coop.cooperative = 1;
    if (he == hipSuccess) he = hipGraphAddChildGraphNode(&n_pre, gph, nullptr, 0, pre);
    if (he == hipSuccess) he = hipGraphAddEventRecordNode(&n_e0, gph, &n_pre, 1, w->ev0);
    if (he == hipSuccess) he = hipGraphAddKernelNode(&n_s, gph, &n_e0, 1, &kp);
    if (he == hipSuccess)
        he = hipGraphKernelNodeSetAttribute(n_s, hipKernelNodeAttributeCooperative, &coop);
    if (he == hipSuccess) he = hipGraphAddEventRecordNode(&n_e1, gph, &n_s, 1, w->ev1);
    if (he == hipSuccess) he = hipGraphAddChildGraphNode(&n_post, gph, &n_e1, 1, post);
    (void)hipGraphDestroy(pre);
    (void)hipGraphDestroy(post);
    if (he == hipSuccess) he = hipGraphInstantiateWithFlags(&p->exec, gph, 0);
    if (he != hipSuccess) {
        if (gph) (void)hipGraphDestroy(gph);
        p->exec = nullptr;
        return fail(MPAP_ERR_HIP, std::string("recording the plan graph: ") + hipGetErrorString(he));
    }
    p->graph = gph;
    ++p->rebuilds;
    return MPAP_OK;
}

// Eager search on the plan's workspace (sizes it), then records the graph.
int plan_eager(mpap_plan *p, hipStream_t s, mpap_result **out) {
    mpap_result *res = new mpap_result();
    res->g = p->g;
    res->ws = p->w;
    res->ws_borrowed = true;
    int r = search_eager(p->g, p->prep, p->shape, p->w, s, res);
    if (!r) r = plan_record(p);
    if (r || !out) {
        mpap_result_free(res);
        return r;
    }
    *out = res;
    return MPAP_OK;
}

}  // namespace

extern "C" {

int mpap_plan_create(mpap_graph *g, const mpap_search_params *sp, int32_t nsp,
                     mpap_graph *const *parts, const mpap_surrogate *const *models,
                     int32_t nparts, int32_t flags, void *stream, mpap_plan **out) {
    if (!out) return fail(MPAP_ERR_INVAL, "out is null");
    *out = nullptr;
    if (!g || !sp) return fail(MPAP_ERR_INVAL, "null graph or params");
    if (flags & ~MPAP_PLAN_ANALYTIC) return fail(MPAP_ERR_INVAL, "unknown plan flags");
    if (nparts != 0 && nparts != g->nq)
        return fail(MPAP_ERR_INVAL, "nparts must be 0 or the graph's query count");
    if (nparts > 0 && (!parts || !models)) return fail(MPAP_ERR_INVAL, "null parts or models");
    mpap_plan *p = new mpap_plan();
    p->g = g;
    p->analytic = (flags & MPAP_PLAN_ANALYTIC) != 0;
    int r = search_prep(g, sp, nsp, p->prep);
    if (!r) r = search_shape(p->prep.stage_cap, p->prep.block_threads, p->prep.wave_min_targets,
                             p->shape, p->prep.merge_halves);
    if (!r) p->shape.obj = uniform_objectives(p->prep);
    auto bail = [&](int st) {
        mpap_plan_free(p);
        return st;
    };
    if (r) return bail(r);
    bool scoring = false;
    if (nparts > 0) {
        long long eo = 0;
        p->parts.assign(parts, parts + nparts);
        p->models.assign(models, models + nparts);
        p->eoff.resize(nparts);
        for (int q = 0; q < nparts; ++q) {
            const mpap_graph *pq = parts[q];
            if (!pq) return bail(fail(MPAP_ERR_INVAL, "null part graph"));
            if (pq->n != g->qoff_h[q + 1] - g->qoff_h[q])
                return bail(fail(MPAP_ERR_INVAL, "a part's node count differs from its query's"));
            p->eoff[q] = eo;
            eo += pq->e;
            if (models[q] || p->analytic) {
                scoring = scoring || models[q] != nullptr;
                if (!pq->pos || !pq->symmetric_alias)
                    return bail(fail(MPAP_ERR_INVAL, "a scored part needs its environment "
                                                     "(mpap_build_graph)"));
            }
        }
        if (eo != g->e) return bail(fail(MPAP_ERR_INVAL, "the parts' edges do not add up"));
    } else if (p->analytic) {
        return bail(fail(MPAP_ERR_INVAL, "MPAP_PLAN_ANALYTIC needs the parts"));
    }
    if ((scoring || p->analytic) && !g->symmetric_alias)
        return bail(fail(MPAP_ERR_INVAL, "scoring inside a plan needs a symmetric roadmap"));
    if (scoring && !g->sdrift && (r = dalloc(&g->sdrift, std::max<long long>(g->e, 1))))
        return bail(r);
    for (int q = 0; q < p->prep.nq; ++q)
        if (p->prep.heur[q] == 1 && !(g->symmetric_alias ? g->sdrift : g->srdrift))
            return bail(fail(MPAP_ERR_INVAL, "no surrogate drift on this graph"));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // score once eagerly so the sizing search sees the same drift
    for (int q = 0; q < nparts && !r; ++q) {
        if (models[q])
            r = sur_enqueue_score(models[q], parts[q], g->sdrift + p->eoff[q], s);
        else if (p->analytic)
            r = enqueue_analytic_drift(parts[q], g->odrift + p->eoff[q], s);
    }
    if (r) return bail(r);
    p->w = new Workspace();
    if ((r = ws_alloc_nodes(p->w, g->n, p->shape.nblocks))) return bail(r);
    if ((r = plan_eager(p, s, nullptr))) return bail(r);
    *out = p;
    return MPAP_OK;
}

int mpap_plan_run(mpap_plan *p, void *stream, mpap_result **out) {
    if (!p || !out) return fail(MPAP_ERR_INVAL, "null argument");
    *out = nullptr;
    if (!p->exec) return fail(MPAP_ERR_INVAL, "plan has no recorded graph");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(hipGraphLaunch(p->exec, s));
    HIP_TRY(hipStreamSynchronize(s));
    ++p->launches;
    const int status = (int)p->h_out[kOutStatus];
    const int err = *p->h_err;
    if (err & kErrTimeout)
        return fail(MPAP_ERR_HIP, "a grid or half-workgroup barrier wait timed out");
    if (err & kErrTarget)
        return fail(MPAP_ERR_HIP, "internal error: a queued merge target is not a node");
    if (status == kStatusNoConverge)
        return fail(MPAP_ERR_NOCONVERGE, "max_waves reached with open plans");
    if (status != kStatusOk || err != 0 || *p->h_ovf != 0) {
        // a capacity was exceeded: search eagerly (growing), record again
        ++p->fallbacks;
        return plan_eager(p, s, out);
    }
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, p->w->ev0, p->w->ev1));
    mpap_result *res = new mpap_result();
    res->g = p->g;
    res->ws = p->w;
    res->ws_borrowed = true;
    search_finish(res, p->prep, p->h_out, p->h_count, p->h_plab, p->h_pnode, p->h_qlast,
                  p->h_qstop, p->h_trace, ms, 0, p->shape);
    *out = res;
    return MPAP_OK;
}

int mpap_plan_info(const mpap_plan *p, int32_t *launches, int32_t *records,
                   int32_t *fallbacks) {
    if (!p) return fail(MPAP_ERR_INVAL, "null plan");
    if (launches) *launches = p->launches;
    if (records) *records = p->rebuilds;
    if (fallbacks) *fallbacks = p->fallbacks;
    return MPAP_OK;
}

void mpap_plan_free(mpap_plan *p) {
    if (!p) return;
    plan_drop_graph(p);
    if (p->w) {
        p->w->free_all();
        delete p->w;
    }
    delete p;
}

}  // extern "C"
