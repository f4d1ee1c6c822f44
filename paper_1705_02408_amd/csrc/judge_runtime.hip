// The learned heuristic's judge and analytic fallback (include/mpap.h,
// mpap_judge, mpap_rescore_front).
//
// The learned per-edge drift stands in for the heuristic precompute of
// Alg. 1 step 2 (learned heuristics, Sec. 5.2).  Its search is accepted per
// query only when every goal-front plan, re-walked with the analytic drift,
// stays feasible and keeps its drift within a relative tolerance; a query
// that fails is searched again on the analytic drift, in one launch with the
// accepted queries skipped, and the result then answers it from that exact
// search.
#include <chrono>

#include "runtime_internal.h"

namespace {

constexpr int kRewalkMaxLen = 4096;

// Re-walk labels (ids into `arena`) on g's analytic drift; with sur, also the
// judge's per-label decision.  out and pass are resized to the label count.
int rewalk(const int2 *arena, const mpap_graph *g, const std::vector<int> &lab,
           const std::vector<float> &beta, const std::vector<int> &nobj, const float4 *sur,
           float tol, std::vector<float4> &out, std::vector<uint8_t> &pass, hipStream_t s) {
    const int n = (int)lab.size();
    out.assign(n, make_float4(0.f, 0.f, 0.f, 0.f));
    pass.assign(n, 0);
    if (n == 0) return MPAP_OK;
    int *dlab = nullptr, *dnobj = nullptr, *dpath = nullptr, *derr = nullptr;
    float *dbeta = nullptr;
    float4 *dout = nullptr, *dsur = nullptr;
    uint8_t *dpass = nullptr;
    auto cleanup = [&]() {
        dfree(dlab); dfree(dnobj); dfree(dpath); dfree(derr); dfree(dbeta); dfree(dout);
        dfree(dsur); dfree(dpass);
    };
    int rc;
    if ((rc = dalloc(&dlab, n)) || (rc = dalloc(&dnobj, n)) || (rc = dalloc(&dbeta, n)) ||
        (rc = dalloc(&dpath, (size_t)n * kRewalkMaxLen)) || (rc = dalloc(&derr, 1)) ||
        (rc = dalloc(&dout, n)) || (sur && ((rc = dalloc(&dsur, n)) || (rc = dalloc(&dpass, n))))) {
        cleanup();
        return rc;
    }
    int err = 0;
    hipError_t he = hipMemcpyAsync(dlab, lab.data(), sizeof(int) * n, hipMemcpyHostToDevice, s);
    if (he == hipSuccess)
        he = hipMemcpyAsync(dnobj, nobj.data(), sizeof(int) * n, hipMemcpyHostToDevice, s);
    if (he == hipSuccess)
        he = hipMemcpyAsync(dbeta, beta.data(), sizeof(float) * n, hipMemcpyHostToDevice, s);
    if (he == hipSuccess) he = hipMemcpyAsync(derr, &err, sizeof(int), hipMemcpyHostToDevice, s);
    if (he == hipSuccess && sur)
        he = hipMemcpyAsync(dsur, sur, sizeof(float4) * n, hipMemcpyHostToDevice, s);
    if (he == hipSuccess) {
        k_rescore<<<div_up(n, 256), 256, 0, s>>>(arena, g->optr, g->ocol, g->ocost, g->odrift,
                                                 g->nflag, dlab, dbeta, dnobj, n, dpath,
                                                 kRewalkMaxLen, dout, derr, dsur, tol, dpass);
        he = hipGetLastError();
    }
    if (he == hipSuccess)
        he = hipMemcpyAsync(out.data(), dout, sizeof(float4) * n, hipMemcpyDeviceToHost, s);
    if (he == hipSuccess && sur)
        he = hipMemcpyAsync(pass.data(), dpass, n, hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipMemcpyAsync(&err, derr, sizeof(int), hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    cleanup();
    if (he != hipSuccess) return fail(MPAP_ERR_HIP, hipGetErrorString(he));
    if (err) return fail(MPAP_ERR_HIP, "a plan could not be re-walked (longer than 4096 steps?)");
    return MPAP_OK;
}

inline int label_of(const float4 &L) {
    int id;
    std::memcpy(&id, &L.w, sizeof(int));
    return id;
}

}  // namespace

extern "C" {

int mpap_rescore_front(const mpap_result *r, int32_t query, float *cost, float *drift,
                       float *maxdrift, uint8_t *feasible, int32_t capacity, int32_t *count) {
    if (!r || !count) return fail(MPAP_ERR_INVAL, "null argument");
    const int nq = r->g->nq;
    if (query < -1 || query >= nq) return fail(MPAP_ERR_INVAL, "query out of range");
    const int q0 = query < 0 ? 0 : query, q1 = query < 0 ? nq : query + 1;
    const int64_t o = r->front_off[q0];
    const int n = (int)(r->front_off[q1] - o);
    *count = n;
    if (capacity < n) return fail(MPAP_ERR_CAPACITY, "capacity below the front size");
    if (n == 0) return MPAP_OK;
    // labels of the first search, and those of the fallback re-search (ids
    // shifted by id_offset in r), each re-walked on its own arena
    std::vector<int> lab[2], nobj[2], where[2];
    std::vector<float> beta[2];
    for (int q = q0; q < q1; ++q) {
        const int k = (r->fallback && r->qfall[q]) ? 1 : 0;
        for (int64_t i = r->front_off[q]; i < r->front_off[q + 1]; ++i) {
            lab[k].push_back(label_of(r->front[i]) - (k ? (int)r->id_offset : 0));
            beta[k].push_back(r->qbeta[q]);
            nobj[k].push_back(r->qnobj[q]);
            where[k].push_back((int)(i - o));
        }
    }
    for (int k = 0; k < 2; ++k) {
        if (lab[k].empty()) continue;
        const int2 *arena = k ? r->fallback->ws->arena : r->ws->arena;
        std::vector<float4> out;
        std::vector<uint8_t> pass;
        const int rc = rewalk(arena, r->g, lab[k], beta[k], nobj[k], nullptr, 0.f, out, pass,
                              nullptr);
        if (rc) return rc;
        for (size_t j = 0; j < out.size(); ++j) {
            const int i = where[k][j];
            if (cost) cost[i] = out[j].x;
            if (drift) drift[i] = out[j].y;
            if (maxdrift) maxdrift[i] = out[j].z;
            if (feasible) feasible[i] = out[j].w > 0.5f ? 1 : 0;
        }
    }
    return MPAP_OK;
}

int mpap_judge(mpap_result *r, float tol, int32_t fallback, void *stream, uint8_t *failed,
               int32_t *n_failed) {
    if (!r) return fail(MPAP_ERR_INVAL, "null result");
    if (!(tol > 0.0f) || !std::isfinite(tol)) return fail(MPAP_ERR_INVAL, "tol must be > 0");
    if (fallback != 0 && fallback != 1) return fail(MPAP_ERR_INVAL, "fallback must be 0 or 1");
    if (r->judged) return fail(MPAP_ERR_INVAL, "result already judged");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    mpap_graph *g = r->g;
    const int nq = g->nq;
    const auto t0 = std::chrono::steady_clock::now();
    // the goal-front labels of every query searched on the learned drift
    std::vector<int> lab, nobj, owner;
    std::vector<float> beta;
    std::vector<float4> sur;
    for (int q = 0; q < nq; ++q) {
        if (q >= (int)r->qheur.size() || r->qheur[q] != 1) continue;
        for (int64_t i = r->front_off[q]; i < r->front_off[q + 1]; ++i) {
            lab.push_back(label_of(r->front[i]));
            beta.push_back(r->qbeta[q]);
            nobj.push_back(r->qnobj[q]);
            sur.push_back(r->front[i]);
            owner.push_back(q);
        }
    }
    std::vector<uint8_t> qfail(nq, 0);
    if (!lab.empty()) {
        std::vector<float4> out;
        std::vector<uint8_t> pass;
        const int rc = rewalk(r->ws->arena, g, lab, beta, nobj, sur.data(), tol, out, pass, s);
        if (rc) return rc;
        for (size_t i = 0; i < pass.size(); ++i)
            if (!pass[i]) qfail[owner[i]] = 1;
    }
    int nf = 0;
    for (int q = 0; q < nq; ++q) nf += qfail[q];
    const double judge_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    r->judged = true;
    r->stats.judged_failed = nf;
    if (failed) std::memcpy(failed, qfail.data(), nq);
    if (n_failed) *n_failed = nf;
    if (!fallback || nf == 0) return MPAP_OK;

    // the analytic re-search of the rejected queries, one launch
    SearchPrep p;
    p.nq = nq;
    p.delta = r->qdelta;
    p.beta = r->qbeta;
    p.nobj = r->qnobj;
    p.root = r->qroot;
    p.heur.assign(nq, 0);
    p.skip.assign(nq, 1);
    p.early = r->qearly;
    for (int q = 0; q < nq; ++q) p.early_any = p.early_any || (qfail[q] && r->qearly[q]);
    for (int q = 0; q < nq; ++q) p.skip[q] = qfail[q] ? 0 : 1;
    p.max_waves = r->max_waves;
    p.near_scan = r->near_scan;
    p.stage_cap = r->stage_cap;
    p.block_threads = r->block_threads;
    p.wave_min_targets = r->wave_min_targets;
    p.merge_halves = r->merge_halves;
    SearchShape L;
    int rc = search_shape(p.stage_cap, p.block_threads, p.wave_min_targets, L, p.merge_halves);
    if (rc) return rc;
    L.obj = uniform_objectives(p);
    Workspace *w = nullptr;
    if ((rc = acquire_workspace(g, L, &w))) return rc;
    mpap_result *fb = new mpap_result();
    fb->g = g;
    fb->ws = w;
    if ((rc = search_eager(g, p, L, w, s, fb))) {
        mpap_result_free(fb);
        return rc;
    }
    const long long off = r->arena_labels;
    if (off + fb->arena_labels > 0x7fffffffll) {
        mpap_result_free(fb);
        return fail(MPAP_ERR_OVERFLOW, "label ids of the two searches exceed int32");
    }
    // goal fronts: the rejected queries' from the re-search, ids shifted
    std::vector<float4> front;
    std::vector<int32_t> node;
    std::vector<int64_t> foff(nq + 1, 0);
    for (int q = 0; q < nq; ++q) {
        const mpap_result *src = qfail[q] ? fb : r;
        for (int64_t i = src->front_off[q]; i < src->front_off[q + 1]; ++i) {
            float4 L4 = src->front[i];
            if (qfail[q]) {
                const int id = label_of(L4) + (int)off;
                std::memcpy(&L4.w, &id, sizeof(int));
            }
            front.push_back(L4);
            node.push_back(src->front_node[i]);
        }
        foff[q + 1] = (int64_t)front.size();
        if (qfail[q]) {
            r->qlast[q] = fb->qlast[q];
            r->qlatency_ms[q] = (float)(r->stats.gpu_ms + judge_ms + fb->qlatency_ms[q]);
        }
    }
    r->front.swap(front);
    r->front_node.swap(node);
    r->front_off.swap(foff);
    r->stats.fallback_ms = fb->stats.gpu_ms;
    r->fallback = fb;
    r->qfall = qfail;
    r->id_offset = off;
    return MPAP_OK;
}

}  // extern "C"
