// Online updates (Sec. 3, online implementation): obstacles discovered after
// a roadmap was built, and a search of the changed roadmap that continues
// from an earlier result's labels instead of starting from the root.
//
// mpap_graph_add_boxes: the roadmap's edges are checked against the new boxes
// only (the earlier ones were checked when it was built) and the colliding
// ones dropped; costs, drifts and node flags are kept.  The result is the
// roadmap mpap_build_graph makes for the same samples with the boxes added.
//
// mpap_search_update: the earlier search's labels stay where their plans use
// no edge that changed (removed, added, or other cost or drift bits); the
// others are dropped.  Nodes that lost labels may now keep plans those labels
// dominated, so the labels of their in-neighbours are opened again, as are
// the labels at the tails of new or changed edges; the persistent search then
// runs from that state until no label is open.  At the end every label has
// been extended along every out-edge of its node with the edge's current
// values and the children merged, the fixpoint of Alg. 3's loop, whose only
// solution with positive costs is the exact front of every node (a plan
// dominated at its node is dominated by a kept label, whose extension
// dominates the plan's).  Dropping a valid label is only extra work (its node
// is then re-derived), so changes are detected conservatively.
#include "device_common.h"
#include "runtime_internal.h"

namespace {

// source node of every forward edge
__global__ void k_edge_sources(int n, const int *row_ptr, int *src) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    for (int e = row_ptr[u]; e < row_ptr[u + 1]; ++e) src[e] = u;
}

__global__ void k_compact_f32(long long m, const int *keep, const int *kscan, const float *in,
                              float *out) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m || !keep[e]) return;
    out[kscan[e]] = in[e];
}

// Per node u, its out-rows in the earlier (o*) and current (n*) roadmap:
// ochg[e] = 1 for an earlier edge u -> v with no current edge u -> v of the
// same cost and drift bits, or whose head's relocalisation flag changed (the
// child's drift differs); odirty[u] = some earlier edge of u changed;
// ndirty[u] = some current edge of u is new or changed.
__global__ void k_edge_changes(int n, const int *optr, const int *ocol, const float *ocost,
                               const float *odrift, const uint8_t *oflag, const int *nptr,
                               const int *ncol, const float *ncost, const float *ndrift,
                               const uint8_t *nflag, uint8_t *ochg, uint8_t *odirty,
                               uint8_t *ndirty) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const int o0 = optr[u], o1 = optr[u + 1], n0 = nptr[u], n1 = nptr[u + 1];
    bool od = false, nd = false;
    for (int e = o0; e < o1; ++e) {
        bool same = ((oflag[ocol[e]] ^ nflag[ocol[e]]) & 1u) == 0u;
        if (!same) {
            ochg[e] = 1;
            od = true;
            continue;
        }
        same = false;
        for (int f = n0; f < n1 && !same; ++f)
            same = ncol[f] == ocol[e] && __float_as_uint(ncost[f]) == __float_as_uint(ocost[e]) &&
                   __float_as_uint(ndrift[f]) == __float_as_uint(odrift[e]);
        ochg[e] = same ? 0 : 1;
        od = od || !same;
    }
    for (int f = n0; f < n1; ++f) {
        bool same = false;
        if (((oflag[ncol[f]] ^ nflag[ncol[f]]) & 1u) != 0u) {
            nd = true;
            continue;
        }
        for (int e = o0; e < o1 && !same; ++e)
            same = ncol[f] == ocol[e] && __float_as_uint(ncost[f]) == __float_as_uint(ocost[e]) &&
                   __float_as_uint(ndrift[f]) == __float_as_uint(odrift[e]);
        nd = nd || !same;
    }
    odirty[u] = od ? 1 : 0;
    ndirty[u] = nd ? 1 : 0;
}

// Labels of one earlier group (ids [lo, hi)): a label is dropped when its
// parent was, or when the edge from the parent's node to its own changed
// (any earlier edge between the two nodes, so parallel edges count too).
__global__ void k_label_drop(long long lo, long long hi, const int2 *arena, const int *optr,
                             const int *ocol, const uint8_t *ochg, const uint8_t *odirty,
                             uint8_t *drop) {
    const long long id = lo + (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= hi) return;
    const int2 me = arena[id];
    if (me.y < 0) {
        drop[id] = 0;
        return;
    }
    bool d = drop[me.y] != 0;
    if (!d) {
        const int u = arena[me.y].x;
        if (odirty[u])
            for (int e = optr[u]; e < optr[u + 1] && !d; ++e) d = ocol[e] == me.x && ochg[e];
    }
    drop[id] = d ? 1 : 0;
}

// One wave per node: dropped labels leave the front, in place, order kept
// (a lane writes at or below the slot it read, after the wave's reads of the
// same 64 slots); lost[v] = 1 when the node lost any.  Every label left is
// closed (its own id).
__global__ void k_front_prune(int n, int4 *nb, float4 *pool, const uint8_t *drop,
                              uint8_t *lost) {
    const int l = threadIdx.x & 63;
    const int v = (int)(((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (v >= n) return;
    const int4 b = nb[v];
    int out = 0;
    for (int k0 = 0; k0 < b.z; k0 += 64) {
        const int k = k0 + l;
        bool keep = false;
        float4 L = make_float4(0.f, 0.f, 0.f, 0.f);
        if (k < b.z) {
            L = pool[(size_t)(unsigned)b.x + k];
            keep = !drop[__float_as_int(L.w)];
        }
        const uint64_t m = ballot64(keep);
        if (keep) pool[(size_t)(unsigned)b.x + out + lanes_below(m)] = L;
        out += (int)__popcll(m);
    }
    if (l == 0) {
        nb[v] = make_int4(b.x, b.y, out, 0);
        lost[v] = out < b.z ? 1 : 0;
    }
}

// seeds: the tails of new or changed edges (k_seed_tails), and every
// in-neighbour (current roadmap) of a node that lost labels (k_mark_seeds,
// after it: idempotent stores of 1)
__global__ void k_seed_tails(int n, const uint8_t *ndirty, uint8_t *seed) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) seed[v] = ndirty[v];
}
__global__ void k_mark_seeds(int n, const uint8_t *lost, const int *rptr, const int *rsrc,
                             uint8_t *seed) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n || !lost[v]) return;
    for (int e = rptr[v]; e < rptr[v + 1]; ++e) seed[rsrc[e]] = 1;
}

// Per node: the labels of a seed open again (meta = parent + 1 with the open
// bit); node state for the next search (group bookkeeping cleared).
__global__ void k_reopen(int n, int4 *nb, float4 *pool, const int2 *arena, const uint8_t *seed,
                         float *minopen, int4 *fo, int *gcnt, int *mark, int *wt) {
    const int l = threadIdx.x & 63;
    const int v = (int)(((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (v >= n) return;
    const int4 b = nb[v];
    const bool s = seed[v] != 0 && b.z > 0;
    if (s)
        for (int k = l; k < b.z; k += 64) {
            const size_t slot = (size_t)(unsigned)b.x + k;
            const int id = __float_as_int(pool[slot].w);
            const unsigned meta = MPAP_OPEN_BIT | (unsigned)(arena[id].y + 1);
            reinterpret_cast<unsigned *>(&pool[slot])[3] = meta;
        }
    if (l == 0) {
        nb[v] = make_int4(b.x, b.y, b.z, s ? b.z : 0);
        minopen[v] = s ? pool[(size_t)(unsigned)b.x].x : MPAP_INF;
        fo[v] = make_int4(0, 0, -1, s ? 0 : b.z);
        gcnt[v] = 0;
        mark[v] = -1;
        wt[v] = 0;
    }
}

// the launch-wide words a search starts from (as k_search_init, without the
// node state), and the one query's bookkeeping
__global__ void k_update_words(SearchArgs a) {
    if (blockIdx.x != 0) return;
    for (int i = threadIdx.x; i < 2 * kListRegions; i += blockDim.x) {
        a.acnt[i] = 0;
        a.mcur[i] = 0;
    }
    for (int i = threadIdx.x; i < kOutWords; i += blockDim.x) a.out[i] = 0;
    for (long long i = threadIdx.x; i < (long long)a.wstat_cap * kTraceWords; i += blockDim.x)
        a.wstat[i] = 0;
    if (threadIdx.x == 0) {
        *a.bar = 0u;
        *a.err = 0;
        a.qlast[0] = 0;
        a.qstop[0] = -2;
    }
}

// Where each group of the result's arena starts (parents are always in an
// earlier group), and the arena size last: an update's stored list, else the
// group sizes of the search's trace.  False when the trace was cut short.
bool group_bounds(const mpap_result *r, std::vector<long long> &gs) {
    if (!r->group_start.empty()) {
        gs = r->group_start;
        return gs.back() == r->arena_labels;
    }
    const int waves = r->stats.waves;
    if (waves > kTraceCap || (long long)r->trace.size() < (long long)waves * kTraceWords)
        return false;
    gs.assign(waves + 1, 0);
    for (int w = 0; w < waves; ++w)
        gs[w + 1] = gs[w] + r->trace[(size_t)w * kTraceWords + kTrGroup];
    return gs.back() == r->arena_labels;
}

template <typename T>
int copy_d2d(T *dst, const T *src, size_t count, hipStream_t s) {
    if (count) HIP_TRY(hipMemcpyAsync(dst, src, sizeof(T) * count, hipMemcpyDeviceToDevice, s));
    return MPAP_OK;
}

}  // namespace

extern "C" {

int mpap_graph_add_boxes(const mpap_graph *gc, int32_t n_boxes, const float *box_lo,
                         const float *box_hi, void *stream, mpap_graph **out) {
    if (!out) return fail(MPAP_ERR_INVAL, "out is null");
    *out = nullptr;
    if (!gc || n_boxes < 0 || (n_boxes > 0 && (!box_lo || !box_hi)))
        return fail(MPAP_ERR_INVAL, "null graph or box arrays, or n_boxes < 0");
    const mpap_graph *g = gc;
    if ((g->dim != 2 && g->dim != 3) || !g->pos || g->nq != 1)
        return fail(MPAP_ERR_INVAL, "boxes are added to 2D/3D roadmaps built by mpap_build_graph");
    const int dim = g->dim, n = g->n;
    for (long long i = 0; i < (long long)n_boxes * dim; ++i)
        if (!std::isfinite(box_lo[i]) || !std::isfinite(box_hi[i]))
            return fail(MPAP_ERR_INVAL, "non-finite box corner");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != g->dev) return fail(MPAP_ERR_INVAL, "the graph lives on another device");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const long long m = g->e;
    float *d_blo = nullptr, *d_bhi = nullptr;
    int *src = nullptr, *keep = nullptr, *kscan = nullptr, *tmp = nullptr;
    mpap_graph *ng = nullptr;
    auto cleanup = [&]() {
        dfree(d_blo); dfree(d_bhi); dfree(src); dfree(keep); dfree(kscan); dfree(tmp);
    };
    auto bail = [&](int st) {
        cleanup();
        if (ng) graph_release(ng);
        return st;
    };
    int r;
    const size_t nb_ = (size_t)n_boxes * dim;
    if ((r = dalloc(&d_blo, nb_)) || (r = dalloc(&d_bhi, nb_)) || (r = dalloc(&src, m)) ||
        (r = dalloc(&keep, m)) || (r = dalloc(&kscan, m)) ||
        (r = dalloc(&tmp, div_up(std::max(m, 1LL), kScanTile) + 1)))
        return bail(r);
    if (nb_) {
        HIP_TRY(hipMemcpyAsync(d_blo, box_lo, sizeof(float) * nb_, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d_bhi, box_hi, sizeof(float) * nb_, hipMemcpyHostToDevice, s));
    }
    BuildArgs a{};
    a.n = n; a.dim = dim; a.pos = g->pos; a.nbox = n_boxes; a.blo = d_blo; a.bhi = d_bhi;
    a.step = g->check_step;
    long long e_new = 0;
    if (m > 0) {
        k_edge_sources<<<div_up(n, 256), 256, 0, s>>>(n, g->optr, src);
        // Collision against the new boxes only (Alg. 2 Collision; the earlier
        // boxes were tested when the roadmap was built)
        k_collide<<<div_up(m, 256), 256, sizeof(float) * 2 * nb_, s>>>(a, m, src, g->ocol,
                                                                       g->ocost, keep);
        if ((r = scan_i32(keep, kscan, m, tmp, s))) return bail(r);
        int last_keep = 0, last_ks = 0;
        HIP_TRY(hipMemcpyAsync(&last_keep, keep + (m - 1), sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&last_ks, kscan + (m - 1), sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        e_new = (long long)last_keep + last_ks;
    }
    ng = new mpap_graph();
    ng->dev = g->dev;
    ng->n = n;
    ng->e = e_new;
    ng->n_goal = g->n_goal;
    ng->symmetric_alias = true;
    const size_t nf = (size_t)g->nblob;
    if ((r = dalloc(&ng->optr, n + 1)) || (r = dalloc(&ng->ocol, e_new)) ||
        (r = dalloc(&ng->ocost, e_new)) || (r = dalloc(&ng->odrift, e_new)) ||
        (r = dalloc(&ng->nflag, n)) || (r = dalloc(&ng->goal_list, std::max(g->n_goal, 1))) ||
        (r = dalloc(&ng->pos, (size_t)n * dim)) || (r = dalloc(&ng->bmu, nf * dim)) ||
        (r = dalloc(&ng->bsig, nf)) || (r = dalloc(&ng->bamp, nf)) ||
        (r = dalloc(&ng->blo, (size_t)(g->nbox + n_boxes) * dim)) ||
        (r = dalloc(&ng->bhi, (size_t)(g->nbox + n_boxes) * dim)))
        return bail(r);
    if (m > 0) {
        k_compact_edges<<<div_up(m, 256), 256, 0, s>>>(m, keep, kscan, g->ocol, g->ocost,
                                                       ng->ocol, ng->ocost);
        k_compact_f32<<<div_up(m, 256), 256, 0, s>>>(m, keep, kscan, g->odrift, ng->odrift);
        k_row_ptr<<<div_up(n + 1, 256), 256, 0, s>>>(n, m, g->optr, kscan, keep, ng->optr);
    } else {
        k_zero_i32<<<div_up(n + 1, 256), 256, 0, s>>>(ng->optr, n + 1);
    }
    HIP_TRY(hipGetLastError());
    if ((r = copy_d2d(ng->nflag, g->nflag, n, s)) ||
        (r = copy_d2d(ng->goal_list, g->goal_list, g->n_goal, s)) ||
        (r = copy_d2d(ng->pos, g->pos, (size_t)n * dim, s)) ||
        (r = copy_d2d(ng->bmu, g->bmu, nf * dim, s)) || (r = copy_d2d(ng->bsig, g->bsig, nf, s)) ||
        (r = copy_d2d(ng->bamp, g->bamp, nf, s)) ||
        (r = copy_d2d(ng->blo, g->blo, (size_t)g->nbox * dim, s)) ||
        (r = copy_d2d(ng->bhi, g->bhi, (size_t)g->nbox * dim, s)) ||
        (r = copy_d2d(ng->blo + (size_t)g->nbox * dim, d_blo, nb_, s)) ||
        (r = copy_d2d(ng->bhi + (size_t)g->nbox * dim, d_bhi, nb_, s)))
        return bail(r);
    ng->rptr = ng->optr; ng->rsrc = ng->ocol; ng->rcost = ng->ocost; ng->rdrift = ng->odrift;
    ng->dim = dim; ng->nbox = g->nbox + n_boxes; ng->nblob = g->nblob;
    ng->check_step = g->check_step; ng->reset_q = g->reset_q; ng->radius = g->radius;
    if ((r = build_pair_index(ng, s))) return bail(r);
    HIP_TRY(hipStreamSynchronize(s));
    cleanup();
    if ((r = graph_set_single_query(ng))) {
        graph_release(ng);
        return r;
    }
    *out = ng;
    return MPAP_OK;
}

int mpap_search_update(const mpap_result *prev, const mpap_graph *gc,
                       const mpap_search_params *sp, void *stream, mpap_result **out) {
    if (!out) return fail(MPAP_ERR_INVAL, "out is null");
    *out = nullptr;
    if (!prev || !gc || !sp) return fail(MPAP_ERR_INVAL, "null result, graph or params");
    mpap_graph *g = const_cast<mpap_graph *>(gc);
    const mpap_graph *og = prev->g;
    if (g->nq != 1 || og->nq != 1 || g->n != og->n)
        return fail(MPAP_ERR_INVAL, "single-query roadmaps over the same nodes");
    if (prev->fallback || prev->judged)
        return fail(MPAP_ERR_INVAL, "the earlier result was judged (search afresh)");
    if (!prev->qstop.empty() && prev->qstop[0] >= 0)
        return fail(MPAP_ERR_INVAL, "the earlier search stopped early (search afresh)");
    if (sp->early_stop) return fail(MPAP_ERR_INVAL, "an update runs to the exact fronts");
    if (sp->skip) return fail(MPAP_ERR_INVAL, "skip must be 0");
    if (sp->n_obj != prev->n_obj ||
        std::memcmp(&sp->beta, &prev->qbeta[0], sizeof(float)) != 0 ||
        sp->init_node + g->qoff_h[0] != prev->qroot[0] || sp->heuristic != prev->qheur[0])
        return fail(MPAP_ERR_INVAL, "bound, objectives, root and heuristic must be the earlier "
                                    "search's");
    if (sp->heuristic != 0) return fail(MPAP_ERR_INVAL, "updates run on the analytic drift");
    if (prev->ws_borrowed)
        return fail(MPAP_ERR_INVAL, "a plan's result (search afresh or with mpap_search)");
    std::vector<long long> gstart;
    if (!group_bounds(prev, gstart) || prev->pool_used < 16)
        return fail(MPAP_ERR_INVAL, "the earlier search ran more iterations than its trace "
                                    "keeps (search afresh)");
    const int ngroups = (int)gstart.size() - 1;
    SearchPrep p;
    int r = search_prep(g, sp, 1, p);
    if (r) return r;
    SearchShape L;
    if ((r = search_shape(p.stage_cap, p.block_threads, p.wave_min_targets, L, p.merge_halves)))
        return r;
    L.obj = uniform_objectives(p);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Workspace *ow = prev->ws;
    const int n = g->n;
    const long long La = prev->arena_labels;

    uint8_t *ochg = nullptr, *odirty = nullptr, *ndirty = nullptr, *drop = nullptr,
            *lost = nullptr, *seed = nullptr;
    auto cleanup = [&]() {
        dfree(ochg); dfree(odirty); dfree(ndirty); dfree(drop); dfree(lost); dfree(seed);
    };
    const unsigned long long used = prev->pool_used;
    if ((r = dalloc(&ochg, og->e)) || (r = dalloc(&odirty, n)) || (r = dalloc(&ndirty, n)) ||
        (r = dalloc(&drop, La)) || (r = dalloc(&lost, n)) || (r = dalloc(&seed, n))) {
        cleanup();
        return r;
    }
    Workspace *w = nullptr;
    if ((r = acquire_workspace(g, L, &w))) {
        cleanup();
        return r;
    }
    mpap_result *res = new mpap_result();
    res->g = g;
    res->ws = w;
    auto bail = [&](int st) {
        cleanup();
        mpap_result_free(res);
        return st;
    };
    if ((r = search_upload(w, p, s))) return bail(r);
    unsigned long long pool_cap = std::max<unsigned long long>(
        std::max<unsigned long long>(w->pool_cap, used + 65536), 2 * used);
    long long arena_cap = std::max<long long>(w->arena_cap, La + 128ll * n + 65536);
    long long F_cap = std::max<long long>(w->F_cap, 32ll * n + 65536);
    pool_cap = std::min<unsigned long long>(pool_cap, (1ull << 31) - 1);
    long long capG = std::max<long long>(w->spill_cap, std::max(4 * L.capB, 32768));
    long long dev_out[kOutWords];
    int dev_err = 0, retries = 0;
    float ms = 0.f;
    SearchArgs a{};
    // which edges changed, and which earlier labels stay (independent of the
    // workspace; done once)
    k_edge_changes<<<div_up(n, 256), 256, 0, s>>>(n, og->optr, og->ocol, og->ocost, og->odrift,
                                                  og->nflag, g->optr, g->ocol, g->ocost,
                                                  g->odrift, g->nflag, ochg, odirty, ndirty);
    for (int wv = 0; wv < ngroups; ++wv) {
        const long long lo = gstart[wv], hi = gstart[wv + 1];
        if (hi > lo)
            k_label_drop<<<div_up(hi - lo, 256), 256, 0, s>>>(lo, hi, ow->arena, og->optr,
                                                              og->ocol, ochg, odirty, drop);
    }
    HIP_TRY(hipGetLastError());
    for (;;) {
        if ((r = ws_grow(w, pool_cap, arena_cap, F_cap, 0))) return bail(r);
        if ((r = ws_spill(w, capG))) return bail(r);
        a = search_args(g, w, p, L);
        a.arena_base = La;
        // the earlier state, then the changes
        if ((r = copy_d2d(w->nb, ow->nb, n, s)) || (r = copy_d2d(w->pool, ow->pool, used, s)) ||
            (r = copy_d2d(w->arena, ow->arena, La, s)) ||
            (r = copy_d2d(w->pool_top, ow->pool_top, 1, s)))
            return bail(r);
        k_front_prune<<<div_up(64ll * n, 256), 256, 0, s>>>(n, w->nb, w->pool, drop, lost);
        k_seed_tails<<<div_up(n, 256), 256, 0, s>>>(n, ndirty, seed);
        k_mark_seeds<<<div_up(n, 256), 256, 0, s>>>(n, lost, g->rptr, g->rsrc, seed);
        k_reopen<<<div_up(64ll * n, 256), 256, 0, s>>>(n, w->nb, w->pool, w->arena, seed,
                                                       w->minopen, w->fo, w->gcnt, w->mark,
                                                       w->wt);
        k_update_words<<<1, 256, 0, s>>>(a);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipEventRecord(w->ev0, s));
        void *kargs[] = {&a};
        HIP_TRY(hipLaunchCooperativeKernel(search_kernel_for(L, g->n), dim3(L.nblocks),
                                           dim3(L.threads), kargs, L.lds, s));
        HIP_TRY(hipEventRecord(w->ev1, s));
        k_count_front<<<std::max(1, std::min(div_up(g->n, 256), 1024)), 256, 0, s>>>(a);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(dev_out, w->out, sizeof(dev_out), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&dev_err, w->err, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipEventElapsedTime(&ms, w->ev0, w->ev1));
        const int status = (int)dev_out[kOutStatus];
        if (status == kStatusOk && dev_err == 0) break;
        if (dev_err & kErrTimeout)
            return bail(fail(MPAP_ERR_HIP, "a grid or half-workgroup barrier wait timed out"));
        if (dev_err & kErrTarget)
            return bail(fail(MPAP_ERR_HIP, "internal error: a queued merge target is not a node"));
        if (status == kStatusNoConverge)
            return bail(fail(MPAP_ERR_NOCONVERGE, "max_waves reached with open plans"));
        if (++retries > 12) return bail(fail(MPAP_ERR_OVERFLOW, "capacity retries exhausted"));
        if (dev_err & kErrBucket) capG *= 4;
        if (dev_err & kErrPool)
            pool_cap = std::min<unsigned long long>(pool_cap * 4, (1ull << 31) - 1);
        if (status == kStatusArena) {
            if (dev_out[kOutLabels] + dev_out[kOutNeed] > arena_cap) arena_cap *= 4;
            if (dev_out[kOutNeed] > F_cap) F_cap *= 4;
        }
    }
    if ((r = search_goal_finish(g, p, L, w, s, res, a, dev_out, ms, retries))) return bail(r);
    res->stats.labels_expanded = dev_out[kOutLabels] - La;  // this launch's expansions
    res->reused_arena = La;
    // group bounds over the whole arena: the earlier ones, then this launch's
    const int nw = res->stats.waves;
    if (nw <= kTraceCap && (long long)res->trace.size() >= (long long)nw * kTraceWords) {
        res->group_start = gstart;
        for (int wv = 0; wv < nw; ++wv)
            res->group_start.push_back(res->group_start.back() +
                                       res->trace[(size_t)wv * kTraceWords + kTrGroup]);
    }
    cleanup();
    *out = res;
    return MPAP_OK;
}

}  // extern "C"
