// Host runtime and C ABI of libmpap (see include/mpap.h).
//
// Owns device memory for graphs and search workspaces, validates inputs,
// launches the kernels, grows capacities and retries when the device reports
// an overflow, and copies results back.  No part of the search itself runs on
// the host.
#include <cstring>

#include "runtime_internal.h"
#include "steer_kernels.h"

thread_local std::string g_last_error;

extern "C" {

const char *mpap_status_string(int status) {
    switch (status) {
        case MPAP_OK: return "ok";
        case MPAP_ERR_INVAL: return "invalid argument";
        case MPAP_ERR_NOGOAL: return "no roadmap node in the goal region";
        case MPAP_ERR_NOMEM: return "out of memory";
        case MPAP_ERR_HIP: return "HIP runtime error";
        case MPAP_ERR_OVERFLOW: return "capacity overflow";
        case MPAP_ERR_NOCONVERGE: return "wave limit reached";
        case MPAP_ERR_CAPACITY: return "caller buffer too small";
        case MPAP_ERR_DEVICE: return "unsupported device";
        default: return "unknown status";
    }
}

const char *mpap_last_error(void) { return g_last_error.c_str(); }

// ------------------------------------------------------------ graph import
int mpap_graph_from_csr(int32_t n, const int32_t *row_ptr, const int32_t *col,
                        const float *cost, const float *drift, const uint8_t *reset,
                        const uint8_t *goal, void *stream, mpap_graph **out) {
    if (!out) return fail(MPAP_ERR_INVAL, "out is null");
    *out = nullptr;
    if (n < 1 || !row_ptr || !reset || !goal) return fail(MPAP_ERR_INVAL, "null input or n < 1");
    if (row_ptr[0] != 0) return fail(MPAP_ERR_INVAL, "row_ptr[0] != 0");
    for (int32_t u = 0; u < n; ++u)
        if (row_ptr[u + 1] < row_ptr[u]) return fail(MPAP_ERR_INVAL, "row_ptr decreases");
    const int64_t e = row_ptr[n];
    if (e > 0 && (!col || !cost || !drift)) return fail(MPAP_ERR_INVAL, "null edge array");
    for (int32_t u = 0; u < n; ++u)
        for (int32_t k = row_ptr[u]; k < row_ptr[u + 1]; ++k) {
            if (col[k] < 0 || col[k] >= n) return fail(MPAP_ERR_INVAL, "col out of range");
            if (col[k] == u) return fail(MPAP_ERR_INVAL, "self loop");
            if (!(cost[k] > 0.0f) || !std::isfinite(cost[k]))
                return fail(MPAP_ERR_INVAL, "edge cost must be finite and > 0");
            if (!(drift[k] >= 0.0f) || !std::isfinite(drift[k]))
                return fail(MPAP_ERR_INVAL, "edge drift must be finite and >= 0");
        }
    DeviceInfo di;
    int r = device_info(&di);
    if (r) return r;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    // in-edge CSR: stable counting sort of the edges by target
    std::vector<int32_t> rptr(n + 1, 0), rsrc(e), rperm(e);
    std::vector<float> rcost(e), rdrift(e);
    for (int64_t k = 0; k < e; ++k) rptr[col[k] + 1]++;
    for (int32_t v = 0; v < n; ++v) rptr[v + 1] += rptr[v];
    {
        std::vector<int32_t> fill(rptr.begin(), rptr.end() - 1);
        for (int32_t u = 0; u < n; ++u)
            for (int32_t k = row_ptr[u]; k < row_ptr[u + 1]; ++k) {
                const int32_t p = fill[col[k]]++;
                rsrc[p] = u;
                rcost[p] = cost[k];
                rdrift[p] = drift[k];
                rperm[p] = k;
            }
    }
    std::vector<uint8_t> flag(n);
    std::vector<int32_t> glist;
    for (int32_t v = 0; v < n; ++v) {
        flag[v] = (uint8_t)((reset[v] ? 1u : 0u) | (goal[v] ? 2u : 0u));
        if (goal[v]) glist.push_back(v);
    }
    mpap_graph *g = new mpap_graph();
    g->dev = di.dev;
    g->n = n;
    g->e = e;
    g->n_goal = (int32_t)glist.size();
    auto bail = [&](int st) { graph_release(g); return st; };
    if ((r = dalloc(&g->optr, n + 1)) || (r = dalloc(&g->ocol, e)) ||
        (r = dalloc(&g->ocost, e)) || (r = dalloc(&g->odrift, e)) ||
        (r = dalloc(&g->rptr, n + 1)) || (r = dalloc(&g->rsrc, e)) ||
        (r = dalloc(&g->rcost, e)) || (r = dalloc(&g->rdrift, e)) ||
        (r = dalloc(&g->nflag, n)) || (r = dalloc(&g->goal_list, glist.size())) ||
        (r = dalloc(&g->rperm, e)))
        return bail(r);
    hipError_t he = hipSuccess;
    auto cp = [&](void *d, const void *h, size_t bytes) {
        if (he == hipSuccess && bytes) he = hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s);
    };
    cp(g->rperm, rperm.data(), sizeof(int32_t) * e);
    cp(g->optr, row_ptr, sizeof(int32_t) * (n + 1));
    cp(g->ocol, col, sizeof(int32_t) * e);
    cp(g->ocost, cost, sizeof(float) * e);
    cp(g->odrift, drift, sizeof(float) * e);
    cp(g->rptr, rptr.data(), sizeof(int32_t) * (n + 1));
    cp(g->rsrc, rsrc.data(), sizeof(int32_t) * e);
    cp(g->rcost, rcost.data(), sizeof(float) * e);
    cp(g->rdrift, rdrift.data(), sizeof(float) * e);
    cp(g->nflag, flag.data(), n);
    cp(g->goal_list, glist.data(), sizeof(int32_t) * glist.size());
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) {
        graph_release(g);
        return fail(MPAP_ERR_HIP, std::string("graph upload: ") + hipGetErrorString(he));
    }
    if ((r = graph_set_single_query(g))) return bail(r);
    *out = g;
    return MPAP_OK;
}

// ------------------------------------------------------------- graph build
}  // extern "C"

// Double-integrator roadmap: steering selection, compaction, drift on the
// device; the in-edge lists are built by the import path.
static int build_graph6(const mpap_env *env, const mpap_graph_params *gp, void *stream,
                        mpap_graph **out) {
    const int n = env->n_nodes;
    if (n < 2 || !env->vel) return fail(MPAP_ERR_INVAL, "dim 6 needs n >= 2 and velocities");
    if (gp->k_out < 1 || gp->k_out > kSteerMaxOut)
        return fail(MPAP_ERR_INVAL, "k_out must be in 1..64");
    if (!(gp->horizon > 0.0f) || !std::isfinite(gp->horizon))
        return fail(MPAP_ERR_INVAL, "horizon must be finite and > 0");
    if (gp->traj_steps < 1 || gp->traj_steps > kSteerMaxSteps)
        return fail(MPAP_ERR_INVAL, "traj_steps must be in 1..255");
    if (!(gp->radius > 0.0f) || !std::isfinite(gp->radius))
        return fail(MPAP_ERR_INVAL, "radius (the group step) must be finite and > 0");
    if (env->n_boxes < 0 || env->n_boxes > 1024 || env->n_blobs < 0 ||
        (env->n_boxes > 0 && (!env->box_lo || !env->box_hi)) ||
        (env->n_blobs > 0 && (!env->blob_mu || !env->blob_sigma || !env->blob_amp)))
        return fail(MPAP_ERR_INVAL, "bad obstacle or blob arrays (at most 1024 boxes)");
    for (long long i = 0; i < 3ll * n; ++i)
        if (!std::isfinite(env->pos[i]) || !std::isfinite(env->vel[i]))
            return fail(MPAP_ERR_INVAL, "non-finite state");
    for (int j = 0; j < env->n_blobs; ++j)
        if (!(env->blob_sigma[j] > 0.0f)) return fail(MPAP_ERR_INVAL, "blob sigma must be > 0");
    DeviceInfo di;
    int r = device_info(&di);
    if (r) return r;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int k_out = gp->k_out;
    const size_t nb_ = (size_t)env->n_boxes * 3, nf_ = env->n_blobs;
    float *d_pos = nullptr, *d_vel = nullptr, *d_blo = nullptr, *d_bhi = nullptr, *d_mu = nullptr,
          *d_sig = nullptr, *d_amp = nullptr, *ncost = nullptr, *cost = nullptr, *drift = nullptr,
          *elen = nullptr;
    int *nbr = nullptr, *ncnt = nullptr, *rp = nullptr, *col = nullptr, *tmp = nullptr,
        *err = nullptr;
    uint8_t *flag = nullptr;
    auto cleanup = [&]() {
        dfree(d_pos); dfree(d_vel); dfree(d_blo); dfree(d_bhi); dfree(d_mu); dfree(d_sig);
        dfree(d_amp); dfree(ncost); dfree(cost); dfree(drift); dfree(elen); dfree(nbr);
        dfree(ncnt); dfree(rp); dfree(col); dfree(tmp); dfree(err); dfree(flag);
    };
    auto bail = [&](int st) {
        cleanup();
        return st;
    };
    if ((r = dalloc(&d_pos, 3 * (size_t)n)) || (r = dalloc(&d_vel, 3 * (size_t)n)) ||
        (r = dalloc(&d_blo, nb_)) || (r = dalloc(&d_bhi, nb_)) || (r = dalloc(&d_mu, 3 * nf_)) ||
        (r = dalloc(&d_sig, nf_)) || (r = dalloc(&d_amp, nf_)) ||
        (r = dalloc(&nbr, (size_t)n * k_out)) || (r = dalloc(&ncost, (size_t)n * k_out)) ||
        (r = dalloc(&ncnt, n)) || (r = dalloc(&rp, n + 1)) || (r = dalloc(&err, 1)) ||
        (r = dalloc(&flag, n)) || (r = dalloc(&tmp, div_up(n + 1, kScanTile) + 1)))
        return bail(r);
    hipError_t he = hipSuccess;
    auto cp = [&](void *d, const void *h, size_t bytes) {
        if (he == hipSuccess && bytes) he = hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s);
    };
    const int zero = 0;
    cp(d_pos, env->pos, sizeof(float) * 3 * n);
    cp(d_vel, env->vel, sizeof(float) * 3 * n);
    cp(d_blo, env->box_lo, sizeof(float) * nb_);
    cp(d_bhi, env->box_hi, sizeof(float) * nb_);
    cp(d_mu, env->blob_mu, sizeof(float) * 3 * nf_);
    cp(d_sig, env->blob_sigma, sizeof(float) * nf_);
    cp(d_amp, env->blob_amp, sizeof(float) * nf_);
    cp(err, &zero, sizeof(int));
    if (he != hipSuccess) return bail(fail(MPAP_ERR_HIP, hipGetErrorString(he)));

    SteerArgs a{};
    a.n = n; a.pos = d_pos; a.vel = d_vel; a.nbox = env->n_boxes; a.blo = d_blo; a.bhi = d_bhi;
    a.nblob = env->n_blobs; a.mu = d_mu; a.sig = d_sig; a.amp = d_amp;
    a.T = gp->horizon; a.K = gp->traj_steps; a.k_out = k_out;
    const size_t lds = sizeof(int) * 2048 + 2 * (size_t)kSteerMaxWidth * 8 +
                       sizeof(float) * 6 * (size_t)env->n_boxes +
                       sizeof(int) * (kSteerThreads / 64) * (size_t)env->n_boxes;
    k_steer_select<<<n, kSteerThreads, lds, s>>>(a, nbr, ncost, ncnt, err);
    HIP_TRY(hipGetLastError());
    // row pointers: exclusive scan of the counts, total in rp[n]
    if ((r = scan_i32(ncnt, rp, n, tmp, s))) return bail(r);
    int last_cnt = 0, last_off = 0, herr = 0;
    HIP_TRY(hipMemcpyAsync(&last_cnt, ncnt + (n - 1), sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&last_off, rp + (n - 1), sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (herr) return bail(fail(MPAP_ERR_OVERFLOW, "too many candidates share one steering cost"));
    const long long e = (long long)last_cnt + last_off;
    const int e32 = (int)e;
    HIP_TRY(hipMemcpy(rp + n, &e32, sizeof(int), hipMemcpyHostToDevice));
    if ((r = dalloc(&col, std::max(e, 1ll))) || (r = dalloc(&cost, std::max(e, 1ll))) ||
        (r = dalloc(&drift, std::max(e, 1ll))) || (r = dalloc(&elen, std::max(e, 1ll))))
        return bail(r);
    k_steer_compact<<<div_up(n, 256), 256, 0, s>>>(n, k_out, rp, nbr, ncost, ncnt, col, cost);
    k_traj_drift<<<n, 64, sizeof(float) * 5 * nf_, s>>>(a, rp, col, drift, elen);
    {
        BuildArgs b{};
        b.n = n; b.dim = 3; b.pos = d_pos; b.nblob = env->n_blobs; b.mu = d_mu; b.sig = d_sig;
        b.amp = d_amp; b.reset_q = gp->reset_q;
        b.goal[0] = env->goal[0]; b.goal[1] = env->goal[1]; b.goal[2] = env->goal[2];
        b.goal_r = env->goal_radius;
        k_node_flags<<<div_up(n, 256), 256, 0, s>>>(b, flag);
    }
    HIP_TRY(hipGetLastError());
    std::vector<int32_t> h_rp(n + 1), h_col(e);
    std::vector<float> h_cost(e), h_drift(e);
    std::vector<uint8_t> h_flag(n), h_reset(n), h_goal(n);
    HIP_TRY(hipMemcpyAsync(h_rp.data(), rp, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, s));
    if (e > 0) {
        HIP_TRY(hipMemcpyAsync(h_col.data(), col, sizeof(int32_t) * e, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(h_cost.data(), cost, sizeof(float) * e, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(h_drift.data(), drift, sizeof(float) * e, hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipMemcpyAsync(h_flag.data(), flag, n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int n_goal = 0;
    for (int v = 0; v < n; ++v) {
        h_reset[v] = h_flag[v] & 1u;
        h_goal[v] = (h_flag[v] >> 1) & 1u;
        n_goal += h_goal[v];
    }
    if (n_goal == 0) return bail(fail(MPAP_ERR_NOGOAL, "no roadmap node lies in the goal ball"));
    mpap_graph *g = nullptr;
    if ((r = mpap_graph_from_csr(n, h_rp.data(), h_col.data(), h_cost.data(), h_drift.data(),
                                 h_reset.data(), h_goal.data(), stream, &g)))
        return bail(r);
    // keep the environment for the surrogate's inputs
    g->dim = 6; g->nbox = env->n_boxes; g->nblob = env->n_blobs;
    g->check_step = gp->check_step; g->reset_q = gp->reset_q; g->radius = gp->radius;
    g->horizon = gp->horizon; g->traj_steps = gp->traj_steps; g->k_out = k_out;
    g->pos = d_pos; g->vel = d_vel; g->bmu = d_mu; g->bsig = d_sig; g->bamp = d_amp;
    g->blo = d_blo; g->bhi = d_bhi;
    g->elen = elen;
    d_pos = d_vel = d_mu = d_sig = d_amp = elen = d_blo = d_bhi = nullptr;
    cleanup();
    *out = g;
    return MPAP_OK;
}

extern "C" {
int mpap_build_graph(const mpap_env *env, const mpap_graph_params *gp, void *stream,
                     mpap_graph **out) {
    if (!out) return fail(MPAP_ERR_INVAL, "out is null");
    *out = nullptr;
    if (!env || !gp || !env->pos) return fail(MPAP_ERR_INVAL, "null env, params or positions");
    const int dim = env->dim, n = env->n_nodes;
    if (dim == 6) return build_graph6(env, gp, stream, out);
    if ((dim != 2 && dim != 3) || n < 1) return fail(MPAP_ERR_INVAL, "dim must be 2, 3 or 6, n >= 1");
    if (!(gp->radius > 0.0f) || !(gp->check_step > 0.0f) || !std::isfinite(gp->radius))
        return fail(MPAP_ERR_INVAL, "radius and check_step must be > 0");
    if (env->n_boxes < 0 || env->n_blobs < 0 ||
        (env->n_boxes > 0 && (!env->box_lo || !env->box_hi)) ||
        (env->n_blobs > 0 && (!env->blob_mu || !env->blob_sigma || !env->blob_amp)))
        return fail(MPAP_ERR_INVAL, "null obstacle or blob arrays");
    if (gp->near_grid < -1 || gp->near_grid > 1)
        return fail(MPAP_ERR_INVAL, "near_grid must be -1, 0 or 1");
    float plo[3] = {0.f, 0.f, 0.f}, phi[3] = {0.f, 0.f, 0.f};
    for (int k = 0; k < dim; ++k) plo[k] = phi[k] = env->pos[k];
    for (long long i = 0; i < (long long)n * dim; ++i) {
        const float x = env->pos[i];
        if (!std::isfinite(x)) return fail(MPAP_ERR_INVAL, "non-finite position");
        plo[i % dim] = std::min(plo[i % dim], x);
        phi[i % dim] = std::max(phi[i % dim], x);
    }
    for (int j = 0; j < env->n_blobs; ++j)
        if (!(env->blob_sigma[j] > 0.0f)) return fail(MPAP_ERR_INVAL, "blob sigma must be > 0");
    // Grid for Near: cells of edge h >= r (1 + 2^-7), at most 16,000 per axis
    // and max(64, min(2n, 2^30)) in all.  The 2^-7 margin covers the float32 roundings
    // of Cost and of the cell coordinates (relative errors of a few 2^-24
    // at coordinates below 16,384 cells), so a pair with Cost < r is never
    // more than one cell apart on any axis.
    GridArgs gr{};
    gr.gx = gr.gy = gr.gz = 1;
    bool use_grid = false;
    if (gp->near_grid >= 0) {
        double h = (double)gp->radius * (1.0 + 1.0 / 128.0);
        for (int k = 0; k < dim; ++k) h = std::max(h, ((double)phi[k] - plo[k]) / 16000.0);
        const double cap = std::max(64.0, std::min(2.0 * n, 1073741824.0));
        int cells[3] = {1, 1, 1};
        for (;;) {
            double tot = 1.0;
            for (int k = 0; k < dim; ++k) {
                cells[k] = (int)(std::floor(((double)phi[k] - plo[k]) / h) + 1.0);
                tot *= cells[k];
            }
            if (tot <= cap) break;
            h *= 1.25;
        }
        gr.gx = cells[0]; gr.gy = cells[1]; gr.gz = cells[2];
        gr.ncell = gr.gx * gr.gy * gr.gz;
        for (int k = 0; k < 3; ++k) gr.lo[k] = plo[k];
        gr.inv = (float)(1.0 / h);
        // chosen when the adjacent cells are a small part of the box
        const int adj = dim == 3 ? 27 : 9;
        use_grid = gp->near_grid == 1 || (n >= 512 && gr.ncell >= 4 * adj);
    }
    DeviceInfo di;
    int r = device_info(&di);
    if (r) return r;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    float *d_pos = nullptr, *d_blo = nullptr, *d_bhi = nullptr, *d_mu = nullptr,
          *d_sig = nullptr, *d_amp = nullptr, *cand_c = nullptr;
    int *cnt = nullptr, *coff = nullptr, *cand_u = nullptr, *cand_v = nullptr, *keep = nullptr,
        *kscan = nullptr, *tmp = nullptr, *ngoal = nullptr, *gcell = nullptr, *gslot = nullptr,
        *maxc = nullptr;
    mpap_graph *g = nullptr;
    auto cleanup = [&]() {
        dfree(d_pos); dfree(d_blo); dfree(d_bhi); dfree(d_mu); dfree(d_sig); dfree(d_amp);
        dfree(cand_c); dfree(cnt); dfree(coff); dfree(cand_u); dfree(cand_v); dfree(keep);
        dfree(kscan); dfree(tmp); dfree(ngoal); dfree(gcell); dfree(gslot); dfree(maxc);
        dfree(gr.ccount); dfree(gr.cstart); dfree(gr.sid); dfree(gr.spos);
    };
    auto bail = [&](int st) {
        cleanup();
        if (g) graph_release(g);
        return st;
    };
    const size_t nb_ = (size_t)env->n_boxes * dim, nf_ = (size_t)env->n_blobs;
    if ((r = dalloc(&d_pos, (size_t)n * dim)) || (r = dalloc(&d_blo, nb_)) ||
        (r = dalloc(&d_bhi, nb_)) || (r = dalloc(&d_mu, nf_ * dim)) ||
        (r = dalloc(&d_sig, nf_)) || (r = dalloc(&d_amp, nf_)) || (r = dalloc(&cnt, n)) ||
        (r = dalloc(&coff, n)) ||
        (r = dalloc(&tmp, div_up(std::max({n, gr.ncell, 1}), kScanTile) + 1)) ||
        (r = dalloc(&ngoal, 1)))
        return bail(r);
    if (use_grid &&
        ((r = dalloc(&gcell, n)) || (r = dalloc(&gslot, n)) || (r = dalloc(&maxc, 1)) ||
         (r = dalloc(&gr.ccount, gr.ncell)) || (r = dalloc(&gr.cstart, gr.ncell)) ||
         (r = dalloc(&gr.sid, n)) || (r = dalloc(&gr.spos, n))))
        return bail(r);
    hipError_t he = hipSuccess;
    auto cp = [&](void *d, const void *h, size_t bytes) {
        if (he == hipSuccess && bytes) he = hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s);
    };
    cp(d_pos, env->pos, sizeof(float) * n * dim);
    cp(d_blo, env->box_lo, sizeof(float) * nb_);
    cp(d_bhi, env->box_hi, sizeof(float) * nb_);
    cp(d_mu, env->blob_mu, sizeof(float) * nf_ * dim);
    cp(d_sig, env->blob_sigma, sizeof(float) * nf_);
    cp(d_amp, env->blob_amp, sizeof(float) * nf_);
    if (he != hipSuccess) return bail(fail(MPAP_ERR_HIP, hipGetErrorString(he)));

    BuildArgs a{};
    a.n = n; a.dim = dim; a.pos = d_pos; a.nbox = env->n_boxes; a.blo = d_blo; a.bhi = d_bhi;
    a.nblob = env->n_blobs; a.mu = d_mu; a.sig = d_sig; a.amp = d_amp;
    a.r = gp->radius; a.step = gp->check_step; a.reset_q = gp->reset_q;
    a.goal[0] = env->goal[0]; a.goal[1] = env->goal[1]; a.goal[2] = env->goal[2];
    a.goal_r = env->goal_radius;

    const int nblk = div_up(n, 256);
    if (use_grid) {
        k_zero_i32<<<div_up(gr.ncell, 256), 256, 0, s>>>(gr.ccount, gr.ncell);
        k_zero_i32<<<1, 256, 0, s>>>(maxc, 1);
        k_grid_bin<<<nblk, 256, 0, s>>>(a, gr, gcell, gslot);
        if ((r = scan_i32(gr.ccount, gr.cstart, gr.ncell, tmp, s))) return bail(r);
        k_grid_scatter<<<nblk, 256, 0, s>>>(a, gr, gcell, gslot);
        k_near_count_grid<<<nblk, 256, 0, s>>>(a, gr, cnt, maxc);
    } else {
        k_near_count<<<nblk, 256, 0, s>>>(a, cnt);
    }
    if ((r = scan_i32(cnt, coff, n, tmp, s))) return bail(r);
    int last_cnt = 0, last_off = 0, max_row = 0;
    HIP_TRY(hipMemcpyAsync(&last_cnt, cnt + (n - 1), sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&last_off, coff + (n - 1), sizeof(int), hipMemcpyDeviceToHost, s));
    if (use_grid)
        HIP_TRY(hipMemcpyAsync(&max_row, maxc, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const long long m = (long long)last_cnt + last_off;
    if ((r = dalloc(&cand_u, m)) || (r = dalloc(&cand_v, m)) || (r = dalloc(&cand_c, m)) ||
        (r = dalloc(&keep, m)) || (r = dalloc(&kscan, m)))
        return bail(r);
    dfree(tmp);
    if ((r = dalloc(&tmp, div_up(std::max(m, 1LL), kScanTile) + 1))) return bail(r);
    if (use_grid && max_row <= kGridSortMax) {
        k_near_fill_grid<<<nblk, 256, 0, s>>>(a, gr, coff, cand_u, cand_v, cand_c);
        k_sort_rows<<<div_up(n, 4), 256, 0, s>>>(n, coff, cnt, cand_v, cand_c);
    } else
        k_near_fill<<<nblk, 256, 0, s>>>(a, coff, cand_u, cand_v, cand_c);
    if (m > 0) {
        const size_t lds = sizeof(float) * 2 * nb_;
        k_collide<<<div_up(m, 256), 256, lds, s>>>(a, m, cand_u, cand_v, cand_c, keep);
        if ((r = scan_i32(keep, kscan, m, tmp, s))) return bail(r);
    }
    int last_keep = 0, last_ks = 0;
    if (m > 0) {
        HIP_TRY(hipMemcpyAsync(&last_keep, keep + (m - 1), sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&last_ks, kscan + (m - 1), sizeof(int), hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    const long long e = (long long)last_keep + last_ks;

    g = new mpap_graph();
    g->dev = di.dev;
    g->n = n;
    g->e = e;
    g->symmetric_alias = true;
    if ((r = dalloc(&g->optr, n + 1)) || (r = dalloc(&g->ocol, e)) ||
        (r = dalloc(&g->ocost, e)) || (r = dalloc(&g->odrift, e)) ||
        (r = dalloc(&g->nflag, n)) || (r = dalloc(&g->goal_list, n)))
        return bail(r);
    if (m > 0)
        k_compact_edges<<<div_up(m, 256), 256, 0, s>>>(m, keep, kscan, cand_v, cand_c, g->ocol,
                                                       g->ocost);
    k_row_ptr<<<div_up(n + 1, 256), 256, 0, s>>>(n, m, coff, kscan, keep, g->optr);
    if ((r = build_pair_index(g, s))) return bail(r);
    {
        // one thread per id-ordered pair, both directions written
        const size_t lds = sizeof(float) * (nf_ * dim + 2 * nf_);
        if (n > 0 && g->e > 0)
            k_edge_drift_pairs<<<div_up(g->e / 2 + 1, 256), 256, lds, s>>>(
                a, n, g->optr, g->ocol, g->ocost, g->uptr, g->odrift);
    }
    k_node_flags<<<nblk, 256, 0, s>>>(a, g->nflag);
    k_flag_list<<<1, 1024, 0, s>>>(n, g->nflag, 2u, g->goal_list, ngoal);
    HIP_TRY(hipGetLastError());
    int hg = 0;
    HIP_TRY(hipMemcpyAsync(&hg, ngoal, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    g->n_goal = hg;
    // the roadmap is symmetric (same cost, drift and collision result both
    // ways), so the in-edge lists are the out-edge lists
    g->rptr = g->optr; g->rsrc = g->ocol; g->rcost = g->ocost; g->rdrift = g->odrift;
    // keep the environment for the surrogate's inputs
    g->dim = dim; g->nbox = env->n_boxes; g->nblob = env->n_blobs;
    g->check_step = gp->check_step; g->reset_q = gp->reset_q; g->radius = gp->radius;
    g->pos = d_pos; g->bmu = d_mu; g->bsig = d_sig; g->bamp = d_amp;
    g->blo = d_blo; g->bhi = d_bhi;
    d_pos = d_mu = d_sig = d_amp = d_blo = d_bhi = nullptr;
    cleanup();
    if (hg == 0) {
        graph_release(g);
        return fail(MPAP_ERR_NOGOAL, "no roadmap node lies in the goal ball");
    }
    if ((r = graph_set_single_query(g))) {
        graph_release(g);
        return r;
    }
    *out = g;
    return MPAP_OK;
}

int mpap_graph_info(const mpap_graph *g, int32_t *n, int64_t *e, int32_t *n_goal) {
    if (!g) return fail(MPAP_ERR_INVAL, "graph is null");
    if (n) *n = g->n;
    if (e) *e = g->e;
    if (n_goal) *n_goal = g->n_goal;
    return MPAP_OK;
}

int mpap_graph_queries(const mpap_graph *g, int32_t *nq, int32_t *node_offset) {
    if (!g || !nq) return fail(MPAP_ERR_INVAL, "null argument");
    *nq = g->nq;
    if (node_offset)
        for (int q = 0; q <= g->nq; ++q) node_offset[q] = g->qoff_h[q];
    return MPAP_OK;
}

int mpap_graph_concat(const mpap_graph *const *parts, int32_t n_parts, void *stream,
                      mpap_graph **out) {
    if (!out) return fail(MPAP_ERR_INVAL, "out is null");
    *out = nullptr;
    if (!parts || n_parts < 1) return fail(MPAP_ERR_INVAL, "need at least one part");
    long long n = 0, e = 0, ng = 0;
    bool alias = true;
    for (int i = 0; i < n_parts; ++i) {
        if (!parts[i]) return fail(MPAP_ERR_INVAL, "null part");
        n += parts[i]->n;
        e += parts[i]->e;
        ng += parts[i]->n_goal;
        alias = alias && parts[i]->symmetric_alias;
    }
    if (n > 0x7fffffffll || e > 0x7fffffffll)
        return fail(MPAP_ERR_INVAL, "concatenated roadmap exceeds int32 ids");
    DeviceInfo di;
    int r = device_info(&di);
    if (r) return r;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    mpap_graph *g = new mpap_graph();
    g->dev = di.dev;
    g->n = (int32_t)n;
    g->e = e;
    g->n_goal = (int32_t)ng;
    g->symmetric_alias = alias;
    auto bail = [&](int st) { graph_release(g); return st; };
    if ((r = dalloc(&g->optr, n + 1)) || (r = dalloc(&g->ocol, e)) ||
        (r = dalloc(&g->ocost, e)) || (r = dalloc(&g->odrift, e)) ||
        (r = dalloc(&g->nflag, n)) || (r = dalloc(&g->goal_list, ng)))
        return bail(r);
    if (alias) {
        g->rptr = g->optr; g->rsrc = g->ocol; g->rcost = g->ocost; g->rdrift = g->odrift;
    } else if ((r = dalloc(&g->rptr, n + 1)) || (r = dalloc(&g->rsrc, e)) ||
               (r = dalloc(&g->rcost, e)) || (r = dalloc(&g->rdrift, e))) {
        return bail(r);
    }
    g->qoff_h.assign(1, 0);
    g->qgoff_h.assign(1, 0);
    bool all_sur = true;
    for (int i = 0; i < n_parts; ++i) all_sur = all_sur && parts[i]->sdrift != nullptr;
    if (all_sur && alias && (r = dalloc(&g->sdrift, e))) return bail(r);
    long long no = 0, eo = 0, go = 0;
    for (int i = 0; i < n_parts; ++i) {
        const mpap_graph *p = parts[i];
        auto cpy = [&](void *d, const void *src, size_t bytes) -> int {
            if (bytes) HIP_TRY(hipMemcpyAsync(d, src, bytes, hipMemcpyDeviceToDevice, s));
            return MPAP_OK;
        };
        if ((r = cpy(g->optr + no, p->optr, sizeof(int32_t) * (p->n + 1))) ||
            (r = cpy(g->ocol + eo, p->ocol, sizeof(int32_t) * p->e)) ||
            (r = cpy(g->ocost + eo, p->ocost, sizeof(float) * p->e)) ||
            (r = cpy(g->odrift + eo, p->odrift, sizeof(float) * p->e)) ||
            (r = cpy(g->nflag + no, p->nflag, p->n)) ||
            (r = cpy(g->goal_list + go, p->goal_list, sizeof(int32_t) * p->n_goal)) ||
            (g->sdrift && (r = cpy(g->sdrift + eo, p->sdrift, sizeof(float) * p->e))))
            return bail(r);
        k_add_i32<<<std::max(1, div_up(p->n + 1, 256)), 256, 0, s>>>(g->optr + no, p->n + 1, (int)eo);
        if (p->e > 0) k_add_i32<<<div_up(p->e, 256), 256, 0, s>>>(g->ocol + eo, p->e, (int)no);
        if (p->n_goal > 0)
            k_add_i32<<<div_up(p->n_goal, 256), 256, 0, s>>>(g->goal_list + go, p->n_goal, (int)no);
        if (!alias) {
            if ((r = cpy(g->rptr + no, p->rptr, sizeof(int32_t) * (p->n + 1))) ||
                (r = cpy(g->rsrc + eo, p->rsrc, sizeof(int32_t) * p->e)) ||
                (r = cpy(g->rcost + eo, p->rcost, sizeof(float) * p->e)) ||
                (r = cpy(g->rdrift + eo, p->rdrift, sizeof(float) * p->e)))
                return bail(r);
            k_add_i32<<<std::max(1, div_up(p->n + 1, 256)), 256, 0, s>>>(g->rptr + no, p->n + 1, (int)eo);
            if (p->e > 0) k_add_i32<<<div_up(p->e, 256), 256, 0, s>>>(g->rsrc + eo, p->e, (int)no);
        }
        HIP_TRY(hipGetLastError());
        // the part's own query partition, shifted
        for (int q = 0; q < p->nq; ++q) {
            g->qoff_h.push_back((int32_t)(no + p->qoff_h[q + 1]));
            g->qgoff_h.push_back((int32_t)(go + p->qgoff_h[q + 1]));
        }
        // each part's last row pointer must be written after the next part's first
        HIP_TRY(hipStreamSynchronize(s));
        no += p->n;
        eo += p->e;
        go += p->n_goal;
    }
    g->nq = (int32_t)g->qoff_h.size() - 1;
    if ((r = dalloc(&g->qoff, g->nq + 1)) || (r = dalloc(&g->qgoff, g->nq + 1))) return bail(r);
    HIP_TRY(hipMemcpy(g->qoff, g->qoff_h.data(), sizeof(int32_t) * (g->nq + 1), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(g->qgoff, g->qgoff_h.data(), sizeof(int32_t) * (g->nq + 1), hipMemcpyHostToDevice));
    *out = g;
    return MPAP_OK;
}

int mpap_graph_export(const mpap_graph *g, int32_t *row_ptr, int32_t *col, float *cost,
                      float *drift, uint8_t *reset, uint8_t *goal) {
    if (!g || !row_ptr || !reset || !goal || (g->e > 0 && (!col || !cost || !drift)))
        return fail(MPAP_ERR_INVAL, "null argument");
    HIP_TRY(hipMemcpy(row_ptr, g->optr, sizeof(int32_t) * (g->n + 1), hipMemcpyDeviceToHost));
    if (g->e > 0) {
        HIP_TRY(hipMemcpy(col, g->ocol, sizeof(int32_t) * g->e, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(cost, g->ocost, sizeof(float) * g->e, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(drift, g->odrift, sizeof(float) * g->e, hipMemcpyDeviceToHost));
    }
    std::vector<uint8_t> f(g->n);
    HIP_TRY(hipMemcpy(f.data(), g->nflag, g->n, hipMemcpyDeviceToHost));
    for (int32_t v = 0; v < g->n; ++v) {
        reset[v] = f[v] & 1u;
        goal[v] = (f[v] >> 1) & 1u;
    }
    return MPAP_OK;
}

void mpap_graph_free(mpap_graph *g) {
    if (g) graph_release(g);
}

// ----------------------------------------------------------------- search
}  // extern "C"

int search_prep(const mpap_graph *g, const mpap_search_params *sp, int32_t nsp, SearchPrep &p) {
    const int nq = g->nq;
    if (nsp != nq && nsp != 1)
        return fail(MPAP_ERR_INVAL, "need one parameter set per query (or one for all)");
    // merge-target list regions are indexed in int32
    if ((long long)g->n * kListRegions > 0x7fffffffll)
        return fail(MPAP_ERR_INVAL, "graph too large for one search (nodes x 11 >= 2^31)");
    p = SearchPrep{};
    p.nq = nq;
    for (int q = 0; q < nsp; ++q) {
        const mpap_search_params &x = sp[q];
        const int qn = g->qoff_h[(nsp == 1 ? 0 : q) + 1] - g->qoff_h[nsp == 1 ? 0 : q];
        if (x.n_obj != 2 && x.n_obj != 3) return fail(MPAP_ERR_INVAL, "n_obj must be 2 or 3");
        if (x.init_node < 0 || x.init_node >= qn) return fail(MPAP_ERR_INVAL, "init_node out of range");
        if (!(x.lambda > 0.0f) || !(x.radius > 0.0f) || std::isnan(x.beta))
            return fail(MPAP_ERR_INVAL, "lambda and radius must be > 0, beta not NaN");
        const float dq = x.lambda * x.radius;
        if (!(dq > 0.0f) || !std::isfinite(dq))
            return fail(MPAP_ERR_INVAL, "lambda * radius must be finite and > 0");
        p.max_waves = std::max(p.max_waves, x.max_waves);
        if (x.near_scan > 0) p.near_scan = x.near_scan;
        if (x.heuristic != 0 && x.heuristic != 1)
            return fail(MPAP_ERR_INVAL, "heuristic must be 0 (analytic) or 1 (surrogate)");
        if (x.stage_cap > 0) p.stage_cap = x.stage_cap;
        if (x.block_threads != 0 && x.block_threads != 256 && x.block_threads != 512 &&
            x.block_threads != 1024)
            return fail(MPAP_ERR_INVAL, "block_threads must be 0, 256, 512 or 1024");
        if (x.block_threads != 0) p.block_threads = x.block_threads;
        if (x.wave_min_targets != 0) p.wave_min_targets = x.wave_min_targets;
        if (x.merge_halves != 0) p.merge_halves = x.merge_halves;
        if (x.skip != 0 && x.skip != 1) return fail(MPAP_ERR_INVAL, "skip must be 0 or 1");
        if (x.early_stop != 0 && x.early_stop != 1)
            return fail(MPAP_ERR_INVAL, "early_stop must be 0 or 1");
    }
    if (p.max_waves <= 0) p.max_waves = 1 << 18;
    if (nsp == 1 && nq > 1) {
        for (int q = 1; q < nq; ++q)
            if (sp[0].init_node >= g->qoff_h[q + 1] - g->qoff_h[q])
                return fail(MPAP_ERR_INVAL, "init_node out of range for a query");
    }
    p.beta.resize(nq);
    p.delta.resize(nq);
    p.nobj.resize(nq);
    p.root.resize(nq);
    p.heur.resize(nq);
    p.skip.resize(nq);
    p.early.resize(nq);
    for (int q = 0; q < nq; ++q) {
        const mpap_search_params &x = sp[nsp == 1 ? 0 : q];
        p.beta[q] = x.beta;
        p.delta[q] = x.lambda * x.radius;
        p.nobj[q] = x.n_obj;
        p.root[q] = g->qoff_h[q] + x.init_node;
        p.heur[q] = x.heuristic;
        p.skip[q] = x.skip;
        p.early[q] = x.early_stop;
        p.early_any = p.early_any || x.early_stop != 0;
    }
    return MPAP_OK;
}

int search_shape(int stage_cap, int block_threads, int wave_min_targets, SearchShape &L,
                 int merge_halves) {
    DeviceInfo di;
    int r = device_info(&di);
    if (r) return r;
    // 1024, 512 or 256-thread workgroups, one, two or four per CU; LDS staging
    // sized from the device limit shared by the CU's workgroups
    L.threads = block_threads;
    const int per_cu_want = 1024 / L.threads;
    L.capC = std::min(1024, 4 * L.threads);  // a power of two, a multiple of the block size
    const size_t fixed = 16 * (size_t)L.capC + 16 * (size_t)L.threads + 8 * (size_t)L.capC +
                         128 + 32 + L.capC;
    // leave 1 KiB per workgroup for the kernel's static LDS
    const size_t lds_budget = std::min<size_t>(di.max_lds, 160 * 1024) / per_cu_want - 1024;
    if (lds_budget < fixed + 17 * 256 + 64) return fail(MPAP_ERR_DEVICE, "not enough LDS per block");
    // per staged label: 16 B + a flag byte; per 64 labels of the larger of the
    // front stage and the candidate chunk: two segment floats
    const size_t segc = 8 * ((size_t)L.capC / 64 + 2);
    if (lds_budget < fixed + segc + 17 * 256 + 64) return fail(MPAP_ERR_DEVICE, "not enough LDS per block");
    int capB = (int)(((lds_budget - fixed - segc - 16) * 64) / (17 * 64 + 8));
    capB = std::min(capB, 8 * L.threads);
    capB -= capB % 64;
    if (capB < 256) return fail(MPAP_ERR_DEVICE, "not enough LDS per block");
    L.lds = fixed + 17 * (size_t)capB + 8 * (size_t)(std::max(capB, L.capC) / 64 + 2);
    if (stage_cap > 0) capB = std::min(capB, std::max(stage_cap, 1));
    L.capB = capB;
    // single-wave merges: each wave's slice of the same LDS holds a front of
    // wcap labels (16 B + a flag byte each, two floats per 64), 64 children
    // and their flags
    L.wslice = (int)((L.lds / (size_t)(L.threads / 64)) & ~(size_t)15);
    {
        const long long room = (long long)L.wslice - 16 * 64 - 64 - 64;
        int wcap = room > 0 ? (int)((room * 64) / (17 * 64 + 8)) : 0;
        wcap -= wcap % 64;
        if (stage_cap > 0) wcap = std::min(wcap, stage_cap - stage_cap % 64);
        L.wcap = wcap >= 64 ? wcap : 0;
    }
    int per_cu = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_search, L.threads, L.lds));
    if (per_cu < 1) return fail(MPAP_ERR_DEVICE, "search kernel does not fit on a CU");
    L.nblocks = di.cus * std::min(per_cu, per_cu_want);
    // merges by halves: each half of a 1024-thread workgroup gets half the
    // LDS, a 512-label chunk and the largest front stage that fits
    // (in 512-thread workgroups, halves of 256 threads were slower: 3D 35.4
    // against 30.5 ms whole and 25.9 ms by halves of 1024-thread workgroups)
    if (merge_halves >= 0 && L.threads == 1024 && L.nblocks == di.cus) {
        const int ch = 512;
        const size_t half = (L.lds / 2) & ~(size_t)15;
        const size_t hfixed = 16 * (size_t)ch + 16 * 512 + 8 * (size_t)ch + 128 + 32 + ch;
        long long cb = half > hfixed + 16 ? (long long)(((half - hfixed - 16) * 64) / (17 * 64 + 8)) : 0;
        cb -= cb % 64;
        if (stage_cap > 0) cb = std::min<long long>(cb, std::max(stage_cap - stage_cap % 64, 64));
        const size_t need = hfixed + 17 * (size_t)cb + 8 * (size_t)(std::max<long long>(cb, ch) / 64 + 2);
        if (cb >= 1024 && need <= half) {
            L.halves = 1;
            L.half_lds = (int)half;
            L.capBh = (int)cb;
            L.capCh = ch;
            L.big_front = (int)(3 * cb / 4);
            L.big_children = merge_halves > 0 ? std::min(merge_halves, 1 << 24) : 8192;
            // iterations with fewer targets than eight per workgroup merge
            // by whole workgroups: each half would get a few, and one heavy
            // merge by a half sets the pace (two per workgroup when forced)
            L.halves_min = (merge_halves > 0 ? 2 : 8) * L.nblocks;
            L.halves_forced = merge_halves > 0;
        }
    }
    // by default a wave-per-target iteration needs four small targets per wave
    if (wave_min_targets < 0) L.wcap = 0;
    L.wmin = wave_min_targets > 0 ? wave_min_targets : 4 * L.nblocks * (L.threads / 64);
    L.explicit_wmin = wave_min_targets > 0;
    return MPAP_OK;
}

int search_upload(Workspace *w, const SearchPrep &p, hipStream_t s) {
    int r;
    if ((r = ws_queries(w, p.nq))) return r;
    const size_t nq = p.nq;
    // the six per-query arrays, staged in pinned memory (4-byte words each);
    // the staging is free again once the stream has passed these copies
    // (every caller synchronises the stream before it stages anything else)
    HIP_TRY(hipStreamSynchronize(s));
    // (and room after them for the status read-back of the search)
    if ((r = ws_pinned(w, (((size_t)24 * nq + 15) & ~(size_t)15) + 256))) return r;
    int *st = reinterpret_cast<int *>(w->hpin);
    float *stf = reinterpret_cast<float *>(w->hpin);
    for (size_t q = 0; q < nq; ++q) {
        st[q] = p.heur[q];
        stf[nq + q] = p.beta[q];
        stf[2 * nq + q] = p.delta[q];
        st[3 * nq + q] = p.nobj[q];
        st[4 * nq + q] = q < p.early.size() ? p.early[q] : 0;
        // a skipped query's root is not seeded (-1)
        st[5 * nq + q] = (q < p.skip.size() && p.skip[q]) ? -1 : p.root[q];
    }
    HIP_TRY(hipMemcpyAsync(w->qheur, st, sizeof(int) * nq, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(w->qbeta, stf + nq, sizeof(float) * nq, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(w->qdelta, stf + 2 * nq, sizeof(float) * nq, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(w->qnobj, st + 3 * nq, sizeof(int) * nq, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(w->qearly, st + 4 * nq, sizeof(int) * nq, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(w->qroot, st + 5 * nq, sizeof(int) * nq, hipMemcpyHostToDevice, s));
    return MPAP_OK;
}

SearchArgs search_args(const mpap_graph *g, Workspace *w, const SearchPrep &p,
                       const SearchShape &L) {
    SearchArgs a{};
    a.n = g->n; a.rptr = g->rptr; a.rsrc = g->rsrc; a.rcost = g->rcost;
    a.rdrift = g->rdrift; a.optr = g->optr; a.ocol = g->ocol; a.nflag = g->nflag;
    a.sdrift = g->symmetric_alias ? g->sdrift : g->srdrift; a.qheur = w->qheur;
    a.nq = p.nq; a.qoff = g->qoff; a.qbeta = w->qbeta; a.qnobj = w->qnobj;
    a.qroot = w->qroot; a.qlast = w->qlast;
    a.qdelta = w->qdelta; a.max_waves = p.max_waves; a.near_scan = p.near_scan;
    a.qgoff = g->qgoff; a.goal_list = g->goal_list; a.qearly = w->qearly; a.qstop = w->qstop;
    a.early_any = p.early_any ? 1 : 0;
    a.capB = L.capB; a.capC = L.capC; a.nblocks = L.nblocks;
    a.wcap = L.wcap; a.wslice = L.wslice; a.wmin = L.wmin;
    a.halves = L.halves; a.half_lds = L.half_lds; a.capBh = L.capBh; a.capCh = L.capCh;
    a.big_front = L.big_front; a.big_children = L.big_children; a.halves_min = L.halves_min;
    a.pool = w->pool; a.pool_cap = w->pool_cap; a.pool_top = w->pool_top; a.nb = w->nb;
    a.minopen = w->minopen; a.gcnt = w->gcnt; a.fo = w->fo; a.mark = w->mark; a.wt = w->wt;
    a.alist = w->alist; a.acnt = w->acnt; a.mcur = w->mcur; a.F = w->F; a.F_cap = w->F_cap;
    a.arena = w->arena; a.arena_cap = std::min<long long>(w->arena_cap, 0x7ffffff0ll);
    a.part_cnt = w->part_cnt; a.part_open = w->part_open; a.part_step = w->part_step;
    a.bar = w->bar; a.err = w->err; a.out = w->out;
    a.wstat = w->wstat; a.wstat_cap = kTraceCap;
    a.spill = w->spill; a.spill_flags = w->spill_flags; a.capG = (int)w->spill_cap;
    return a;
}

GoalArgs goal_args(const mpap_graph *g, Workspace *w) {
    GoalArgs ga{};
    ga.nq = g->nq; ga.qgoff = g->qgoff; ga.goal_list = g->goal_list;
    ga.lab_off = w->g_laboff; ga.lab_cap = w->g_labcap;
    ga.out_lab = w->g_out; ga.out_node = w->g_out_node; ga.out_count = w->g_count;
    ga.overflow = w->g_overflow;
    return ga;
}

void search_finish(mpap_result *res, const SearchPrep &p, const long long *dev_out,
                   const int *counts, const float4 *plab, const int *pnode, const int *qlast,
                   const int *qstop, const long long *trace, float ms, int retries,
                   const SearchShape &L) {
    const mpap_graph *g = res->g;
    const int nq = p.nq;
    res->n_obj = p.nobj.empty() ? 2 : p.nobj[0];
    res->qbeta = p.beta;
    res->qnobj = p.nobj;
    res->qheur = p.heur;
    res->qdelta = p.delta;
    res->qroot = p.root;
    res->max_waves = p.max_waves;
    res->near_scan = p.near_scan;
    res->stage_cap = p.stage_cap;
    res->block_threads = p.block_threads;
    res->wave_min_targets = p.wave_min_targets;
    res->merge_halves = p.merge_halves;
    res->front_off.assign(nq + 1, 0);
    for (int q = 0; q < nq; ++q) res->front_off[q + 1] = res->front_off[q] + counts[q];
    const long long tot = res->front_off[nq];
    res->front.assign(plab, plab + tot);
    res->front_node.assign(pnode, pnode + tot);
    // global goal node ids -> ids within the query
    for (int q = 0; q < nq; ++q)
        for (long long i = res->front_off[q]; i < res->front_off[q + 1]; ++i)
            res->front_node[i] -= g->qoff_h[q];
    res->qlast.assign(qlast, qlast + nq);
    res->qearly.assign(nq, 0);
    for (int q = 0; q < nq && q < (int)p.early.size(); ++q) res->qearly[q] = p.early[q];
    res->qstop.assign(nq, -1);
    for (int q = 0; q < nq; ++q) res->qstop[q] = qstop[q] >= 0 ? qstop[q] : -1;
    res->stats.waves = (int32_t)dev_out[kOutWaves];
    res->stats.retries = retries;
    res->stats.labels_expanded = dev_out[kOutLabels];
    res->arena_labels = dev_out[kOutLabels] + dev_out[kOutClosed];
    res->stats.front_labels = dev_out[kOutFront];
    res->stats.merges = dev_out[kOutMerges];
    res->stats.candidates = dev_out[kOutCandidates];
    res->stats.relaxations = dev_out[kOutRelax];
    res->stats.lds_front_cap = L.capB;
    res->stats.max_front = (int32_t)dev_out[kOutMaxFront];
    res->stats.blocks = L.nblocks;
    res->stats.wave_build = wave_build(L, g->n);
    res->stats.half_front_cap = !wave_build(L, g->n) && halves_build(L, g->n) ? L.capBh : 0;
    res->stats.build_objectives = wave_build(L, g->n) ? (L.obj == 2 ? 2 : 0) : L.obj;
    res->stats.half_merges = dev_out[kOutHalfMerges];
    res->stats.half_backouts = dev_out[kOutBackouts];
    res->stats.gpu_ms = ms;
    // per-query latency from the per-wave device clock (100 MHz)
    const int tw = std::min<int>(res->stats.waves, kTraceCap);
    res->trace.assign(trace, trace + (size_t)tw * kTraceWords);
    res->qlatency_ms.assign(nq, ms);
    if (tw > 0) {
        const int64_t t0 = res->trace[kTrStart];
        for (int q = 0; q < nq; ++q) {
            const int lw = res->qlast[q];
            if (lw >= 0 && lw < tw && res->trace[(size_t)lw * kTraceWords + kTrMerged] > 0)
                res->qlatency_ms[q] =
                    (float)((res->trace[(size_t)lw * kTraceWords + kTrMerged] - t0) * 1e-5);
        }
    }
}

int search_eager(mpap_graph *g, const SearchPrep &p, const SearchShape &L, Workspace *w,
                 hipStream_t s, mpap_result *res) {
    const int nq = p.nq;
    int r;
    if ((r = search_upload(w, p, s))) return r;
    // first guesses; a workspace keeps what earlier searches needed
    unsigned long long pool_cap = std::max<unsigned long long>(w->pool_cap, 256ull * g->n + 65536);
    long long arena_cap = std::max<long long>(w->arena_cap, 128ll * g->n + 65536);
    long long F_cap = std::max<long long>(w->F_cap, 32ll * g->n + 65536);
    pool_cap = std::min<unsigned long long>(pool_cap, (1ull << 31) - 1);
    long long capG = std::max<long long>(w->spill_cap, std::max(4 * L.capB, 32768));
    long long dev_out[kOutWords];
    int dev_err = 0;
    long long gtotal = 0;
    int retries = 0;
    float ms = 0.f;
    SearchArgs a{};
    // read-back staging after the uploads (search_upload sized it): status
    // words, error word, goal bound
    const size_t up = (24 * (size_t)nq + 15) & ~(size_t)15;
    static_assert(sizeof(long long) * kOutWords + 16 <= 256, "status read-back staging");
    for (;;) {
        if ((r = ws_grow(w, pool_cap, arena_cap, F_cap, 0))) return r;
        if ((r = ws_spill(w, capG))) return r;
        long long *h_out = reinterpret_cast<long long *>(w->hpin + up);
        int *h_err = reinterpret_cast<int *>(w->hpin + up + sizeof(dev_out));
        long long *h_total = reinterpret_cast<long long *>(w->hpin + up + sizeof(dev_out) + 8);
        a = search_args(g, w, p, L);
        k_search_init<<<div_up(g->n, 256), 256, 0, s>>>(a);
        k_search_roots<<<div_up(nq, 256), 256, 0, s>>>(a);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipEventRecord(w->ev0, s));
        void *kargs[] = {&a};
        HIP_TRY(hipLaunchCooperativeKernel(search_kernel_for(L, g->n),
                                           dim3(L.nblocks), dim3(L.threads), kargs, L.lds, s));
        HIP_TRY(hipEventRecord(w->ev1, s));
        if (p.early_any) k_close_stopped<<<1, 1024, 0, s>>>(a);
        k_count_front<<<std::max(1, std::min(div_up(g->n, 256), 1024)), 256, 0, s>>>(a);
        // the goal-front bound in the same pass (meaningful only when the
        // search completed)
        {
            GoalArgs ga = goal_args(g, w);
            k_zero_i32<<<div_up(nq, 256), 256, 0, s>>>(w->g_count, nq);
            k_zero_i32<<<1, 32, 0, s>>>(w->g_overflow, 1);
            k_goal_bound<<<1, 1024, 0, s>>>(a, ga, 0x7fffffffffffffffll, w->g_total);
        }
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(h_out, w->out, sizeof(dev_out), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(h_err, w->err, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(h_total, w->g_total, sizeof(long long), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        std::memcpy(dev_out, h_out, sizeof(dev_out));
        dev_err = *h_err;
        gtotal = *h_total;
        HIP_TRY(hipEventElapsedTime(&ms, w->ev0, w->ev1));
        const int status = (int)dev_out[kOutStatus];
        if (status == kStatusOk && dev_err == 0) break;
        if (dev_err & kErrTimeout)
            return fail(MPAP_ERR_HIP, "a grid or half-workgroup barrier wait timed out");
        if (dev_err & kErrTarget)
            return fail(MPAP_ERR_HIP, "internal error: a queued merge target is not a node");
        if (status == kStatusNoConverge)
            return fail(MPAP_ERR_NOCONVERGE, "max_waves reached with open plans");
        if (++retries > 12) return fail(MPAP_ERR_OVERFLOW, "capacity retries exhausted");
        if (dev_err & kErrBucket) {
            if (capG >= (1ll << 22))
                return fail(MPAP_ERR_OVERFLOW, "a per-node front exceeds 2^22 labels");
            capG *= 4;
        }
        if (dev_err & kErrPool) {
            if (w->pool_cap >= (1ull << 31) - 1)
                return fail(MPAP_ERR_OVERFLOW, "bucket pool beyond 2^31 labels");
            pool_cap = std::min<unsigned long long>(pool_cap * 4, (1ull << 31) - 1);
        }
        if (status == kStatusArena) {
            if (dev_out[kOutLabels] + dev_out[kOutNeed] > arena_cap) arena_cap *= 4;
            if (dev_out[kOutNeed] > F_cap) F_cap *= 4;
        }
    }

    return search_goal_finish(g, p, L, w, s, res, a, dev_out, ms, retries, gtotal);
}

int search_goal_finish(mpap_graph *g, const SearchPrep &p, const SearchShape &L, Workspace *w,
                       hipStream_t s, mpap_result *res, const SearchArgs &a,
                       const long long *dev_out, float ms, int retries, long long total) {
    const int nq = p.nq;
    int r;
    // goal fronts (a7): exact per-query regions, the fronts, then packed
    std::vector<int> counts(nq, 0), qlast(nq, 0), qstop(nq, -2);
    GoalArgs ga = goal_args(g, w);
    if (total < 0) {
        k_zero_i32<<<div_up(nq, 256), 256, 0, s>>>(w->g_count, nq);
        k_zero_i32<<<1, 32, 0, s>>>(w->g_overflow, 1);
        k_goal_bound<<<1, 1024, 0, s>>>(a, ga, 0x7fffffffffffffffll, w->g_total);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(&total, w->g_total, sizeof(long long), hipMemcpyDeviceToHost, s));
    }
    // (the stream is idle from here on until the launches below)
    HIP_TRY(hipStreamSynchronize(s));
    if ((r = ws_grow(w, 0, 0, 0, std::max<long long>(total, 1)))) return r;
    // the packed fronts fit in the per-query regions' total
    if ((r = ws_pack(w, std::max<long long>(total, 1)))) return r;
    const int tw = std::min<int>((int)dev_out[kOutWaves], kTraceCap);
    const size_t trace_words = (size_t)std::max(tw, 0) * kTraceWords;
    // staging: counts, qlast, qstop (nq ints each), then pool top, overflow,
    // error, then the trace
    const size_t o_small = 0, o_words = ((12 * (size_t)nq) + 15) & ~(size_t)15;
    const size_t o_trace = o_words + 16;
    if ((r = ws_pinned(w, o_trace + 8 * trace_words))) return r;
    ga = goal_args(g, w);
    if (total > 0) {
        k_goal_front<<<std::min(nq, L.nblocks), L.threads, L.lds, s>>>(a, ga);
        k_goal_pack<<<std::min(nq, 1024), 256, 0, s>>>(ga, w->p_lab, w->p_node, w->p_cap);
        HIP_TRY(hipGetLastError());
    }
    int *h_counts = reinterpret_cast<int *>(w->hpin + o_small);
    int *h_qlast = h_counts + nq, *h_qstop = h_counts + 2 * nq;
    unsigned *h_ptop = reinterpret_cast<unsigned *>(w->hpin + o_words);
    int *h_ovf = reinterpret_cast<int *>(w->hpin + o_words + 4);
    int *h_gerr = reinterpret_cast<int *>(w->hpin + o_words + 8);
    long long *h_trace = reinterpret_cast<long long *>(w->hpin + o_trace);
    HIP_TRY(hipMemcpyAsync(h_counts, w->g_count, sizeof(int) * nq, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h_qlast, w->qlast, sizeof(int) * nq, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h_qstop, w->qstop, sizeof(int) * nq, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h_ptop, w->pool_top, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h_ovf, w->g_overflow, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h_gerr, w->err, sizeof(int), hipMemcpyDeviceToHost, s));
    if (trace_words)
        HIP_TRY(hipMemcpyAsync(h_trace, w->wstat, sizeof(long long) * trace_words,
                               hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (*h_ovf || *h_gerr) return fail(MPAP_ERR_OVERFLOW, "goal front overflow");
    std::memcpy(counts.data(), h_counts, sizeof(int) * nq);
    std::memcpy(qlast.data(), h_qlast, sizeof(int) * nq);
    std::memcpy(qstop.data(), h_qstop, sizeof(int) * nq);
    const unsigned ptop = *h_ptop;
    std::vector<long long> trace(h_trace, h_trace + trace_words);
    long long packed = 0;
    for (int q = 0; q < nq; ++q) packed += counts[q];
    std::vector<float4> plab(packed);
    std::vector<int> pnode(packed);
    if (packed > 0) {
        if ((r = ws_pinned(w, 20 * (size_t)packed))) return r;
        float4 *h_lab = reinterpret_cast<float4 *>(w->hpin);
        int *h_node = reinterpret_cast<int *>(w->hpin + 16 * (size_t)packed);
        HIP_TRY(hipMemcpyAsync(h_lab, w->p_lab, sizeof(float4) * packed, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(h_node, w->p_node, sizeof(int) * packed, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        std::memcpy(plab.data(), h_lab, sizeof(float4) * packed);
        std::memcpy(pnode.data(), h_node, sizeof(int) * packed);
    }
    search_finish(res, p, dev_out, counts.data(), plab.data(), pnode.data(), qlast.data(),
                  qstop.data(), trace.data(), ms, retries, L);
    res->pool_used = ptop;
    return MPAP_OK;
}

int acquire_workspace(mpap_graph *g, const SearchShape &L, Workspace **out) {
    *out = nullptr;
    Workspace *w = nullptr;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        if (!g->spare.empty()) {
            w = g->spare.back();
            g->spare.pop_back();
        }
    }
    if (w && w->nblocks != L.nblocks) {
        w->free_all();
        delete w;
        w = nullptr;
    }
    if (!w) {
        w = new Workspace();
        const int r = ws_alloc_nodes(w, g->n, L.nblocks);
        if (r) {
            w->free_all();
            delete w;
            return r;
        }
    }
    *out = w;
    return MPAP_OK;
}

extern "C" {

int mpap_search_batch(const mpap_graph *gc, const mpap_search_params *sp, int32_t nsp,
                      void *stream, mpap_result **out) {
    if (!out) return fail(MPAP_ERR_INVAL, "out is null");
    *out = nullptr;
    if (!gc || !sp) return fail(MPAP_ERR_INVAL, "null graph or params");
    mpap_graph *g = const_cast<mpap_graph *>(gc);
    SearchPrep p;
    int r = search_prep(g, sp, nsp, p);
    if (r) return r;
    for (int q = 0; q < p.nq; ++q)
        if (p.heur[q] == 1 && !(g->symmetric_alias ? g->sdrift : g->srdrift))
            return fail(MPAP_ERR_INVAL, "no surrogate drift on this graph (mpap_surrogate_score)");
    SearchShape L;
    if ((r = search_shape(p.stage_cap, p.block_threads, p.wave_min_targets, L, p.merge_halves)))
        return r;
    L.obj = uniform_objectives(p);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    Workspace *w = nullptr;
    if ((r = acquire_workspace(g, L, &w))) return r;
    mpap_result *res = new mpap_result();
    res->g = g;
    res->ws = w;
    if ((r = search_eager(g, p, L, w, s, res))) {
        mpap_result_free(res);
        return r;
    }
    *out = res;
    return MPAP_OK;
}

int mpap_search(const mpap_graph *g, const mpap_search_params *sp, void *stream,
                mpap_result **out) {
    return mpap_search_batch(g, sp, 1, stream, out);
}

int mpap_query_goal_front(const mpap_result *r, int32_t query, float *cost, float *drift,
                          float *maxdrift, int32_t *goal_node, int32_t *label_id,
                          int32_t capacity, int32_t *count) {
    if (!r || !count) return fail(MPAP_ERR_INVAL, "null result or count");
    if (query < 0 || query >= r->g->nq) return fail(MPAP_ERR_INVAL, "query out of range");
    const int64_t o = r->front_off[query];
    const int32_t k = (int32_t)(r->front_off[query + 1] - o);
    *count = k;
    if (capacity < k) return fail(MPAP_ERR_CAPACITY, "capacity below the front size");
    for (int32_t i = 0; i < k; ++i) {
        const float4 L = r->front[o + i];
        if (cost) cost[i] = L.x;
        if (drift) drift[i] = L.y;
        if (maxdrift) maxdrift[i] = L.z;
        if (goal_node) goal_node[i] = r->front_node[o + i];
        if (label_id) {
            int id;
            std::memcpy(&id, &L.w, sizeof(int));
            label_id[i] = id;
        }
    }
    return MPAP_OK;
}

int mpap_query_stop(const mpap_result *r, int32_t query, int32_t *groups) {
    if (!r || !groups) return fail(MPAP_ERR_INVAL, "null result or output");
    if (query < 0 || query >= r->g->nq) return fail(MPAP_ERR_INVAL, "query out of range");
    *groups = query < (int)r->qstop.size() ? r->qstop[query] : -1;
    return MPAP_OK;
}

int mpap_refine_front(const mpap_result *r, int32_t query, float beta_prime, int32_t n_obj_out,
                      float *cost, float *drift, float *maxdrift, int32_t *goal_node,
                      int32_t *label_id, int32_t capacity, int32_t *count) {
    if (!r || !count) return fail(MPAP_ERR_INVAL, "null result or count");
    if (query < 0 || query >= r->g->nq) return fail(MPAP_ERR_INVAL, "query out of range");
    if (r->qnobj[query] != 3)
        return fail(MPAP_ERR_INVAL, "refinement needs a search with three objectives");
    if (std::isnan(beta_prime) || beta_prime > r->qbeta[query])
        return fail(MPAP_ERR_INVAL, "beta_prime must not exceed the search's bound");
    if (n_obj_out != 2 && n_obj_out != 3) return fail(MPAP_ERR_INVAL, "n_obj_out must be 2 or 3");
    if (query < (int)r->qstop.size() && r->qstop[query] >= 0)
        return fail(MPAP_ERR_INVAL, "an early-stopped query has no exact front to refine");
    // the front is in ascending (c, d, m) order: members with m <= beta_prime
    // keep it; for two objectives a member survives iff its drift is below
    // that of every kept member before it (the first of equal (c, d) has the
    // least m)
    const int64_t o = r->front_off[query], e = r->front_off[query + 1];
    int32_t k = 0;
    float dmin = INFINITY;
    for (int pass = 0; pass < 2; ++pass) {
        k = 0;
        dmin = INFINITY;
        for (int64_t i = o; i < e; ++i) {
            const float4 L = r->front[i];
            if (!(L.z <= beta_prime)) continue;
            if (n_obj_out == 2) {
                if (!(L.y < dmin)) continue;
                dmin = L.y;
            }
            if (pass == 1) {
                if (cost) cost[k] = L.x;
                if (drift) drift[k] = L.y;
                if (maxdrift) maxdrift[k] = n_obj_out == 2 ? 0.0f : L.z;
                if (goal_node) goal_node[k] = r->front_node[i];
                if (label_id) std::memcpy(&label_id[k], &L.w, sizeof(int));
            }
            ++k;
        }
        if (pass == 0) {
            *count = k;
            if (capacity < k) return fail(MPAP_ERR_CAPACITY, "capacity below the front size");
        }
    }
    return MPAP_OK;
}

int mpap_goal_front(const mpap_result *r, float *cost, float *drift, float *maxdrift,
                    int32_t *goal_node, int32_t *label_id, int32_t capacity, int32_t *count) {
    return mpap_query_goal_front(r, 0, cost, drift, maxdrift, goal_node, label_id, capacity,
                                 count);
}

int mpap_query_info(const mpap_result *r, int32_t query, float *latency_ms,
                    int32_t *last_wave) {
    if (!r) return fail(MPAP_ERR_INVAL, "null result");
    if (query < 0 || query >= r->g->nq) return fail(MPAP_ERR_INVAL, "query out of range");
    if (latency_ms) *latency_ms = r->qlatency_ms[query];
    if (last_wave) *last_wave = r->qlast[query];
    return MPAP_OK;
}

int mpap_node_front(const mpap_result *r, int32_t node, float *cost, float *drift,
                    float *maxdrift, int32_t *label_id, int32_t capacity, int32_t *count) {
    if (!r || !count) return fail(MPAP_ERR_INVAL, "null result or count");
    if (node < 0 || node >= r->g->n) return fail(MPAP_ERR_INVAL, "node out of range");
    if (r->fallback) {
        // a query the judge rejected is answered by the analytic re-search
        const auto &qo = r->g->qoff_h;
        const int q = (int)(std::upper_bound(qo.begin(), qo.end(), node) - qo.begin()) - 1;
        if (q >= 0 && q < (int)r->qfall.size() && r->qfall[q]) {
            const int st = mpap_node_front(r->fallback, node, cost, drift, maxdrift, label_id,
                                           capacity, count);
            if (st == MPAP_OK && label_id)
                for (int i = 0; i < *count; ++i) label_id[i] += (int32_t)r->id_offset;
            return st;
        }
    }
    int4 nbv;
    HIP_TRY(hipMemcpy(&nbv, r->ws->nb + node, sizeof(int4), hipMemcpyDeviceToHost));
    *count = nbv.z;
    if (capacity < nbv.z) return fail(MPAP_ERR_CAPACITY, "capacity below the front size");
    std::vector<float4> L(nbv.z);
    if (nbv.z > 0)
        HIP_TRY(hipMemcpy(L.data(), r->ws->pool + (unsigned)nbv.x, sizeof(float4) * nbv.z,
                          hipMemcpyDeviceToHost));
    for (int i = 0; i < nbv.z; ++i) {
        if (cost) cost[i] = L[i].x;
        if (drift) drift[i] = L[i].y;
        if (maxdrift) maxdrift[i] = L[i].z;
        if (label_id) {
            uint32_t meta;
            std::memcpy(&meta, &L[i].w, sizeof(meta));
            // a plan still open when an early stop ended the loop has no id
            label_id[i] = (meta & 0x80000000u) ? -1 : (int32_t)meta;
        }
    }
    return MPAP_OK;
}

int mpap_label_path(const mpap_result *rc, int32_t label_id, int32_t *nodes, int32_t capacity,
                    int32_t *length) {
    mpap_result *r = const_cast<mpap_result *>(rc);
    if (!r || !length) return fail(MPAP_ERR_INVAL, "null result or length");
    if (r->fallback && label_id >= r->id_offset)
        return mpap_label_path(r->fallback, (int32_t)(label_id - r->id_offset), nodes, capacity,
                               length);
    const long long L = r->arena_labels;
    if (label_id < 0 || label_id >= L) return fail(MPAP_ERR_INVAL, "label id out of range");
    if (!r->arena_loaded) {
        r->arena_host.resize(L);
        HIP_TRY(hipMemcpy(r->arena_host.data(), r->ws->arena, sizeof(int2) * L,
                          hipMemcpyDeviceToHost));
        r->arena_loaded = true;
    }
    int32_t len = 0;
    for (long long a = label_id; a >= 0; a = r->arena_host[a].y) {
        if (++len > L) return fail(MPAP_ERR_HIP, "parent chain does not end");
    }
    *length = len;
    if (capacity < len) return fail(MPAP_ERR_CAPACITY, "capacity below the path length");
    int32_t i = len - 1;
    for (long long a = label_id; a >= 0; a = r->arena_host[a].y) nodes[i--] = r->arena_host[a].x;
    return MPAP_OK;
}

int mpap_wave_trace(const mpap_result *r, int64_t *out, int32_t capacity, int32_t *waves) {
    if (!r || !waves) return fail(MPAP_ERR_INVAL, "null argument");
    const int32_t w = std::min<int32_t>(r->stats.waves, kTraceCap);
    *waves = w;
    if (capacity < w) return fail(MPAP_ERR_CAPACITY, "capacity below the traced wave count");
    if (w > 0 && out)
        std::memcpy(out, r->trace.data(), sizeof(int64_t) * kTraceWords * w);
    return MPAP_OK;
}

int mpap_result_stats(const mpap_result *r, mpap_stats *out) {
    if (!r || !out) return fail(MPAP_ERR_INVAL, "null argument");
    *out = r->stats;
    return MPAP_OK;
}

void mpap_result_free(mpap_result *r) {
    if (!r) return;
    if (r->fallback) mpap_result_free(r->fallback);
    r->fallback = nullptr;
    if (r->ws_borrowed) {
        // the workspace belongs to a plan
    } else if (r->ws && r->g) {
        std::lock_guard<std::mutex> lk(r->g->mu);
        r->g->spare.push_back(r->ws);
    } else if (r->ws) {
        r->ws->free_all();
        delete r->ws;
    }
    delete r;
}

}  // extern "C"

int build_pair_index(mpap_graph *g, hipStream_t s) {
    int *cnt = nullptr, *tmp = nullptr;
    int r;
    if ((r = dalloc(&g->uptr, (size_t)g->n + 1)) || (r = dalloc(&cnt, (size_t)g->n + 1)) ||
        (r = dalloc(&tmp, div_up((long long)g->n + 1, kScanTile) + 1))) {
        dfree(cnt); dfree(tmp); dfree(g->uptr);
        return r;
    }
    k_upper_count<<<div_up((long long)g->n + 1, 256), 256, 0, s>>>(g->n, g->optr, g->ocol, cnt);
    r = scan_i32(cnt, g->uptr, (long long)g->n + 1, tmp, s);
    const hipError_t he = hipStreamSynchronize(s);  // before the temporaries go
    dfree(cnt); dfree(tmp);
    if (!r && he != hipSuccess) r = fail(MPAP_ERR_HIP, hipGetErrorString(he));
    if (r) dfree(g->uptr);
    return r;
}

void graph_release(mpap_graph *g) {
    for (Workspace *w : g->spare) {
        w->free_all();
        delete w;
    }
    g->spare.clear();
    if (!g->symmetric_alias) {
        dfree(g->rptr); dfree(g->rsrc); dfree(g->rcost); dfree(g->rdrift);
    }
    dfree(g->optr); dfree(g->ocol); dfree(g->ocost); dfree(g->odrift);
    dfree(g->nflag); dfree(g->goal_list); dfree(g->qoff); dfree(g->qgoff);
    dfree(g->pos); dfree(g->bmu); dfree(g->bsig); dfree(g->bamp); dfree(g->feat); dfree(g->sbase); dfree(g->sdrift);
    dfree(g->blo); dfree(g->bhi);
    dfree(g->vel); dfree(g->elen); dfree(g->rperm); dfree(g->srdrift); dfree(g->uptr);
    delete g;
}
