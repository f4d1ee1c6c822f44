// Roadmap construction on the GPU: Sec. 3 Alg. 2 (BuildGraph: Near within
// r_n, then Collision against axis-aligned boxes as in Sec. 4.2) and the
// per-edge / per-node inputs of the perception heuristic (Alg. 1 step 2):
// drift increment = length * (1 - mean feature quality over the collision
// sub-steps) and the relocalisation flag q(x) > threshold (Sec. 4.1 drift
// reading with a feature-density quality q).
//
// Every float32 operation on the geometry is rounded separately (built with
// -ffp-contract=off), so neighbour sets and edge lengths are reproducible
// bit for bit by any IEEE float32 evaluation of the same formulas.
#include "device_common.h"
#include "graph_kernels.h"

namespace {

__device__ __forceinline__ float sqdist(const float *a, const float *b, int dim) {
    float dx = b[0] - a[0];
    float s = dx * dx;
    for (int k = 1; k < dim; ++k) {
        float d = b[k] - a[k];
        s = s + d * d;
    }
    return s;
}

// cell coordinate on one axis: floor((x - lo) / h), clamped to the grid
// (monotone in x, so cells of points less than one cell apart differ by at
// most one)
__device__ __forceinline__ int cell_axis(float x, float lo, float inv, int cells) {
    const float t = floorf((x - lo) * inv);
    return (int)fminf(fmaxf(t, 0.0f), (float)(cells - 1));
}

__device__ __forceinline__ int cell_coords(const GridArgs &gr, const float *x, int dim, int &cx,
                                           int &cy, int &cz) {
    cx = cell_axis(x[0], gr.lo[0], gr.inv, gr.gx);
    cy = cell_axis(x[1], gr.lo[1], gr.inv, gr.gy);
    cz = dim == 3 ? cell_axis(x[2], gr.lo[2], gr.inv, gr.gz) : 0;
    return (cz * gr.gy + cy) * gr.gx + cx;
}

// f(j) for every sorted slot j of the cells adjacent to (cx, cy, cz), the
// cell itself included: per (y, z) row of cells one contiguous run
template <class F>
__device__ __forceinline__ void for_adjacent(const GridArgs &gr, int cx, int cy, int cz, F f) {
    const int x0 = max(cx - 1, 0), x1 = min(cx + 1, gr.gx - 1);
    const int z1 = min(cz + 1, gr.gz - 1), y1 = min(cy + 1, gr.gy - 1);
    for (int z = max(cz - 1, 0); z <= z1; ++z)
        for (int y = max(cy - 1, 0); y <= y1; ++y) {
            const int row = (z * gr.gy + y) * gr.gx;
            const int b = gr.cstart[row + x0];
            const int e = gr.cstart[row + x1] + gr.ccount[row + x1];
            for (int j = b; j < e; ++j) f(j);
        }
}

// source row of the t-th id-ordered pair (a, b), a < b, of a symmetric
// roadmap: the last row u with uptr[u] <= t
__device__ __forceinline__ int pair_row(const int *uptr, int n, int t) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (uptr[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// index of edge v -> u in row v (rows sorted by target id), -1 if absent
__device__ __forceinline__ int reverse_edge(const int *row_ptr, const int *col, int v, int u) {
    const int end = row_ptr[v + 1];
    int lo = row_ptr[v], hi = end;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (col[mid] < u) lo = mid + 1; else hi = mid;
    }
    return (lo < end && col[lo] == u) ? lo : -1;
}

// blob parameters staged in LDS (mu[nblob*dim], sig[nblob], amp[nblob]);
// returns g reading them from there
__device__ __forceinline__ BuildArgs stage_blobs(const BuildArgs &g, float *blob) {
    for (int i = threadIdx.x; i < g.nblob * g.dim; i += blockDim.x) blob[i] = g.mu[i];
    for (int i = threadIdx.x; i < g.nblob; i += blockDim.x) {
        blob[g.nblob * g.dim + i] = g.sig[i];
        blob[g.nblob * g.dim + g.nblob + i] = g.amp[i];
    }
    __syncthreads();
    BuildArgs gl = g;
    gl.mu = blob;
    gl.sig = blob + g.nblob * g.dim;
    gl.amp = blob + g.nblob * g.dim + g.nblob;
    return gl;
}

// drift of the id-ordered pair (a, b) of length len: sum_j (len/K)(1 - q(mid_j))
// over the K sub-step midpoints x_a + ((j + 1/2)/K)(x_b - x_a), in float64
// in j order from the float32 positions and length, rounded once to float32
__device__ __forceinline__ float pair_drift(const BuildArgs &gl, int a, int b, float len) {
    double xa[3] = {0.0, 0.0, 0.0}, df[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < gl.dim; ++k) {
        xa[k] = (double)gl.pos[a * gl.dim + k];
        df[k] = (double)gl.pos[b * gl.dim + k] - xa[k];
    }
    int K = (int)ceilf(len / gl.step);
    if (K < 1) K = 1;
    const double dK = (double)K;
    const double w = (double)len / dK;
    double acc = 0.0;
    for (int j = 0; j < K; ++j) {
        const double s = ((double)j + 0.5) / dK;
        double p[3];
        for (int k = 0; k < gl.dim; ++k) p[k] = xa[k] + s * df[k];
        acc = acc + w * (1.0 - blob_quality_f64(gl, p));
    }
    return (float)acc;
}

// surrogate inputs of the id-ordered pair (a, b) of length len: x_a (3), x_b
// (3, zero z in 2D), the length, q at the 8 segment points (k + 1/2)/8, q(x_b);
// bfloat16.  Returns the 8-point estimate of the mean of (1 - q).
__device__ __forceinline__ float pair_features(const BuildArgs &gl, int a, int b, float len,
                                               uint16_t *f) {
    float xa[3] = {0.f, 0.f, 0.f}, xb[3] = {0.f, 0.f, 0.f}, df[3] = {0.f, 0.f, 0.f};
    for (int k = 0; k < gl.dim; ++k) {
        xa[k] = gl.pos[a * gl.dim + k];
        xb[k] = gl.pos[b * gl.dim + k];
        df[k] = xb[k] - xa[k];
    }
    for (int k = 0; k < 3; ++k) {
        f[k] = f2bf(xa[k]);
        f[3 + k] = f2bf(xb[k]);
    }
    f[6] = f2bf(len);
    float acc = 0.0f;
    for (int j = 0; j < 8; ++j) {
        const float s = ((float)j + 0.5f) / 8.0f;
        float p[3] = {0.f, 0.f, 0.f};
        for (int k = 0; k < gl.dim; ++k) p[k] = xa[k] + s * df[k];
        const float w = 1.0f - blob_quality(gl, p);
        f[7 + j] = f2bf(w);
        acc = acc + w;
    }
    f[15] = f2bf(1.0f - blob_quality(gl, xb));
    return acc * 0.125f;
}

}  // namespace

// Grid Near, step 1: each node's cell and its slot among the cell's nodes.
__global__ void __launch_bounds__(256) k_grid_bin(BuildArgs g, GridArgs gr, int *cell, int *slot) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= g.n) return;
    float x[3] = {0.f, 0.f, 0.f};
    for (int k = 0; k < g.dim; ++k) x[k] = g.pos[u * g.dim + k];
    int cx, cy, cz;
    const int c = cell_coords(gr, x, g.dim, cx, cy, cz);
    cell[u] = c;
    slot[u] = atomicAdd(&gr.ccount[c], 1);
}

// Step 2 (after the scan of the cell counts): nodes and positions in cell
// order.
__global__ void __launch_bounds__(256) k_grid_scatter(BuildArgs g, GridArgs gr, const int *cell,
                                                      const int *slot) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= g.n) return;
    float x[3] = {0.f, 0.f, 0.f};
    for (int k = 0; k < g.dim; ++k) x[k] = g.pos[u * g.dim + k];
    const int i = gr.cstart[cell[u]] + slot[u];
    gr.sid[i] = u;
    gr.spos[i] = make_float4(x[0], x[1], x[2], 0.0f);
}

// Step 3: the Near count of each node (the same test as the all-pairs
// kernel on the candidates of the adjacent cells); threads take nodes in
// cell order so the lanes of a wave scan the same cells.  max_cnt gets the
// longest row.
__global__ void __launch_bounds__(256) k_near_count_grid(BuildArgs g, GridArgs gr, int *cnt,
                                                         int *max_cnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int c = 0;
    if (i < g.n) {
        const int u = gr.sid[i];
        const float4 p = gr.spos[i];
        const float xu[3] = {p.x, p.y, p.z};
        int cx, cy, cz;
        cell_coords(gr, xu, g.dim, cx, cy, cz);
        for_adjacent(gr, cx, cy, cz, [&](int j) {
            const float4 q = gr.spos[j];
            const float xv[3] = {q.x, q.y, q.z};
            const float cost = sqrtf(sqdist(xu, xv, g.dim));
            c += (cost < g.r && gr.sid[j] != u) ? 1 : 0;
        });
        cnt[u] = c;
    }
    for (int o = 32; o > 0; o >>= 1) c = max(c, __shfl_xor(c, o));
    if ((threadIdx.x & 63) == 0) atomicMax(max_cnt, c);
}

// Step 4: the candidates of each node written to its row at off[u] in the
// order the cells are scanned.
__global__ void __launch_bounds__(256) k_near_fill_grid(BuildArgs g, GridArgs gr, const int *off,
                                                        int *cand_u, int *cand_v, float *cand_c) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    const int u = gr.sid[i];
    const float4 p = gr.spos[i];
    const float xu[3] = {p.x, p.y, p.z};
    int cx, cy, cz;
    cell_coords(gr, xu, g.dim, cx, cy, cz);
    const int o = off[u];
    int k = 0;
    for_adjacent(gr, cx, cy, cz, [&](int j) {
        const int v = gr.sid[j];
        const float4 q = gr.spos[j];
        const float xv[3] = {q.x, q.y, q.z};
        const float cost = sqrtf(sqdist(xu, xv, g.dim));
        if (cost < g.r && v != u) {
            cand_u[o + k] = u;
            cand_v[o + k] = v;
            cand_c[o + k] = cost;
            ++k;
        }
    });
}

// Step 5: each row put in target-id order, one wave per row (rows of at
// most kGridSortMax entries, staged in LDS): an entry's place is the number
// of smaller ids in its row (the ids of a row are distinct), so the rows
// equal the all-pairs kernel's.
__global__ void __launch_bounds__(256) k_sort_rows(int n, const int *off, const int *cnt,
                                                   int *cand_v, float *cand_c) {
    __shared__ int sv[4][kGridSortMax];
    __shared__ float sc[4][kGridSortMax];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int u = blockIdx.x * 4 + w;
    const int o = u < n ? off[u] : 0;
    const int d = u < n ? min(cnt[u], kGridSortMax) : 0;
    for (int i = l; i < d; i += 64) {
        sv[w][i] = cand_v[o + i];
        sc[w][i] = cand_c[o + i];
    }
    __syncthreads();
    for (int i = l; i < d; i += 64) {
        const int v = sv[w][i];
        int rank = 0;
        for (int j = 0; j < d; ++j) rank += sv[w][j] < v ? 1 : 0;
        cand_v[o + rank] = v;
        cand_c[o + rank] = sc[w][i];
    }
}

// Near: number of v != u with Cost(u, v) < r.  Positions are staged in LDS
// tiles shared by the block.
__global__ void __launch_bounds__(256) k_near_count(BuildArgs g, int *cnt) {
    __shared__ float tile[256 * 3];
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    float xu[3] = {0.f, 0.f, 0.f};
    if (u < g.n)
        for (int k = 0; k < g.dim; ++k) xu[k] = g.pos[u * g.dim + k];
    int c = 0;
    for (int t0 = 0; t0 < g.n; t0 += 256) {
        __syncthreads();
        const int v = t0 + threadIdx.x;
        if (v < g.n)
            for (int k = 0; k < g.dim; ++k) tile[threadIdx.x * 3 + k] = g.pos[v * g.dim + k];
        __syncthreads();
        const int m = min(256, g.n - t0);
        if (u < g.n)
            for (int i = 0; i < m; ++i) {
                const float cost = sqrtf(sqdist(xu, &tile[i * 3], g.dim));
                c += (cost < g.r && t0 + i != u) ? 1 : 0;
            }
    }
    if (u < g.n) cnt[u] = c;
}

__global__ void __launch_bounds__(256) k_near_fill(BuildArgs g, const int *off, int *cand_u,
                                                   int *cand_v, float *cand_c) {
    __shared__ float tile[256 * 3];
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    float xu[3] = {0.f, 0.f, 0.f};
    if (u < g.n)
        for (int k = 0; k < g.dim; ++k) xu[k] = g.pos[u * g.dim + k];
    int o = (u < g.n) ? off[u] : 0;
    for (int t0 = 0; t0 < g.n; t0 += 256) {
        __syncthreads();
        const int v = t0 + threadIdx.x;
        if (v < g.n)
            for (int k = 0; k < g.dim; ++k) tile[threadIdx.x * 3 + k] = g.pos[v * g.dim + k];
        __syncthreads();
        const int m = min(256, g.n - t0);
        if (u < g.n)
            for (int i = 0; i < m; ++i) {
                const float cost = sqrtf(sqdist(xu, &tile[i * 3], g.dim));
                if (cost < g.r && t0 + i != u) {
                    cand_u[o] = u;
                    cand_v[o] = t0 + i;
                    cand_c[o] = cost;
                    ++o;
                }
            }
    }
}

// Collision(a, b), (a, b) the candidate pair in id order: points
// x_a + (k/K)(x_b - x_a), k = 0..K, K = ceil(cost/step), against closed boxes.
__global__ void __launch_bounds__(256) k_collide(BuildArgs g, long long m, const int *cand_u,
                                                 const int *cand_v, const float *cand_c,
                                                 int *keep) {
    extern __shared__ float boxes[];  // lo[nbox*dim], hi[nbox*dim]
    for (int i = threadIdx.x; i < g.nbox * g.dim; i += blockDim.x) {
        boxes[i] = g.blo[i];
        boxes[g.nbox * g.dim + i] = g.bhi[i];
    }
    __syncthreads();
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const int u = cand_u[e], v = cand_v[e];
    const int a = min(u, v), b = max(u, v);
    float xa[3] = {0.f, 0.f, 0.f}, df[3] = {0.f, 0.f, 0.f};
    for (int k = 0; k < g.dim; ++k) {
        xa[k] = g.pos[a * g.dim + k];
        df[k] = g.pos[b * g.dim + k] - xa[k];
    }
    int K = (int)ceilf(cand_c[e] / g.step);
    if (K < 1) K = 1;
    const float fK = (float)K;
    // Each rounded coordinate xa + t df is monotone in s (t = s/K rounded,
    // t = 1 at s = K), so the points lie between the first (xa) and the
    // last (xa + df rounded) on every axis: a box missing that range on an
    // axis holds none of them.  The boxes are taken one at a time and only
    // those meeting the range are tested point by point (the same set of
    // point-in-box tests, grouped by box).
    float plo[3] = {0.f, 0.f, 0.f}, phi[3] = {0.f, 0.f, 0.f};
    for (int k = 0; k < g.dim; ++k) {
        const float last = xa[k] + df[k];
        plo[k] = fminf(xa[k], last);
        phi[k] = fmaxf(xa[k], last);
    }
    bool hit = false;
    for (int j = 0; j < g.nbox && !hit; ++j) {
        const float *lo = &boxes[j * g.dim];
        const float *hi = &boxes[g.nbox * g.dim + j * g.dim];
        bool meets = true;
        for (int k = 0; k < g.dim; ++k) meets = meets && phi[k] >= lo[k] && plo[k] <= hi[k];
        if (!meets) continue;
        for (int s = 0; s <= K && !hit; ++s) {
            const float t = (float)s / fK;
            bool in = true;
            for (int k = 0; k < g.dim; ++k) {
                const float p = xa[k] + t * df[k];
                in = in && (p >= lo[k]) && (p <= hi[k]);
            }
            hit = in;
        }
    }
    keep[e] = hit ? 0 : 1;
}

__global__ void __launch_bounds__(256) k_compact_edges(long long m, const int *keep,
                                                       const int *kscan, const int *cand_v,
                                                       const float *cand_c, int *col,
                                                       float *cost) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m || !keep[e]) return;
    const int o = kscan[e];
    col[o] = cand_v[e];
    cost[o] = cand_c[e];
}

__global__ void __launch_bounds__(256) k_row_ptr(int n, long long m, const int *cand_off,
                                                 const int *kscan, const int *keep,
                                                 int *row_ptr) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u > n) return;
    const long long o = (u < n) ? cand_off[u] : m;
    row_ptr[u] = (o < m) ? kscan[o] : (m > 0 ? kscan[m - 1] + keep[m - 1] : 0);
}

// drift of edge row u -> col[e] (pair_drift of the id-ordered pair: the same
// value for both directions of an edge)
__global__ void __launch_bounds__(256) k_edge_drift(BuildArgs g, int n, const int *row_ptr,
                                                    const int *col, const float *cost,
                                                    float *drift) {
    extern __shared__ float blob[];  // mu[nblob*dim], sig[nblob], amp[nblob]
    const BuildArgs gl = stage_blobs(g, blob);
    // one thread per edge; its source u: last row with row_ptr[u] <= e
    const int m = row_ptr[n];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (row_ptr[mid] <= e) lo = mid; else hi = mid - 1;
    }
    const int u = lo, v = col[e];
    drift[e] = pair_drift(gl, min(u, v), max(u, v), cost[e]);
}

// The same drift on a symmetric roadmap (rows sorted by target id), one
// thread per id-ordered pair: the t-th pair's value is evaluated once and
// written to both of its edges.  uptr[u] counts the entries v > u of the
// rows before u (uptr[n] pairs in all).
__global__ void __launch_bounds__(256) k_edge_drift_pairs(BuildArgs g, int n, const int *row_ptr,
                                                          const int *col, const float *cost,
                                                          const int *uptr, float *drift) {
    extern __shared__ float blob[];
    const BuildArgs gl = stage_blobs(g, blob);
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= uptr[n]) return;
    const int u = pair_row(uptr, n, t);
    const int e = row_ptr[u + 1] - (uptr[u + 1] - t);
    const int v = col[e];
    const float d = pair_drift(gl, u, v, cost[e]);
    drift[e] = d;
    const int r = reverse_edge(row_ptr, col, v, u);
    if (r >= 0) drift[r] = d;
}

// uptr helper: cnt[u] = entries v > u of row u (u < n), cnt[n] = 0; rows
// sorted by target id, no self loops
__global__ void __launch_bounds__(256) k_upper_count(int n, const int *row_ptr, const int *col,
                                                     int *cnt) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u > n) return;
    if (u == n) {
        cnt[n] = 0;
        return;
    }
    const int end = row_ptr[u + 1];
    int lo = row_ptr[u], hi = end;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (col[mid] < u) lo = mid + 1; else hi = mid;
    }
    cnt[u] = end - lo;
}

__global__ void __launch_bounds__(256) k_node_flags(BuildArgs g, uint8_t *flag) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.n) return;
    float x[3] = {0.f, 0.f, 0.f};
    double xd[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < g.dim; ++k) {
        x[k] = g.pos[v * g.dim + k];
        xd[k] = (double)x[k];
    }
    uint8_t f = 0;
    if (blob_quality_f64(g, xd) > (double)g.reset_q) f |= 1u;
    float gg[3] = {g.goal[0], g.goal[1], g.goal[2]};
    const float r = g.goal_r;
    if (sqdist(gg, x, g.dim) <= r * r) f |= 2u;
    flag[v] = f;
}

// Ordered list of the nodes with flag bit `bit` set (single block).
__global__ void __launch_bounds__(1024) k_flag_list(int n, const uint8_t *flag, unsigned bit,
                                                    int *list, int *count) {
    __shared__ int scan[32];
    int carry = 0;
    for (int t0 = 0; t0 < n; t0 += blockDim.x) {
        const int v = t0 + threadIdx.x;
        const int f = (v < n && (flag[v] & bit)) ? 1 : 0;
        int tot;
        const int ex = block_excl_scan(f, scan, &tot);
        if (f) list[carry + ex] = v;
        carry += tot;
    }
    if (threadIdx.x == 0) *count = carry;
}

// ------------------------------------------------------------------- scan
// Exclusive prefix sum of int32 values in three passes (block sums, scan of
// block sums in one block, add-back).  Each block covers kScanTile items.
__global__ void __launch_bounds__(256) k_scan_block_sums(const int *in, long long n,
                                                         int *bsum) {
    __shared__ int scan[16];
    const long long base = (long long)blockIdx.x * kScanTile;
    int s = 0;
    for (int i = threadIdx.x; i < kScanTile; i += blockDim.x)
        if (base + i < n) s += in[base + i];
    int tot;
    block_excl_scan(s, scan, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) k_scan_sums(int *bsum, int nb) {
    __shared__ int scan[32];
    int carry = 0;
    for (int t0 = 0; t0 < nb; t0 += blockDim.x) {
        const int i = t0 + threadIdx.x;
        const int v = (i < nb) ? bsum[i] : 0;
        int tot;
        const int ex = block_excl_scan(v, scan, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
}

__global__ void __launch_bounds__(256) k_scan_apply(const int *in, long long n,
                                                    const int *bsum, int *out) {
    __shared__ int scan[16];
    const long long base = (long long)blockIdx.x * kScanTile;
    int carry = bsum[blockIdx.x];
    constexpr int per = kScanTile / 256;
    // each thread owns `per` consecutive items
    int v[per];
    int s = 0;
    for (int k = 0; k < per; ++k) {
        const long long i = base + (long long)threadIdx.x * per + k;
        v[k] = (i < n) ? in[i] : 0;
        s += v[k];
    }
    int tot;
    int ex = block_excl_scan(s, scan, &tot);
    int run = carry + ex;
    for (int k = 0; k < per; ++k) {
        const long long i = base + (long long)threadIdx.x * per + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
}

// p[i] += add for i < n (id shifts when roadmaps are concatenated)
__global__ void __launch_bounds__(256) k_add_i32(int *p, long long n, int add) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] += add;
}

// p[i] = 0 for i < n (used instead of memset so the sequence can be captured)
__global__ void __launch_bounds__(256) k_zero_i32(int *p, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Inputs of the learned drift surrogate for edge row u -> col[e]
// (pair_features of the id-ordered pair, so both directions agree) and, if
// base is not null, the 8-point estimate.  One thread per edge (its source
// found by a binary search of row_ptr), so every lane has an edge whatever
// the node degrees.
__global__ void __launch_bounds__(256) k_edge_features(BuildArgs g, int n, const int *row_ptr,
                                                       const int *col, const float *cost,
                                                       uint16_t *X, float *base) {
    extern __shared__ float blob[];
    const BuildArgs gl = stage_blobs(g, blob);
    const int m = row_ptr[n];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    int lo = 0, hi = n - 1;  // source u: last row with row_ptr[u] <= e
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (row_ptr[mid] <= e) lo = mid; else hi = mid - 1;
    }
    const int u = lo, v = col[e];
    const float b8 = pair_features(gl, min(u, v), max(u, v), cost[e], X + (size_t)e * 16);
    if (base) base[e] = b8;
}

// The same inputs on a symmetric roadmap, one thread per id-ordered pair,
// written to both of its edges (uptr as for k_edge_drift_pairs).
__global__ void __launch_bounds__(256) k_edge_features_pairs(BuildArgs g, int n,
                                                             const int *row_ptr, const int *col,
                                                             const float *cost, const int *uptr,
                                                             uint16_t *X, float *base) {
    extern __shared__ float blob[];
    const BuildArgs gl = stage_blobs(g, blob);
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= uptr[n]) return;
    const int u = pair_row(uptr, n, t);
    const int e = row_ptr[u + 1] - (uptr[u + 1] - t);
    const int v = col[e];
    uint16_t f[16];
    const float b8 = pair_features(gl, u, v, cost[e], f);
    const int r = reverse_edge(row_ptr, col, v, u);
    uint4 *xe = reinterpret_cast<uint4 *>(X + (size_t)e * 16);
    const uint4 w0 = make_uint4(f[0] | ((unsigned)f[1] << 16), f[2] | ((unsigned)f[3] << 16),
                                f[4] | ((unsigned)f[5] << 16), f[6] | ((unsigned)f[7] << 16));
    const uint4 w1 = make_uint4(f[8] | ((unsigned)f[9] << 16), f[10] | ((unsigned)f[11] << 16),
                                f[12] | ((unsigned)f[13] << 16), f[14] | ((unsigned)f[15] << 16));
    xe[0] = w0;
    xe[1] = w1;
    if (base) base[e] = b8;
    if (r >= 0) {
        uint4 *xr = reinterpret_cast<uint4 *>(X + (size_t)r * 16);
        xr[0] = w0;
        xr[1] = w1;
        if (base) base[r] = b8;
    }
}

// t[e] = scale * (drift[e] / cost[e] - base[e]): the analytic per-edge mean
// of (1 - q) less its 8-point estimate, scaled, the surrogate network's
// training target
__global__ void __launch_bounds__(256) k_drift_ratio(long long m, const float *drift,
                                                     const float *cost, const float *base,
                                                     float scale, float *t) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) t[e] = scale * (drift[e] / cost[e] - (base ? base[e] : 0.0f));
}
