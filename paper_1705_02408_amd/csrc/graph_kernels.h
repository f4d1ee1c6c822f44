// Kernel argument block of the roadmap construction kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

constexpr int kScanTile = 4096;

struct BuildArgs {
    int n;
    int dim;
    const float *pos;  // device [n][dim]
    int nbox;
    const float *blo;  // device [nbox][dim]
    const float *bhi;
    int nblob;
    const float *mu;   // device [nblob][dim]
    const float *sig;  // [nblob]
    const float *amp;  // [nblob]
    float r;
    float step;
    float reset_q;
    float goal[3];
    float goal_r;
};

// Feature quality q(x) = clamp(sum_j a_j exp(-|x - mu_j|^2 / (2 s_j^2)), 0, 1)
// over the blobs of g (dim coordinates), float32 in blob order.
__device__ __forceinline__ float blob_quality(const BuildArgs &g, const float *x) {
    float acc = 0.0f;
    for (int j = 0; j < g.nblob; ++j) {
        float d2 = 0.0f;
        for (int k = 0; k < g.dim; ++k) {
            const float t = x[k] - g.mu[j * g.dim + k];
            d2 = d2 + t * t;
        }
        const float s = g.sig[j];
        acc = acc + g.amp[j] * expf(-d2 / (2.0f * s * s));
    }
    return fminf(fmaxf(acc, 0.0f), 1.0f);
}

// The same quality in float64 on a float64 point (float32 blob parameters
// widened exactly), summed in blob order and clamped: the definition the
// per-edge drift and the relocalisation flag are evaluated with, rounded to
// float32 only at the end by the caller.
__device__ __forceinline__ double blob_quality_f64(const BuildArgs &g, const double *x) {
    double acc = 0.0;
    for (int j = 0; j < g.nblob; ++j) {
        double d2 = 0.0;
        for (int k = 0; k < g.dim; ++k) {
            const double t = x[k] - (double)g.mu[j * g.dim + k];
            d2 = d2 + t * t;
        }
        const double s = (double)g.sig[j];
        acc = acc + (double)g.amp[j] * exp(-d2 / (2.0 * (s * s)));
    }
    return fmin(fmax(acc, 0.0), 1.0);
}

// Uniform grid over the bounding box of the positions for Near: cells of
// edge h >= r (1 + 2^-7) on each used axis, so any pair with Cost < r lies
// in the same or adjacent cells even after the float32 roundings of the
// distance and of the cell coordinates.  Nodes are counting-sorted by cell
// (x fastest), so the three x-neighbour cells of a cell are one contiguous
// run of the sorted arrays.
struct GridArgs {
    int gx, gy, gz;       // cells per axis (1 on an unused axis)
    float lo[3];          // bounding-box corner (minimum of each coordinate)
    float inv;            // 1 / h
    int ncell;            // gx * gy * gz
    int *ccount;          // [ncell] nodes per cell
    int *cstart;          // [ncell] exclusive scan of ccount
    int *sid;             // [n] node id at each sorted slot
    float4 *spos;         // [n] its position (unused coordinates 0)
};

// longest row the grid path sorts (one wave per row, staged in LDS); a
// longer row makes the host fill with the all-pairs kernel instead
constexpr int kGridSortMax = 256;

__global__ void k_grid_bin(BuildArgs g, GridArgs gr, int *cell, int *slot);
__global__ void k_grid_scatter(BuildArgs g, GridArgs gr, const int *cell, const int *slot);
__global__ void k_near_count_grid(BuildArgs g, GridArgs gr, int *cnt, int *max_cnt);
__global__ void k_near_fill_grid(BuildArgs g, GridArgs gr, const int *off, int *cand_u,
                                 int *cand_v, float *cand_c);
__global__ void k_sort_rows(int n, const int *off, const int *cnt, int *cand_v, float *cand_c);
__global__ void k_near_count(BuildArgs g, int *cnt);
__global__ void k_near_fill(BuildArgs g, const int *off, int *cand_u, int *cand_v,
                            float *cand_c);
__global__ void k_collide(BuildArgs g, long long m, const int *cand_u, const int *cand_v,
                          const float *cand_c, int *keep);
__global__ void k_compact_edges(long long m, const int *keep, const int *kscan,
                                const int *cand_v, const float *cand_c, int *col, float *cost);
__global__ void k_row_ptr(int n, long long m, const int *cand_off, const int *kscan,
                          const int *keep, int *row_ptr);
__global__ void k_edge_drift(BuildArgs g, int n, const int *row_ptr, const int *col,
                             const float *cost, float *drift);
// symmetric roadmaps: one thread per id-ordered pair, both edges written;
// uptr[u] = entries v > u in rows before u (k_upper_count + exclusive scan)
__global__ void k_edge_drift_pairs(BuildArgs g, int n, const int *row_ptr, const int *col,
                                   const float *cost, const int *uptr, float *drift);
__global__ void k_upper_count(int n, const int *row_ptr, const int *col, int *cnt);
__global__ void k_node_flags(BuildArgs g, uint8_t *flag);
__global__ void k_flag_list(int n, const uint8_t *flag, unsigned bit, int *list, int *count);
__global__ void k_scan_block_sums(const int *in, long long n, int *bsum);
__global__ void k_scan_sums(int *bsum, int nb);
__global__ void k_scan_apply(const int *in, long long n, const int *bsum, int *out);
__global__ void k_add_i32(int *p, long long n, int add);
__global__ void k_zero_i32(int *p, long long n);
// surrogate inputs per edge (16 bf16) and the 8-point estimate of the mean
// of (1 - q) along it (base, nullable)
__global__ void k_edge_features(BuildArgs g, int n, const int *row_ptr, const int *col,
                                const float *cost, uint16_t *X, float *base);
__global__ void k_edge_features_pairs(BuildArgs g, int n, const int *row_ptr, const int *col,
                                      const float *cost, const int *uptr, uint16_t *X,
                                      float *base);
__global__ void k_drift_ratio(long long m, const float *drift, const float *cost,
                              const float *base, float scale, float *t);
