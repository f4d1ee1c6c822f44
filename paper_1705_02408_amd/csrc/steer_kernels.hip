// Double-integrator roadmap on the GPU (the state space of the quadrotor
// experiments, Sec. 4.1 and Sec. 5: position and velocity in 3D), built as
// BuildGraph does (Sec. 3, Alg. 2) with a steering cost for the neighbour
// relation, plus the per-edge drift inputs of the perception heuristic
// (Alg. 1 step 2).
//
// Steering (u -> v) is the minimum-energy control of p'' = a over the fixed
// time T: per axis, with a = (p_v - p_u) - v_u T and b = v_v - v_u, the control
// c0 + c1 t with c0 = 6a/T^2 - 2b/T and c1 = (6bT - 12a)/T^3, of energy
// J = 12a^2/T^3 - 12ab/T^2 + 4b^2/T (summed over the axes: the edge cost).
// The trajectory is checked at t_k = (k T)/K, k = 0..K: in the closed unit
// cube, in no closed box, speed at most 1.  Each state keeps the k_out
// reachable targets of least (J, id).  All of it in float32 with every
// operation rounded separately (-ffp-contract=off, correctly rounded
// division), so selection is reproducible bit for bit by any IEEE evaluation
// in the same order.
#include "device_common.h"
#include "graph_kernels.h"
#include "steer_kernels.h"

namespace {

__device__ __forceinline__ void load3(const float *a, int i, float *x) {
    x[0] = a[3 * i];
    x[1] = a[3 * i + 1];
    x[2] = a[3 * i + 2];
}

// energy J and control coefficients of the steer p0,v0 -> p1,v1 in time T
__device__ __forceinline__ float steer3(const float *p0, const float *v0, const float *p1,
                                        const float *v1, float T, float *c0, float *c1) {
    const float T2 = T * T, T3 = T2 * T;
    float ja[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float a = (p1[k] - p0[k]) - v0[k] * T;
        const float b = v1[k] - v0[k];
        ja[k] = ((12.0f * a) * a) / T3 - ((12.0f * a) * b) / T2 + ((4.0f * b) * b) / T;
        c0[k] = (6.0f * a) / T2 - (2.0f * b) / T;
        c1[k] = ((6.0f * b) * T - 12.0f * a) / T3;
    }
    return (ja[0] + ja[1]) + ja[2];
}

__device__ __forceinline__ float steer_cost(const float *p0, const float *v0, const float *p1,
                                            const float *v1, float T) {
    const float T2 = T * T, T3 = T2 * T;
    float ja[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float a = (p1[k] - p0[k]) - v0[k] * T;
        const float b = v1[k] - v0[k];
        ja[k] = ((12.0f * a) * a) / T3 - ((12.0f * a) * b) / T2 + ((4.0f * b) * b) / T;
    }
    return (ja[0] + ja[1]) + ja[2];
}

// position and velocity on the steered trajectory at time t (Horner order)
__device__ __forceinline__ void traj_at(const float *p0, const float *v0, const float *c0,
                                        const float *c1, float t, float *p, float *v) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float h2 = c0[k] * 0.5f, h3 = c1[k] / 6.0f, g1 = c1[k] * 0.5f;
        p[k] = p0[k] + t * (v0[k] + t * (h2 + t * h3));
        if (v) v[k] = v0[k] + t * (c0[k] + t * g1);
    }
}

__device__ __forceinline__ float check_time(int k, float T, int K) {
    return ((float)k * T) / (float)K;
}

// float order -> unsigned order (J + 0 turns -0 into +0)
__device__ __forceinline__ uint32_t ukey(float J) {
    const uint32_t b = __float_as_uint(J + 0.0f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float unkey(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// Reachability of the steer u -> v, decided by one wave (every lane returns
// the result).  sblo/sbhi: the boxes in LDS; wlist: per-wave LDS scratch of
// nbox ints.
__device__ bool wave_reachable(const SteerArgs &a, const float *p0, const float *v0, int v,
                               const float *sblo, const float *sbhi, int *wlist) {
    const int l = lane_id();
    float p1[3], v1[3], c0[3], c1[3];
    load3(a.pos, v, p1);
    load3(a.vel, v, v1);
    (void)steer3(p0, v0, p1, v1, a.T, c0, c1);
    float pts[4][3];
    bool ok = true;
    float lo[3] = {MPAP_INF, MPAP_INF, MPAP_INF}, hi[3] = {-MPAP_INF, -MPAP_INF, -MPAP_INF};
    int np = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int k = l + 64 * i;
        if (k <= a.K) {
            float p[3], vv[3];
            traj_at(p0, v0, c0, c1, check_time(k, a.T, a.K), p, vv);
            const float sp = (vv[0] * vv[0] + vv[1] * vv[1]) + vv[2] * vv[2];
            ok = ok && sp <= 1.0f;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                ok = ok && p[d] >= 0.0f && p[d] <= 1.0f;
                pts[i][d] = p[d];
                lo[d] = fminf(lo[d], p[d]);
                hi[d] = fmaxf(hi[d], p[d]);
            }
            np = i + 1;
        }
    }
    if (ballot64(!ok)) return false;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        lo[d] = wave_min(lo[d]);
        hi[d] = wave_max_f(hi[d]);
    }
    // boxes that meet the bounding box of the points
    int nl = 0;
    for (int j0 = 0; j0 < a.nbox; j0 += 64) {
        const int j = j0 + l;
        bool m = false;
        if (j < a.nbox)
            m = hi[0] >= sblo[3 * j] && lo[0] <= sbhi[3 * j] && hi[1] >= sblo[3 * j + 1] &&
                lo[1] <= sbhi[3 * j + 1] && hi[2] >= sblo[3 * j + 2] && lo[2] <= sbhi[3 * j + 2];
        const uint64_t bm = ballot64(m);
        if (m) wlist[nl + lanes_below(bm)] = j;
        nl += (int)__popcll(bm);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    bool hit = false;
    for (int i = 0; i < nl; ++i) {
        const int j = wlist[i];
        const float bl0 = sblo[3 * j], bl1 = sblo[3 * j + 1], bl2 = sblo[3 * j + 2];
        const float bh0 = sbhi[3 * j], bh1 = sbhi[3 * j + 1], bh2 = sbhi[3 * j + 2];
#pragma unroll
        for (int qi = 0; qi < 4; ++qi)
            if (qi < np)
                hit = hit || (pts[qi][0] >= bl0 && pts[qi][0] <= bh0 && pts[qi][1] >= bl1 &&
                              pts[qi][1] <= bh1 && pts[qi][2] >= bl2 && pts[qi][2] <= bh2);
    }
    const bool clear = ballot64(hit) == 0;
    __builtin_amdgcn_wave_barrier();  // wlist is reused by the next call
    return clear;
}

// The bin (of 2048) where the running count of hist first reaches need
// (1-based); sres[0] = bin, sres[1] = count below it.  Every thread calls.
__device__ void find_bin(const int *hist, int need, int *scratch, int *sres) {
    const int t = threadIdx.x;
    int loc = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) loc += hist[8 * t + i];
    int total;
    const int ex = block_excl_scan(loc, scratch, &total);
    if (ex < need && need <= ex + loc) {
        int c = ex;
        for (int i = 0; i < 8; ++i) {
            const int h = hist[8 * t + i];
            if (c + h >= need) {
                sres[0] = 8 * t + i;
                sres[1] = c;
                break;
            }
            c += h;
        }
    }
    __syncthreads();
}

}  // namespace

__global__ void __launch_bounds__(kSteerThreads) k_steer_select(SteerArgs a, int *nbr,
                                                                float *ncost, int *ncnt,
                                                                int *err) {
    extern __shared__ __align__(16) unsigned char lds[];
    int *hist = reinterpret_cast<int *>(lds);                          // 2048
    uint32_t *bkey = reinterpret_cast<uint32_t *>(hist + 2048);       // 2 * W
    int *bid = reinterpret_cast<int *>(bkey + 2 * kSteerMaxWidth);    // 2 * W
    float *sblo = reinterpret_cast<float *>(bid + 2 * kSteerMaxWidth);  // 3 * nbox
    float *sbhi = sblo + 3 * a.nbox;
    int *wlist = reinterpret_cast<int *>(sbhi + 3 * a.nbox);          // 4 * nbox
    __shared__ int scratch[kSteerThreads / 64 + 1];
    __shared__ int sres[2];
    __shared__ int s_cnt, s_found;
    __shared__ int out_id[kSteerMaxOut];
    __shared__ uint32_t out_key[kSteerMaxOut];
    __shared__ int okf[kSteerThreads / 64];

    for (int i = threadIdx.x; i < 3 * a.nbox; i += blockDim.x) {
        sblo[i] = a.blo[i];
        sbhi[i] = a.bhi[i];
    }
    const int u = blockIdx.x;
    const int w = threadIdx.x >> 6;
    float p0[3], v0[3];
    load3(a.pos, u, p0);
    load3(a.vel, u, v0);
    if (threadIdx.x == 0) s_found = 0;
    __syncthreads();

    uint32_t prev_key = 0u;
    int prev_id = -1;
    bool first = true;
    int width = 64;
    int found = 0;
    auto eligible = [&](int v, uint32_t k) {
        return v != u && (first || k > prev_key || (k == prev_key && v > prev_id));
    };
    auto key_of = [&](int v) {
        float p1[3], v1[3];
        load3(a.pos, v, p1);
        load3(a.vel, v, v1);
        return ukey(steer_cost(p0, v0, p1, v1, a.T));
    };
    while (found < a.k_out) {
        // radix select of the width-th smallest eligible key: 11 + 11 + 10 bits
        uint32_t tau = 0xffffffffu;
        int total = 0;
        {
            int need = width;
            uint32_t prefix = 0u;
            const int shifts[3] = {21, 10, 0};
            const uint32_t masks[3] = {2047u, 2047u, 1023u};
            for (int pass = 0; pass < 3; ++pass) {
                for (int i = threadIdx.x; i < 2048; i += blockDim.x) hist[i] = 0;
                __syncthreads();
                for (int v = threadIdx.x; v < a.n; v += blockDim.x) {
                    const uint32_t k = key_of(v);
                    if (!eligible(v, k)) continue;
                    if (pass > 0 && (k >> (shifts[pass - 1])) != prefix) continue;
                    atomicAdd(&hist[(k >> shifts[pass]) & masks[pass]], 1);
                }
                __syncthreads();
                if (pass == 0) {
                    int loc = 0;
                    for (int i = 0; i < 8; ++i) loc += hist[8 * threadIdx.x + i];
                    block_excl_scan(loc, scratch, &total);
                    if (total <= width) break;  // every eligible candidate fits
                }
                find_bin(hist, need, scratch, sres);
                const int bin = sres[0];
                need -= sres[1];
                prefix = (prefix << (pass == 0 ? 11 : (pass == 1 ? 11 : 10))) | (uint32_t)bin;
                if (pass == 2) tau = prefix;
                __syncthreads();
            }
        }
        if (total == 0) break;
        // gather the eligible keys <= tau, sort them by (key, id)
        if (threadIdx.x == 0) s_cnt = 0;
        __syncthreads();
        const int cap = 2 * width;
        for (int v = threadIdx.x; v < a.n; v += blockDim.x) {
            const uint32_t k = key_of(v);
            if (!eligible(v, k) || k > tau) continue;
            const int slot = atomicAdd(&s_cnt, 1);
            if (slot < cap) {
                bkey[slot] = k;
                bid[slot] = v;
            }
        }
        __syncthreads();
        int m = s_cnt;
        if (m > cap) {
            if (threadIdx.x == 0) atomicOr(err, 1);
            m = cap;
        }
        int P = 1;
        while (P < m) P <<= 1;
        for (int i = m + threadIdx.x; i < P; i += blockDim.x) {
            bkey[i] = 0xffffffffu;
            bid[i] = 0x7fffffff;
        }
        __syncthreads();
        for (int k = 2; k <= P; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = threadIdx.x; i < P; i += blockDim.x) {
                    const int x = i ^ j;
                    if (x > i) {
                        const bool up = (i & k) == 0;
                        const uint32_t ki = bkey[i], kx = bkey[x];
                        const int ii = bid[i], ix = bid[x];
                        const bool gt = ki > kx || (ki == kx && ii > ix);
                        if (gt == up) {
                            bkey[i] = kx; bkey[x] = ki;
                            bid[i] = ix; bid[x] = ii;
                        }
                    }
                }
                __syncthreads();
            }
        const int cnt = min(m, width);
        // check the ranked candidates in order, one wave each
        for (int base = 0; base < cnt && found < a.k_out; base += kSteerThreads / 64) {
            const int ci = base + w;
            bool ok = false;
            if (ci < cnt) ok = wave_reachable(a, p0, v0, bid[ci], sblo, sbhi, wlist + w * a.nbox);
            if (lane_id() == 0) okf[w] = ok ? 1 : 0;
            __syncthreads();
            if (threadIdx.x == 0) {
                int f = s_found;
                for (int i = 0; i < kSteerThreads / 64 && base + i < cnt && f < a.k_out; ++i)
                    if (okf[i]) {
                        out_id[f] = bid[base + i];
                        out_key[f] = bkey[base + i];
                        ++f;
                    }
                s_found = f;
            }
            __syncthreads();
            found = s_found;
        }
        if (cnt == 0 || total <= width) break;  // every eligible candidate was ranked
        prev_key = bkey[cnt - 1];
        prev_id = bid[cnt - 1];
        first = false;
        width = min(2 * width, kSteerMaxWidth);
        __syncthreads();
    }
    for (int i = threadIdx.x; i < found; i += blockDim.x) {
        nbr[(size_t)u * a.k_out + i] = out_id[i];
        ncost[(size_t)u * a.k_out + i] = unkey(out_key[i]);
    }
    if (threadIdx.x == 0) ncnt[u] = found;
}

__global__ void __launch_bounds__(256) k_steer_compact(int n, int k_out, const int *row_ptr,
                                                       const int *nbr, const float *ncost,
                                                       const int *ncnt, int *col, float *cost) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const int o = row_ptr[u], c = ncnt[u];
    int ids[kSteerMaxOut];
    float js[kSteerMaxOut];
    for (int i = 0; i < c; ++i) {
        int v = nbr[(size_t)u * k_out + i];
        float j = ncost[(size_t)u * k_out + i];
        int p = i;
        while (p > 0 && ids[p - 1] > v) {  // insertion by target id
            ids[p] = ids[p - 1];
            js[p] = js[p - 1];
            --p;
        }
        ids[p] = v;
        js[p] = j;
    }
    for (int i = 0; i < c; ++i) {
        col[o + i] = ids[i];
        cost[o + i] = js[i];
    }
}

// one wave per source row: drift = sum over the K chords of the checked
// points of |chord| (1 - q(chord midpoint)), the terms in float64 from the
// float32 check points, summed in chord order and rounded once to float32;
// elen = float32 sum of |chord| (the trajectory length of the surrogate's
// inputs)
__global__ void __launch_bounds__(64) k_traj_drift(SteerArgs a, const int *row_ptr,
                                                   const int *col, float *drift, float *elen) {
    extern __shared__ float blob[];
    __shared__ double term[kSteerMaxSteps + 1];
    for (int i = threadIdx.x; i < 3 * a.nblob; i += blockDim.x) blob[i] = a.mu[i];
    for (int i = threadIdx.x; i < a.nblob; i += blockDim.x) {
        blob[3 * a.nblob + i] = a.sig[i];
        blob[4 * a.nblob + i] = a.amp[i];
    }
    __syncthreads();
    BuildArgs q{};
    q.dim = 3;
    q.nblob = a.nblob;
    q.mu = blob;
    q.sig = blob + 3 * a.nblob;
    q.amp = blob + 4 * a.nblob;
    const int u = blockIdx.x;
    if (u >= a.n) return;
    const int l = lane_id();
    float p0[3], v0[3];
    load3(a.pos, u, p0);
    load3(a.vel, u, v0);
    for (int e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
        float p1[3], v1[3], c0[3], c1[3];
        load3(a.pos, col[e], p1);
        load3(a.vel, col[e], v1);
        (void)steer3(p0, v0, p1, v1, a.T, c0, c1);
        float len = 0.0f;
        for (int k = l; k < a.K; k += 64) {
            float pa[3], pb[3];
            traj_at(p0, v0, c0, c1, check_time(k, a.T, a.K), pa, nullptr);
            traj_at(p0, v0, c0, c1, check_time(k + 1, a.T, a.K), pb, nullptr);
            const float fx = pb[0] - pa[0], fy = pb[1] - pa[1], fz = pb[2] - pa[2];
            len = len + sqrtf((fx * fx + fy * fy) + fz * fz);
            double sq = 0.0, mid[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double t = (double)pb[d] - (double)pa[d];
                sq = sq + t * t;
                mid[d] = 0.5 * ((double)pb[d] + (double)pa[d]);
            }
            term[k] = sqrt(sq) * (1.0 - blob_quality_f64(q, mid));
        }
        len = wave_sum(len);
        __syncthreads();
        if (l == 0) {
            double acc = 0.0;
            for (int k = 0; k < a.K; ++k) acc = acc + term[k];
            drift[e] = (float)acc;
            if (elen) elen[e] = len;
        }
        __syncthreads();
    }
}

// one thread per edge of the row: p_u (3), p_v (3), trajectory length,
// 1 - q at t = (k + 1/2) T / 8, k = 0..7, and 1 - q(p_v); base = the
// speed-weighted mean of the eight 1 - q values (arc-length weighting)
__global__ void __launch_bounds__(256) k_traj_features(SteerArgs a, const int *row_ptr,
                                                       const int *col, const float *elen,
                                                       uint16_t *X, float *base) {
    extern __shared__ float blob[];
    for (int i = threadIdx.x; i < 3 * a.nblob; i += blockDim.x) blob[i] = a.mu[i];
    for (int i = threadIdx.x; i < a.nblob; i += blockDim.x) {
        blob[3 * a.nblob + i] = a.sig[i];
        blob[4 * a.nblob + i] = a.amp[i];
    }
    __syncthreads();
    BuildArgs q{};
    q.dim = 3;
    q.nblob = a.nblob;
    q.mu = blob;
    q.sig = blob + 3 * a.nblob;
    q.amp = blob + 4 * a.nblob;
    // one thread per edge; its source u: last row with row_ptr[u] <= e
    const int m = row_ptr[a.n];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    int lo = 0, hi = a.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (row_ptr[mid] <= e) lo = mid; else hi = mid - 1;
    }
    const int u = lo;
    float p0[3], v0[3];
    load3(a.pos, u, p0);
    load3(a.vel, u, v0);
    {
        float p1[3], v1[3], c0[3], c1[3];
        load3(a.pos, col[e], p1);
        load3(a.vel, col[e], v1);
        (void)steer3(p0, v0, p1, v1, a.T, c0, c1);
        uint16_t *f = X + (size_t)e * 16;
        for (int d = 0; d < 3; ++d) {
            f[d] = f2bf(p0[d]);
            f[3 + d] = f2bf(p1[d]);
        }
        f[6] = f2bf(elen[e]);
        float sw = 0.0f, ss = 0.0f, sm = 0.0f;
        for (int j = 0; j < 8; ++j) {
            const float t = (((float)j + 0.5f) * a.T) / 8.0f;
            float p[3], vv[3];
            traj_at(p0, v0, c0, c1, t, p, vv);
            const float wq = 1.0f - blob_quality(q, p);
            const float sp = sqrtf((vv[0] * vv[0] + vv[1] * vv[1]) + vv[2] * vv[2]);
            f[7 + j] = f2bf(wq);
            sw = sw + sp * wq;
            ss = ss + sp;
            sm = sm + wq;
        }
        f[15] = f2bf(1.0f - blob_quality(q, p1));
        if (base) base[e] = ss > 0.0f ? sw / ss : sm * 0.125f;
    }
}
