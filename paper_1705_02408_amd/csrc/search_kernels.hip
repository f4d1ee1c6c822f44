// Wavefront multiobjective label search (Sec. 3, Alg. 3 Explore) for gfx950.
//
// One cooperative persistent launch runs every Explore iteration.  Each
// iteration is three grid phases separated by grid barriers:
//
//   P1 count  : per node, the open labels whose cost is within the group
//               threshold (the group G of Alg. 3), plus open totals and the
//               least open cost (to skip empty thresholds).
//   P2 select : a device-wide scan of the group counts gives every group label
//               a frontier slot and an arena id (ids are dense and follow node
//               order, so runs are deterministic); the label is closed
//               (P_open <- P_open \ G), its (node, parent) goes to the arena and
//               the out-neighbours of its node are queued as merge targets.
//   P3 merge  : one workgroup per target node x pulls every group label at an
//               in-neighbour along its in-edge (cost, drift, bound, relocal-
//               isation: the child line and cutoff of Alg. 3), and merges the
//               children into P(x) with weak-Pareto RemoveDominated, staged in
//               LDS.  Each node has exactly one writer per iteration, so the
//               merge needs no atomics.
//
// Labels live in per-node buckets carved out of one pool (grown by doubling
// into a fresh region when a front outgrows its capacity).  The loop ends when
// no label is open.
#include "device_common.h"
#include "search_kernels.h"

namespace {

constexpr unsigned long long kSpinLimit = 1ull << 22;

__device__ __forceinline__ unsigned wave_par(int w) { return (unsigned)w & 1u; }

// weight class of a merge target with w children queued (see kWeightClasses)
__device__ __forceinline__ int weight_class(int w) {
    static_assert((kWeightClassBase & (kWeightClassBase - 1)) == 0, "power of two");
    if (w < kWeightClassBase) return 0;
    const int c = 1 + (31 - __clz(w)) - (31 - __clz(kWeightClassBase));
    return min(c, kWeightClasses - 1);
}

// query owning global node v: last q with qoff[q] <= v
__device__ __forceinline__ int query_of(const SearchArgs &a, int v) {
    int lo = 0, hi = a.nq - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.qoff[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// group step of the query owning node v
__device__ __forceinline__ float step_of(const SearchArgs &a, int v) {
    return a.qdelta[a.nq > 1 ? query_of(a, v) : 0];
}

// threshold of iteration i for a query of step d: T = i * d (float32)
__device__ __forceinline__ float threshold(long long i, float d) { return (float)i * d; }

// least iteration index whose threshold reaches cost c (float32 exact)
__device__ __forceinline__ long long first_step(float c, float d) {
    const float r = ceilf(c / d);
    long long i = r < 9.0e15f ? (long long)fmaxf(r, 0.0f) : (1ll << 53);
    while (threshold(i, d) < c) ++i;
    while (i > 0 && threshold(i - 1, d) >= c) --i;
    return i;
}

// ------------------------------------------------------------------ P1
// Nodes of the block's range are taken a tile (one per thread) at a time; the
// nodes whose least open cost is within the threshold go to an LDS list and
// the block's waves count their group labels in parallel, one node per wave.
__device__ __forceinline__ void phase_count(const SearchArgs &a, long long istep, int par, int lo, int hi,
                            int *list, int *scan, long long *red_ll) {
    const int l = lane_id();
    const int w = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    long long grp = 0, open_nodes = 0;
    long long mn = 0x7fffffffffffffffll;
    for (int tb = lo; tb < hi; tb += blockDim.x) {
        const int v = tb + threadIdx.x;
        bool need = false;
        if (v < hi) {
            const float mo = a.minopen[v];
            // the open plans of a query whose loop has ended are left alone
            const bool live =
                mo < MPAP_INF && (!a.early_any || a.qstop[a.nq > 1 ? query_of(a, v) : 0] < 0);
            if (live) {
                const float d = step_of(a, v);
                need = mo <= threshold(istep, d);
                open_nodes += 1;
                mn = min(mn, first_step(mo, d));
            }
            if (!need) a.gcnt[v] = 0;
        }
        int nflag;
        const int ex = block_excl_scan(need ? 1 : 0, scan, &nflag);
        if (need) list[ex] = v;
        __syncthreads();
        for (int i = w; i < nflag; i += nw) {
            const int vv = list[i];
            const int4 nbv = a.nb[vv];
            const float T = threshold(istep, step_of(a, vv));
            // open labels at or below T lie in the prefix of the sorted bucket,
            // from its first open label on
            int cnt = 0;
            for (int k = a.fo[vv].w + l; k < nbv.z; k += 64) {
                const float4 L = a.pool[(size_t)(unsigned)nbv.x + k];
                if (L.x > T) break;
                cnt += lab_open(L) ? 1 : 0;
            }
            cnt = wave_sum(cnt);
            if (l == 0) {
                a.gcnt[vv] = cnt;
                grp += cnt;
            }
        }
        __syncthreads();
    }
    long long g = block_sum_ll(grp, red_ll);
    long long o = block_sum_ll(open_nodes, red_ll);
    long long bm = block_min_ll(mn, red_ll);
    if (threadIdx.x == 0) {
        a.part_cnt[par * a.nblocks + blockIdx.x] = g;
        a.part_open[par * a.nblocks + blockIdx.x] = o;
        a.part_step[par * a.nblocks + blockIdx.x] = bm;
    }
}

// ------------------------------------------------------------------ P2
// Group labels get consecutive frontier slots in node order (a block-wide scan
// of the per-node counts on top of the block's offset); each flagged node is
// then handled by one wave: its group labels are copied to the frontier,
// closed and given their arena ids, and its out-neighbours are queued.
template <bool kSplit>
__device__ __forceinline__ void phase_select(const SearchArgs &a, long long istep, int wave, long long abase,
                             long long myoff, int lo, int hi, int *list, int *list_off,
                             int *scan) {
    const int l = lane_id();
    const int w = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    const unsigned wp = wave_par(wave);
    long long carry = myoff;
    for (int tb = lo; tb < hi; tb += blockDim.x) {
        const int v = tb + threadIdx.x;
        const int g = (v < hi) ? a.gcnt[v] : 0;
        int tot;
        const int ex = block_excl_scan(g, scan, &tot);
        int nflag;
        const int fx = block_excl_scan(g > 0 ? 1 : 0, scan, &nflag);
        if (g > 0) {
            list[fx] = v;
            list_off[fx] = (int)(carry + ex);  // frontier offsets fit in int32
        }
        __syncthreads();
        for (int i = w; i < nflag; i += nw) {
            const int vv = list[i];
            const int goff = list_off[i];
            // the node's record, its first open label, and its out-edges (the
            // row and its first 64 targets) are read together: none depends
            // on another
            const int4 nbv = a.nb[vv];
            const int fo_w = a.fo[vv].w;
            const int eb = a.optr[vv], ee = a.optr[vv + 1];
            const int x_first = eb + l < ee ? a.ocol[eb + l] : -1;
            const float T = threshold(istep, step_of(a, vv));
            int run = 0;
            float rmin = MPAP_INF;
            int first_open = nbv.z;
            // the bucket is sorted by cost: group labels lie below T from the
            // first open label on; past T only the first open label (the least
            // remaining open cost) matters, and it is the next first open one
            for (int k0 = fo_w; k0 < nbv.z; k0 += 64) {
                const int k = k0 + l;
                bool in = false, op = false, le = false;
                float4 L = make_float4(0.f, 0.f, 0.f, 0.f);
                const size_t slot = (size_t)(unsigned)nbv.x + k;
                if (k < nbv.z) {
                    L = a.pool[slot];
                    op = lab_open(L);
                    le = L.x <= T;
                    in = op && le;
                    if (op && !le) rmin = fminf(rmin, L.x);
                }
                const uint64_t bm = ballot64(in);
                if (in) {
                    const int pos = goff + run + lanes_below(bm);
                    const long long id = abase + pos;
                    a.F[pos] = make_float4(L.x, L.y, L.z, __int_as_float((int)id));
                    a.arena[id] = make_int2(vv, lab_parent(L));
                    reinterpret_cast<int *>(&a.pool[slot])[3] = (int)id;
                }
                run += (int)__popcll(bm);
                const bool past = ballot64(k < nbv.z && !le) != 0;
                const uint64_t beyond = ballot64(op && !le);
                if (beyond) first_open = k0 + (int)__ffsll((unsigned long long)beyond) - 1;
                if (past && (beyond != 0 || nbv.w - run == 0)) break;
            }
            rmin = wave_min(rmin);
            if (l == 0) {
                a.nb[vv].w = nbv.w - run;
                a.minopen[vv] = rmin;
                a.fo[vv] = make_int4(goff, run, wave, first_open);
                if (a.nq > 1) atomicMax(&a.qlast[query_of(a, vv)], wave);
                else if (vv >= 0) a.qlast[0] = wave;
            }
            // queue out-neighbours as merge targets of this wave, by the size
            // of their front (one slot reservation per wave of 64 out-edges)
            for (int e0 = eb; e0 < ee; e0 += 64) {
                const int e = e0 + l;
                int x = -1;
                bool fresh = false, big = false;
                if (e < ee) {
                    x = e0 == eb ? x_first : a.ocol[e];
                    if constexpr (kSplit) {
                        fresh = atomicExch(&a.mark[x], wave) != wave;
                        if (fresh) big = a.nb[x].z > a.wcap;
                    } else {
                        // the weight (children queued) starts at zero each iteration
                        fresh = atomicAdd(&a.wt[x], max(run, 1)) == 0;
                    }
                }
                const uint64_t fs = ballot64(fresh && !big), fb = ballot64(fresh && big);
                if (fs) {
                    int base = 0;
                    if (l == 0) base = atomicAdd(&a.acnt[wp], (int)__popcll(fs));
                    base = __shfl(base, 0, 64);
                    if (fresh && !big) a.alist[base + lanes_below(fs)] = x;
                }
                if (fb) {
                    int base = 0;
                    if (l == 0) base = atomicAdd(&a.acnt[2 + wp], (int)__popcll(fb));
                    base = __shfl(base, 0, 64);
                    if (fresh && big) a.alist[a.n + base + lanes_below(fb)] = x;
                }
            }
        }
        carry += tot;
        __syncthreads();
    }
}

// ------------------------------------------------------------------ P3
// Buckets are kept in lexicographic order of (c, d, m) (then the meta bits,
// which makes the order total and the run deterministic).  With that order a
// label b can weakly dominate a candidate q only if b.c <= q.c, i.e. b lies in
// the prefix of the bucket below q's cost, and the dominator of a dominated
// candidate is nearly always among the last few labels of that prefix (the
// labels of similar cost), so the merge tests those first.
__device__ __forceinline__ bool lex_lt(const float4 &a, const float4 &b) {
    if (a.x != b.x) return a.x < b.x;
    if (a.y != b.y) return a.y < b.y;
    if (a.z != b.z) return a.z < b.z;
    return __float_as_uint(a.w) < __float_as_uint(b.w);
}
// drift and max-drift part of weak dominance (the cost part is known)
__device__ __forceinline__ bool dm_le(const float4 &b, const float4 &q) {
    return b.y <= q.y && b.z <= q.z;
}

struct MergeLds {
    float4 *B;      // the front being built, lexicographic order (LDS or spill space)
    uint8_t *bdead; // flags for B
    bool spilled;   // B lives in the block's global spill space
    float4 *Bl;     // [capB] LDS staging of the front
    uint8_t *bdeadl;
    float4 *Bg0, *Bg1;  // [capG] each: this block's global spill space (double buffer)
    uint8_t *bdeadg;    // [capG]
    int capG;
    float4 *C;      // [capC] candidates of the current chunk
    uint8_t *cdead; // [capC]
    int *e_off;     // [blockDim] frontier offset of the in-neighbour
    int *e_pre;     // [blockDim] inclusive prefix of candidate counts
    float *e_c;     // [blockDim] edge cost
    float *e_d;     // [blockDim] edge drift
    int *u_idx;     // [capC] candidates still undecided after the near scan
    int *u_end;     // [capC] per candidate: end of the bucket prefix left to scan
    int *scan;      // [32]
    int *misc;      // [8]
    float *segd;    // [segcap] per 64-label segment: least d
    float *segm;    // [segcap] per 64-label segment: least m
    int segcap;
    int capB;       // LDS staging capacity of a front (labels)
    int capC;       // candidate chunk capacity (labels)
};


// ------------------------------------------------------------ merge groups
// A merge runs on a group of threads: the whole workgroup (workgroup
// barriers), or one half of it, so that the two halves merge two targets at
// once.  A half synchronises through LDS words of its own: an arrival count
// that only grows (each wave adds one per barrier without waiting for the
// result, then waits until the count reaches the waves' total for this
// barrier), and three count slots used in rotation.  A half's merge reads
// global memory but writes it only in its write-back, which no other thread
// of the half reads, so its barriers order LDS only.
template <bool kHalf>
struct Grp {
    int tid;   // thread index in the group
    int nt;    // threads in the group
    int w;     // wave index in the group
    int nw;    // waves in the group
    int *bar;  // kHalf: LDS words {arrivals, unused, three count slots}
    int k;     // kHalf: gcount calls so far, modulo 3 (selects the slot)
    int *err;  // kHalf: error word (a barrier wait beyond its bound sets kErrTimeout)
    unsigned arrive;  // kHalf: the arrival count that ends the last barrier
};

// polls of a half's barrier before it gives up (about 0.1 s; a wait is
// normally one merge step)
constexpr unsigned kHalfSpinLimit = 1u << 20;

__device__ __forceinline__ Grp<false> whole_group() {
    return Grp<false>{(int)threadIdx.x, (int)blockDim.x,
                      __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)),
                      (int)(blockDim.x >> 6), nullptr, 0, nullptr, 0};
}

template <bool kHalf>
__device__ __forceinline__ void gsync(Grp<kHalf> &gp) {
    if constexpr (!kHalf) {
        __syncthreads();
    } else {
        // this wave's LDS writes complete before it arrives
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        gp.arrive += (unsigned)gp.nw;
        if (lane_id() == 0) {
            int *cnt = gp.bar;
            __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            unsigned polls = 0;
            // (the difference, not the values, is compared: the count may wrap)
            while ((int)((unsigned)__hip_atomic_load(cnt, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_WORKGROUP) -
                         gp.arrive) < 0) {
                __builtin_amdgcn_s_sleep(1);
                if (++polls > kHalfSpinLimit) {
                    atomicOr(gp.err, kErrTimeout);
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    }
}

// number of threads of the group with p set (every thread calls)
template <bool kHalf>
__device__ __forceinline__ int gcount(Grp<kHalf> &gp, bool p) {
    if constexpr (!kHalf) {
        return __syncthreads_count(p);
    } else {
        int *slot = gp.bar + 2;
        const int cur = gp.k, nxt = gp.k == 2 ? 0 : gp.k + 1;
        gp.k = nxt;
        // the next call's slot was last read before the previous barrier
        if (gp.tid == 0) slot[nxt] = 0;
        const uint64_t m = ballot64(p);
        if (lane_id() == 0 && m) atomicAdd(&slot[cur], (int)__popcll(m));
        gsync(gp);
        return slot[cur];
    }
}

template <bool kHalf>
__device__ __forceinline__ bool gor(Grp<kHalf> &gp, bool p) {
    if constexpr (!kHalf) return __syncthreads_or(p) != 0;
    else return gcount(gp, p) != 0;
}

// group-wide exclusive scan of one int per thread (scratch: one int per wave)
template <bool kHalf>
__device__ __forceinline__ int g_excl_scan(Grp<kHalf> &gp, int v, int *scratch, int *total) {
    const int l = lane_id();
    const int incl = wave_incl_scan_add(v);
    gsync(gp);
    if (l == 63) scratch[gp.w] = incl;
    gsync(gp);
    int before = 0, all = 0;
    for (int i = 0; i < gp.nw; ++i) {
        const int t = scratch[i];
        if (i < gp.w) before += t;
        all += t;
    }
    *total = all;
    gsync(gp);
    return before + incl - v;
}

template <bool kHalf>
__device__ __forceinline__ long long g_min_ll(Grp<kHalf> &gp, long long v, long long *scratch) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, (long long)__shfl_xor(v, o, 64));
    gsync(gp);
    if (lane_id() == 0) scratch[gp.w] = v;
    gsync(gp);
    long long r = scratch[0];
    for (int i = 1; i < gp.nw; ++i) r = min(r, scratch[i]);
    gsync(gp);
    return r;
}

template <bool kHalf>
__device__ __forceinline__ float g_min(Grp<kHalf> &gp, float v, float *scratch) {
    v = wave_min(v);
    gsync(gp);
    if (lane_id() == 0) scratch[gp.w] = v;
    gsync(gp);
    float r = MPAP_INF;
    for (int i = 0; i < gp.nw; ++i) r = fminf(r, scratch[i]);
    gsync(gp);
    return r;
}


// compact the alive entries of arr[0..n) to the front, stable.
template <bool kHalf>
__device__ int compact_alive(Grp<kHalf> &gp, float4 *arr, const uint8_t *dead, int n, int *scan) {
    int out = 0;
    for (int t0 = 0; t0 < n; t0 += gp.nt) {
        const int i = t0 + gp.tid;
        const bool alive = i < n && !dead[i];
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (alive) v = arr[i];
        int tot;
        const int ex = g_excl_scan(gp, alive ? 1 : 0, scan, &tot);
        if (alive) arr[out + ex] = v;
        out += tot;
        gsync(gp);
    }
    return out;
}

// first index j of the sorted arr[0..n) with arr[j].c > c
__device__ __forceinline__ int upper_c(const float4 *arr, int n, float c) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (arr[mid].x <= c) lo = mid + 1; else hi = mid;
    }
    return lo;
}
// first index j of the sorted arr[0..n) with arr[j].c >= c
__device__ __forceinline__ int lower_c(const float4 *arr, int n, float c) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (arr[mid].x < c) lo = mid + 1; else hi = mid;
    }
    return lo;
}
// number of entries of the sorted arr[0..n) lexicographically below v
__device__ __forceinline__ int lex_rank(const float4 *arr, int n, const float4 &v) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (lex_lt(arr[mid], v)) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// block-wide bitonic sort of v[0..n), n a power of two
template <bool kHalf>
__device__ void bitonic_sort(Grp<kHalf> &gp, float4 *v, int n) {
    for (int k = 2; k <= n; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = gp.tid; i < n; i += gp.nt) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const float4 p = v[i], q = v[ixj];
                    const bool up = (i & k) == 0;
                    if (lex_lt(q, p) == up) {
                        v[i] = q;
                        v[ixj] = p;
                    }
                }
            }
            gsync(gp);
        }
    }
}

// Per 64-label segment of the sorted arr[0..n): the least d and the least m.
// A segment whose least d exceeds q.d (or least m exceeds q.m) holds no label
// that weakly dominates q, so dominance scans skip it.  Returns false (and
// writes nothing) when the n labels need more than segcap segments.
template <bool kHalf>
__device__ bool seg_summary(Grp<kHalf> &gp, const float4 *arr, int n, float *sd, float *sm,
                            int segcap) {
    const int l = lane_id(), w = gp.w, nw = gp.nw;
    const int nseg = (n + 63) >> 6;
    if (nseg > segcap) return false;
    for (int sg = w; sg < nseg; sg += nw) {
        const int i = sg * 64 + l;
        float d = MPAP_INF, m = MPAP_INF;
        if (i < n) {
            const float4 v = arr[i];
            d = v.y;
            m = v.z;
        }
        d = wave_min(d);
        m = wave_min(m);
        if (l == 0) {
            sd[sg] = d;
            sm[sg] = m;
        }
    }
    gsync(gp);
    return true;
}

// does some label of the sorted arr[0..end) weakly dominate q (its cost is
// known to be <= q's)?  Scanned from the top, segment by segment, by the gs
// threads of a group (sub = rank in the group); flag is the group's shared
// result, polled between segments.
__device__ __forceinline__ bool any_dominates(const float4 *arr, int end, const float4 &q,
                                              const float *sd, const float *sm, bool use_seg,
                                              int gs, int sub, const uint8_t *flag) {
    for (int sg = (end - 1) >> 6; sg >= 0; --sg) {
        if (use_seg && !(sd[sg] <= q.y && sm[sg] <= q.z)) continue;
        const int lo = sg << 6;
        int j = min(end, lo + 64) - 1 - sub;
        // four independent reads of (d, m) per step: a label that does not
        // dominate is usually followed by more such, and the answer does not
        // depend on the order of the tests
        for (; j - 3 * gs >= lo; j -= 4 * gs) {
            const float d0 = arr[j].y, m0 = arr[j].z;
            const float d1 = arr[j - gs].y, m1 = arr[j - gs].z;
            const float d2 = arr[j - 2 * gs].y, m2 = arr[j - 2 * gs].z;
            const float d3 = arr[j - 3 * gs].y, m3 = arr[j - 3 * gs].z;
            if ((int)(d0 <= q.y && m0 <= q.z) | (int)(d1 <= q.y && m1 <= q.z) |
                (int)(d2 <= q.y && m2 <= q.z) | (int)(d3 <= q.y && m3 <= q.z))
                return true;
        }
        for (; j >= lo; j -= gs)
            if (dm_le(arr[j], q)) return true;
        if (flag && *(volatile const uint8_t *)flag) return false;
    }
    return false;
}

// block-wide exclusive prefix minimum of one float per thread (scratch: one
// float per wave); every thread calls
template <bool kHalf>
__device__ __forceinline__ float g_excl_min(Grp<kHalf> &gp, float v, float *scratch) {
    const int l = lane_id(), w = gp.w;
    float incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const float u = __shfl_up(incl, o, 64);
        if (l >= o) incl = fminf(incl, u);
    }
    float ex = __shfl_up(incl, 1, 64);
    if (l == 0) ex = MPAP_INF;
    gsync(gp);
    if (l == 63) scratch[w] = incl;
    gsync(gp);
    float before = MPAP_INF;
    for (int i = 0; i < w; ++i) before = fminf(before, scratch[i]);
    gsync(gp);
    return fminf(before, ex);
}

constexpr int kPairMax = 256;  // survivors handled by the all-pairs step (at most capC / 2)
constexpr int kChunkFill = 192; // candidates gathered before a chunk is merged

// claims a slot for each lane with keep set, at *counter (LDS), one atomic per
// wave; the slots of one call are dense but in no particular order
__device__ __forceinline__ void wave_append(bool keep, int *counter, int &slot) {
    const uint64_t m = ballot64(keep);
    int base = 0;
    if (lane_id() == 0 && m) base = atomicAdd(counter, (int)__popcll(m));
    base = __shfl(base, 0, 64);
    slot = base + lanes_below(m);
}

// P(x) <- Min(P(x) U C): B[0..nB) sorted, C[0..nC) unsorted; result sorted in B.
// With two objectives (m = 0 everywhere) a Pareto front sorted by cost has
// strictly falling drift, so the only possible dominator of a label among
// the front's labels of cost <= its own is the last of them: every test is a
// binary search.  With three objectives the tests scan cost prefixes,
// skipping 64-label segments that cannot hold a dominator.
// lo: lowered to the first index of B this merge changes (labels below it
// keep their places).  The append counters misc[6] and misc[7] must be zero
// on entry.
// 1. First bucket test of candidate q against the front B[0..nB).  Two
// objectives: the last label of cost <= q.c decides.  Three: the near_scan
// labels just below q's cost are tested; `stop` is the end of the bucket
// prefix still to scan (0: decided).
__device__ __forceinline__ bool near_dead(const float4 *B, int nB, const float4 &q, int near_scan,
                                          bool three, int &stop) {
    const int k = upper_c(B, nB, q.x);
    stop = 0;
    if (!three) return k > 0 && B[k - 1].y <= q.y;
    const int st = max(0, k - near_scan);
    bool dead = false;
    for (int j = k - 1; j >= st && !dead; --j) dead = dm_le(B[j], q);
    if (!dead) stop = st;
    return dead;
}

// `prescanned`: the candidates have passed the first test already (none
// dead, the undecided ones listed in u_idx[0..misc[6]) with their u_end).
// kWide: the all-pairs survivor step keeps four reads in flight (more
// registers; the wave-first build, whose single-wave merges share the
// kernel, keeps one).
template <bool kWide, bool kHalf>
__device__ __forceinline__ bool merge_chunk(MergeLds &s, Grp<kHalf> &gp, int &nB, int nC, int near_scan,
                            bool three, int &lo, int *err, bool prescanned) {
    const int bd = gp.nt;
    const int capB = s.capB;
    if (!prescanned) {
        // 1. first test; 2. list the undecided candidates
        for (int t0 = 0; t0 < nC; t0 += bd) {
            const int i = t0 + gp.tid;
            bool und = false;
            if (i < nC) {
                int stop;
                const bool dead = near_dead(s.B, nB, s.C[i], near_scan, three, stop);
                s.cdead[i] = dead ? 1 : 0;
                s.u_end[i] = stop;
                und = stop > 0;
            }
            int slot;
            wave_append(und, &s.misc[6], slot);
            if (und) s.u_idx[slot] = i;
        }
        gsync(gp);
    }
    if (three) {
        const int nU = s.misc[6];
        // 3. the rest of the prefix, gs threads per candidate, by segments
        if (nU > 0) {
            const bool use_seg = seg_summary(gp, s.B, nB, s.segd, s.segm, s.segcap);
            int gs = 1;
            while (gs < 64 && gs * 2 * nU <= bd) gs <<= 1;
            const int per_round = bd / gs;
            for (int base = 0; base < nU; base += per_round) {
                const int u = base + gp.tid / gs;
                const int sub = gp.tid % gs;
                if (u < nU) {
                    const int i = s.u_idx[u];
                    if (any_dominates(s.B, s.u_end[i], s.C[i], s.segd, s.segm, use_seg, gs, sub,
                                      &s.cdead[i]))
                        s.cdead[i] = 1;
                }
            }
            gsync(gp);
        }
    }
    // 4. survivors of the bucket test, gathered (any order) into tmp (the
    // undecided-scan space, free now) while they fit the all-pairs step
    // (u_idx and u_end, adjacent: capC / 2 labels)
    float4 *tmp = reinterpret_cast<float4 *>(s.u_idx);
    const int pair_max = min(min(kPairMax, s.capC / 2), bd);  // one thread or more each
    for (int t0 = 0; t0 < nC; t0 += bd) {
        const int i = t0 + gp.tid;
        const bool alive = i < nC && !s.cdead[i];
        int slot;
        wave_append(alive, &s.misc[7], slot);
        if (alive && slot < pair_max) tmp[slot] = s.C[i];
    }
    gsync(gp);
    const int nS = s.misc[7];
    if (nS == 0) return true;
    int nS2;
    if (nS <= pair_max) {
        // 4-5 for up to pair_max survivors, all pairs at once: g threads per
        // survivor, each over a slice of the others.  A survivor dies if a
        // lexicographically smaller one dominates it; its rank among the
        // living ones is its place in the sorted run.
        int g = 1;
        while (g < 64 && g * 2 * nS <= bd) g <<= 1;
        const int i = gp.tid / g, sub = gp.tid % g;
        const bool mine = i < nS;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        bool dead = false;
        // (four independent LDS reads in flight per step)
        if (mine) {
            v = tmp[i];
            int j = sub;
            if constexpr (kWide)
            for (; j + 3 * g < nS; j += 4 * g) {
                const float4 o0 = tmp[j], o1 = tmp[j + g], o2 = tmp[j + 2 * g], o3 = tmp[j + 3 * g];
                // (bitwise on purpose: the four tests without branches)
                dead |= (int)(lex_lt(o0, v) && dm_le(o0, v)) | (int)(lex_lt(o1, v) && dm_le(o1, v)) |
                        (int)(lex_lt(o2, v) && dm_le(o2, v)) | (int)(lex_lt(o3, v) && dm_le(o3, v));
            }
            for (; j < nS; j += g) {
                const float4 o = tmp[j];
                dead |= lex_lt(o, v) && dm_le(o, v);
            }
        }
        for (int o = 1; o < g; o <<= 1) dead = __shfl_xor((int)dead, o, 64) != 0 || dead;
        if (mine && sub == 0) s.cdead[i] = dead ? 1 : 0;
        gsync(gp);
        int pos = 0;
        if (mine && !dead) {
            int j = sub;
            if constexpr (kWide)
            for (; j + 3 * g < nS; j += 4 * g) {
                const float4 o0 = tmp[j], o1 = tmp[j + g], o2 = tmp[j + 2 * g], o3 = tmp[j + 3 * g];
                const int d0 = s.cdead[j], d1 = s.cdead[j + g], d2 = s.cdead[j + 2 * g],
                          d3 = s.cdead[j + 3 * g];
                pos += (!d0 && lex_lt(o0, v)) + (!d1 && lex_lt(o1, v)) + (!d2 && lex_lt(o2, v)) +
                       (!d3 && lex_lt(o3, v));
            }
            for (; j < nS; j += g) pos += (!s.cdead[j] && lex_lt(tmp[j], v)) ? 1 : 0;
        }
        for (int o = 1; o < g; o <<= 1) pos += __shfl_xor(pos, o, 64);
        const bool lead = mine && sub == 0 && !dead;
        if (lead) s.C[pos] = v;  // tmp is the input, C the sorted output
        nS2 = gcount(gp, lead);
    } else {
        // many survivors: compact them in place, sort, sweep
        const int nSc = compact_alive(gp, s.C, s.cdead, nC, s.scan);
        (void)nSc;
        int P = 1;
        while (P < nS) P <<= 1;
        for (int i = nS + gp.tid; i < P; i += bd)
            s.C[i] = make_float4(MPAP_INF, MPAP_INF, MPAP_INF, __uint_as_float(0xffffffffu));
        gsync(gp);
        bitonic_sort(gp, s.C, P);
        // 5. candidates among themselves: an earlier (lexicographically
        // smaller) one may dominate
        if (!three) {
        float carry = MPAP_INF;
        for (int t0 = 0; t0 < nS; t0 += bd) {
            const int i = t0 + gp.tid;
            const float d = i < nS ? s.C[i].y : MPAP_INF;
            const float ex = fminf(carry, g_excl_min(gp, d, reinterpret_cast<float *>(s.scan)));
            if (i < nS) s.cdead[i] = ex <= d ? 1 : 0;
            carry = fminf(carry, g_min(gp, d, reinterpret_cast<float *>(s.scan)));
        }
        gsync(gp);
        } else {
            const bool seg = seg_summary(gp, s.C, nS, s.segd, s.segm, s.segcap);
            for (int i = gp.tid; i < nS; i += bd)
                s.cdead[i] =
                    any_dominates(s.C, i, s.C[i], s.segd, s.segm, seg, 1, 0, nullptr) ? 1 : 0;
            gsync(gp);
        }
        nS2 = compact_alive(gp, s.C, s.cdead, nS, s.scan);
    }
    // 6. bucket labels a surviving candidate dominates leave (only labels at
    // least as costly as the cheapest survivor can be dominated)
    bool any_dead = false;
    long long first_dead = nB;
    const int js = lower_c(s.B, nB, s.C[0].x);
    if (!three) {
        for (int j = js + gp.tid; j < nB; j += bd) {
            const float4 b = s.B[j];
            const int kk = upper_c(s.C, nS2, b.x);
            const bool dead = kk > 0 && s.C[kk - 1].y <= b.y;
            s.bdead[j] = dead ? 1 : 0;
            any_dead = any_dead || dead;
            if (dead) first_dead = min(first_dead, (long long)j);
        }
    } else {
        const bool seg = nS2 > 64 && seg_summary(gp, s.C, nS2, s.segd, s.segm, s.segcap);
        for (int j = js + gp.tid; j < nB; j += bd) {
            const float4 b = s.B[j];
            const int kk = upper_c(s.C, nS2, b.x);
            const bool dead = any_dominates(s.C, kk, b, s.segd, s.segm, seg, 1, 0, nullptr);
            s.bdead[j] = dead ? 1 : 0;
            any_dead = any_dead || dead;
            if (dead) first_dead = min(first_dead, (long long)j);
        }
    }
    int nBs = nB;
    if (gor(gp, any_dead)) {
        // labels below the first removed one keep their places
        const int fd = (int)g_min_ll(gp, first_dead, reinterpret_cast<long long *>(s.scan));
        lo = min(lo, fd);
        nBs = fd + compact_alive(gp, s.B + fd, s.bdead + fd, nB - fd, s.scan);
    }
    // the first survivor's place: labels below it keep their places
    const int r0 = lex_rank(s.B, nBs, s.C[0]);
    lo = min(lo, r0);
    const int total = nBs + nS2;
    if constexpr (kHalf) {
        // a half has no spill space: the merge backs out (nothing was written
        // to global memory) and the whole workgroup merges the target again
        if (total > capB) {
            nB = nBs;
            gsync(gp);
            return false;
        }
    }
    if (total > (s.spilled ? s.capG : capB) && (s.spilled || total > s.capG)) {
        if (gp.tid == 0) atomicOr(err, kErrBucket);
        nB = nBs;
        gsync(gp);
        return true;
    }
    if (s.spilled || total > capB) {
        // 7a. merge out of place into the (other) spill buffer
        float4 *outb = (s.spilled && s.B == s.Bg0) ? s.Bg1 : s.Bg0;
        for (int k = gp.tid; k < nBs; k += bd) {
            const float4 v = s.B[k];
            outb[k + lex_rank(s.C, nS2, v)] = v;
        }
        for (int i = gp.tid; i < nS2; i += bd) {
            const float4 v = s.C[i];
            outb[i + lex_rank(s.B, nBs, v)] = v;
        }
        s.B = outb;
        s.bdead = s.bdeadg;
        s.spilled = true;
        nB = total;
        gsync(gp);
        return true;
    }
    // 7b. merge the two sorted runs in place in LDS.  Positions by rank: the
    // survivors' places are found first (B still intact); B's labels only
    // move up, so B is moved chunk by chunk from the top (each chunk read,
    // then written, never over a label still to be read); the survivors go
    // to their places last.
    for (int i = gp.tid; i < nS2; i += bd) s.u_idx[i] = i + lex_rank(s.B, nBs, s.C[i]);
    gsync(gp);
    for (int top = nBs; top > r0; top -= bd) {
        const int k = top - bd + gp.tid;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        int pos = -1;
        if (k >= r0) {
            v = s.B[k];
            pos = k + lex_rank(s.C, nS2, v);
        }
        gsync(gp);
        if (pos >= 0) s.B[pos] = v;
        gsync(gp);
    }
    for (int i = gp.tid; i < nS2; i += bd) s.B[s.u_idx[i]] = s.C[i];
    nB = total;
    gsync(gp);
    return true;
}

// ------------------------------------------------ single-wave merges (small fronts)
// A target whose front holds at most wcap labels is merged by one wave in its
// own LDS slice, without workgroup barriers, so the 16 waves of a workgroup
// merge 16 targets at once.  The steps are those of merge_chunk, per chunk
// of 64 children (one per lane).  A front that would outgrow the slice is
// left untouched (nothing is written back) and handed to the workgroup path.
struct WaveLds {
    float4 *B;    // [wcap] the front, lexicographic order
    float4 *C;    // [64] the chunk's children
    float *sd;    // [wcap/64] per segment of B: least d
    float *sm;    // [wcap/64] per segment of B: least m
    uint8_t *bd;  // [wcap] flags of B
    uint8_t *cd;  // [64] flags of C (1: dead)
};

__device__ void carve_wave(unsigned char *lds, const SearchArgs &a, WaveLds &w) {
    unsigned char *p = lds + (size_t)(threadIdx.x >> 6) * a.wslice;
    w.B = reinterpret_cast<float4 *>(p);
    p += 16 * (size_t)a.wcap;
    w.C = reinterpret_cast<float4 *>(p);
    p += 16 * 64;
    w.sd = reinterpret_cast<float *>(p);
    p += 4 * (size_t)(a.wcap / 64);
    w.sm = reinterpret_cast<float *>(p);
    p += 4 * (size_t)(a.wcap / 64);
    w.bd = p;
    p += a.wcap;
    w.cd = p;
}

// LDS writes of the wave's lanes visible to its other lanes
__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_min_i(int v) { return -wave_max_i(-v); }

// segment summaries of the wave's front B[0..n)
__device__ void wave_seg_summary(const WaveLds &W, int n) {
    const int l = lane_id();
    for (int sg = 0; sg < ((n + 63) >> 6); ++sg) {
        const int i = sg * 64 + l;
        float d = MPAP_INF, m = MPAP_INF;
        if (i < n) {
            d = W.B[i].y;
            m = W.B[i].z;
        }
        d = wave_min(d);
        m = wave_min(m);
        if (l == 0) {
            W.sd[sg] = d;
            W.sm[sg] = m;
        }
    }
    wsync();
}

// Returns false when the front would outgrow the slice (the target then
// goes to the workgroup path; nothing has been written).  kObj: 2 or 3 when
// every query has that many objectives, 0 when the query decides.
template <int kObj>
__device__ bool wave_merge_node(const SearchArgs &a, int x, int wave, const WaveLds &W,
                                long long &cand_out) {
    const int l = lane_id();
    const int4 nbx = a.nb[x];
    int nB = nbx.z;
    if (nB > a.wcap) return false;
    for (int i = l; i < nB; i += 64) W.B[i] = a.pool[(size_t)(unsigned)nbx.x + i];
    wsync();
    const bool rst = (a.nflag[x] & 1u) != 0u;
    const int q = (a.nq > 1) ? query_of(a, x) : 0;
    const float beta = a.qbeta[q];
    const bool three = kObj == 0 ? a.qnobj[q] >= 3 : kObj == 3;
    const float *edrift = a.qheur[q] ? a.sdrift : a.rdrift;
    if (three) wave_seg_summary(W, nB);
    int lo = nB;
    bool changed = false;
    long long cand = 0;
    const int e1 = a.rptr[x + 1];
    for (int t0 = a.rptr[x]; t0 < e1; t0 += 64) {
        // 64 in-edges at once: group sizes of their sources, packed by a prefix
        const int e = t0 + l;
        int cnt = 0, off = 0;
        float ce = 0.f, de = 0.f;
        if (e < e1) {
            const int4 fu = a.fo[a.rsrc[e]];
            if (fu.z == wave) {
                cnt = fu.y;
                off = fu.x;
                ce = a.rcost[e];
                de = edrift[e];
            }
        }
        const int pre = wave_incl_scan_add(cnt);
        const int tot = __shfl(pre, 63, 64);
        for (int j0 = 0; j0 < tot; j0 += 64) {
            // child j of the tile: in-edge t = first lane with prefix > j
            const int j = j0 + l;
            float4 ch = make_float4(0.f, 0.f, 0.f, 0.f);
            bool alive = false;
            {
                int lo2 = 0, hi2 = 63;
                while (lo2 < hi2) {
                    const int mid = (lo2 + hi2) >> 1;
                    if (__shfl(pre, mid, 64) > j) hi2 = mid; else lo2 = mid + 1;
                }
                const int t = lo2;
                // every lane takes part in each shuffle (a lane not executing
                // one would hand 0 to the lanes reading from it)
                const int pb = __shfl(pre, t > 0 ? t - 1 : 0, 64);
                const int before = t > 0 ? pb : 0;
                const int o_t = __shfl(off, t, 64);
                const float ce_t = __shfl(ce, t, 64), de_t = __shfl(de, t, 64);
                if (j < tot) {
                    const float4 P = a.F[o_t + (j - before)];
                    const float c2 = P.x + ce_t;
                    const float dpre = P.y + de_t;
                    alive = dpre <= beta;
                    const float d2 = rst ? 0.0f : dpre;
                    const float m2 = three ? fmaxf(P.z, dpre) : 0.0f;
                    const unsigned meta = MPAP_OPEN_BIT | (unsigned)(__float_as_int(P.w) + 1);
                    ch = make_float4(c2, d2, m2, __uint_as_float(meta));
                }
            }
            cand += alive ? 1 : 0;
            // bucket test
            if (!three) {
                if (alive) {
                    const int kk = upper_c(W.B, nB, ch.x);
                    alive = !(kk > 0 && W.B[kk - 1].y <= ch.y);
                }
            } else {
                // near scan per lane, then the rest of each undecided child's
                // prefix by the whole wave, 64 labels a step
                int stop = 0;
                if (alive) {
                    const int kk = upper_c(W.B, nB, ch.x);
                    stop = max(0, kk - a.near_scan);
                    for (int jj = kk - 1; jj >= stop && alive; --jj) alive = !dm_le(W.B[jj], ch);
                }
                uint64_t um = ballot64(alive && stop > 0);
                while (um) {
                    const int src = (int)__ffsll((unsigned long long)um) - 1;
                    um &= um - 1;
                    float4 qv;
                    qv.x = __shfl(ch.x, src, 64);
                    qv.y = __shfl(ch.y, src, 64);
                    qv.z = __shfl(ch.z, src, 64);
                    const int end = __shfl(stop, src, 64);
                    bool dom = false;
                    for (int sg = (end - 1) >> 6; sg >= 0 && !dom; --sg) {
                        if (!(W.sd[sg] <= qv.y && W.sm[sg] <= qv.z)) continue;
                        const int jj = (sg << 6) + l;
                        dom = ballot64(jj < end && dm_le(W.B[jj], qv)) != 0;
                    }
                    if (l == src) alive = !dom;
                }
            }
            const uint64_t am = ballot64(alive);
            const int na = (int)__popcll(am);
            if (na == 0) continue;
            // children among themselves: a lexicographically smaller one may
            // dominate; the survivors end up in W.C[0..ns)
            if (alive) W.C[lanes_below(am)] = ch;
            wsync();
            bool dead = true;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (l < na) {
                v = W.C[l];
                dead = false;
                for (int jj = 0; jj < na && !dead; ++jj) {
                    const float4 o = W.C[jj];
                    dead = lex_lt(o, v) && dm_le(o, v);
                }
            }
            const uint64_t smask = ballot64(!dead);
            const int ns = (int)__popcll(smask);
            wsync();
            if (!dead) W.C[lanes_below(smask)] = v;
            wsync();
            // front labels a survivor dominates leave (only those at least as
            // costly as the cheapest survivor)
            const float cmin = wave_min(dead ? MPAP_INF : v.x);
            const int js = lower_c(W.B, nB, cmin);
            int fd = nB;
            for (int i = js + l; i < nB; i += 64) {
                const float4 bl = W.B[i];
                bool bdd = false;
                for (int jj = 0; jj < ns && !bdd; ++jj) {
                    const float4 o = W.C[jj];
                    bdd = o.x <= bl.x && dm_le(o, bl);
                }
                W.bd[i] = bdd ? 1 : 0;
                if (bdd) fd = min(fd, i);
            }
            fd = wave_min_i(fd);
            wsync();
            int nBs = nB;
            if (fd < nB) {
                // stable compaction from the first removed label; each chunk is
                // read before it is written, and writes never pass the reads
                int out = fd;
                for (int c0 = fd; c0 < nB; c0 += 64) {
                    const int i = c0 + l;
                    const bool keep = i < nB && !W.bd[i];
                    float4 u = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (keep) u = W.B[i];
                    const uint64_t km = ballot64(keep);
                    wsync();
                    if (keep) W.B[out + lanes_below(km)] = u;
                    out += (int)__popcll(km);
                    wsync();
                }
                nBs = out;
                lo = min(lo, fd);
            }
            if (nBs + ns > a.wcap) return false;
            // the survivors' places, then B moved up from the top, then the survivors
            int pos = -1, r = 0x7fffffff;
            if (l < ns) {
                const float4 sv = W.C[l];
                int rs = 0;
                for (int jj = 0; jj < ns; ++jj) rs += lex_lt(W.C[jj], sv) ? 1 : 0;
                r = lex_rank(W.B, nBs, sv);
                pos = r + rs;
                v = sv;
            }
            const int r0 = wave_min_i(r);
            for (int top = nBs; top > r0; top -= 64) {
                const int i = top - 64 + l;
                float4 u = make_float4(0.f, 0.f, 0.f, 0.f);
                int np = -1;
                if (i >= r0) {
                    u = W.B[i];
                    int c = 0;
                    for (int jj = 0; jj < ns; ++jj) c += lex_lt(W.C[jj], u) ? 1 : 0;
                    np = i + c;
                }
                wsync();
                if (np >= 0) W.B[np] = u;
                wsync();
            }
            if (l < ns) W.B[pos] = v;
            wsync();
            nB = nBs + ns;
            lo = min(lo, r0);
            changed = true;
            if (three) wave_seg_summary(W, nB);
        }
    }
    cand = wave_sum(cand);
    if (l == 0) cand_out += cand;
    if (!changed) return true;
    // write back the changed suffix (a fresh region if the front outgrew its own)
    int off = nbx.x, cap = nbx.y;
    if (nB > cap) {
        int o = 0, nc = 16;
        while (nc < nB) nc <<= 1;
        if (l == 0) {
            o = (int)atomicAdd(a.pool_top, (unsigned)nc);
            if ((unsigned long long)(unsigned)o + (unsigned)nc > a.pool_cap) {
                atomicOr(a.err, kErrPool);
                o = -1;
            }
        }
        o = __shfl(o, 0, 64);
        if (o < 0) return true;
        off = o;
        cap = nc;
        lo = 0;
    }
    float mn = MPAP_INF;
    int nopen = 0, first = nB;
    for (int i = l; i < nB; i += 64) {
        const float4 L = W.B[i];
        if (i >= lo) a.pool[(size_t)(unsigned)off + i] = L;
        if (lab_open(L)) {
            mn = fminf(mn, L.x);
            ++nopen;
            first = min(first, i);
        }
    }
    mn = wave_min(mn);
    nopen = wave_sum(nopen);
    first = wave_min_i(first);
    if (l == 0) {
        a.nb[x] = make_int4(off, cap, nB, nopen);
        reinterpret_cast<int *>(&a.fo[x])[3] = first;
        a.minopen[x] = mn;
    }
    return true;
}

// Stage P(x) (pool region nbv) for merging: LDS if it fits, else spill space
// (whole workgroup only: false for a half, which then leaves the target to
// the whole workgroup, and false with an error when the spill space is too
// small).
template <bool kHalf>
__device__ bool stage_front(const SearchArgs &a, MergeLds &s, Grp<kHalf> &gp, const int4 &nbv) {
    s.spilled = nbv.z > s.capB;
    if constexpr (kHalf) {
        if (s.spilled) return false;
    }
    s.B = s.spilled ? s.Bg0 : s.Bl;
    s.bdead = s.spilled ? s.bdeadg : s.bdeadl;
    if (nbv.z > (s.spilled ? s.capG : s.capB)) {
        if (gp.tid == 0) atomicOr(a.err, kErrBucket);
        return false;
    }
    for (int i = gp.tid; i < nbv.z; i += gp.nt) s.B[i] = a.pool[(size_t)(unsigned)nbv.x + i];
    gsync(gp);
    return true;
}

// Merges the children of x's in-neighbours' group labels into P(x).  Returns
// false when a half backs out (the front outgrows the half's LDS stage;
// nothing was written), true otherwise.
template <bool kWide, int kObj, bool kHalf>
__device__ __forceinline__ bool merge_node(const SearchArgs &a, int x, int wave, MergeLds &s,
                                           Grp<kHalf> &gp,
                           long long &st_cand) {
    const int4 nbx = a.nb[x];
    int nB = nbx.z;
    int lo = nB;  // first index the merges change
    if (!stage_front(a, s, gp, nbx)) return !kHalf;
    const bool rst = (a.nflag[x] & 1u) != 0u;
    const int q = (a.nq > 1) ? query_of(a, x) : 0;
    const float beta = a.qbeta[q];
    const bool three = kObj == 0 ? a.qnobj[q] >= 3 : kObj == 3;
    const float *edrift = a.qheur[q] ? a.sdrift : a.rdrift;
    const int e0 = a.rptr[x], e1 = a.rptr[x + 1];
    bool changed = false, fits = true;
    // Children are made in rounds of up to one per thread and given the first
    // bucket test at once; those it does not kill gather in C (any order)
    // across rounds and in-edge tiles until C holds kChunkFill of them, then
    // the chunk is merged.  Testing against the front as it was before the
    // last chunk went in is sound: a label removed since is dominated by one
    // that stayed, which then dominates the child too.
    if (gp.tid == 0) {
        s.misc[4] = 0;  // children within the bound
        s.misc[5] = 0;  // candidates kept
        s.misc[6] = 0;  // undecided after the first test
        s.misc[7] = 0;  // survivors of the bucket test
    }
    gsync(gp);
    int nC = 0;  // kept so far (from the barrier counts: the same in every thread)
    auto flush = [&]() {
        fits = merge_chunk<kWide>(s, gp, nB, nC, a.near_scan, three, lo, a.err, true);
        changed = true;
        nC = 0;
        if (gp.tid == 0) {
            s.misc[5] = 0;
            s.misc[6] = 0;
            s.misc[7] = 0;
        }
        gsync(gp);
    };
    for (int t0 = e0; t0 < e1; t0 += gp.nt) {
        // in-edge tile: frontier label counts of each in-neighbour
        const int e = t0 + gp.tid;
        int cnt = 0, off = 0;
        float ce = 0.f, de = 0.f;
        if (e < e1) {
            const int u = a.rsrc[e];
            const int4 fu = a.fo[u];
            if (fu.z == wave) {
                cnt = fu.y;
                off = fu.x;
                ce = a.rcost[e];
                de = edrift[e];
            }
        }
        int tot;
        const int ex = g_excl_scan(gp, cnt, s.scan, &tot);
        s.e_off[gp.tid] = off;
        s.e_pre[gp.tid] = ex + cnt;
        s.e_c[gp.tid] = ce;
        s.e_d[gp.tid] = de;
        gsync(gp);
        const int ntile = min(gp.nt, e1 - t0);
        for (int j0 = 0; j0 < tot;) {
            if (nC >= kChunkFill) {
                flush();
                if (!fits) return false;
                continue;
            }
            // children j0 .. j0+cnt-1 of this tile (C has room for all)
            const int cnt = min(min(gp.nt, s.capC - nC), tot - j0);
            {
                const int j = j0 + gp.tid;
                bool ok = false, keep = false;
                int stop = 0;
                float4 ch = make_float4(0.f, 0.f, 0.f, 0.f);
                if (j < j0 + cnt) {
                    // in-edge t: first with inclusive prefix > j
                    int lo2 = 0, hi2 = ntile - 1;
                    while (lo2 < hi2) {
                        const int mid = (lo2 + hi2) >> 1;
                        if (s.e_pre[mid] > j) hi2 = mid; else lo2 = mid + 1;
                    }
                    const int t = lo2;
                    const int k = j - (t > 0 ? s.e_pre[t - 1] : 0);
                    const float4 P = a.F[s.e_off[t] + k];
                    const float c2 = P.x + s.e_c[t];
                    const float dpre = P.y + s.e_d[t];
                    ok = dpre <= beta;
                    const float d2 = rst ? 0.0f : dpre;
                    const float m2 = three ? fmaxf(P.z, dpre) : 0.0f;
                    const unsigned meta = MPAP_OPEN_BIT | (unsigned)(__float_as_int(P.w) + 1);
                    ch = make_float4(c2, d2, m2, __uint_as_float(meta));
                    if (ok) keep = !near_dead(s.B, nB, ch, a.near_scan, three, stop);
                }
                int slot;
                wave_append(keep, &s.misc[5], slot);
                if (keep) {
                    s.C[slot] = ch;
                    s.cdead[slot] = 0;
                    s.u_end[slot] = stop;
                }
                int us;
                wave_append(stop > 0, &s.misc[6], us);
                if (stop > 0) s.u_idx[us] = slot;
                const uint64_t okm = ballot64(ok);
                if (lane_id() == 0 && okm) atomicAdd(&s.misc[4], (int)__popcll(okm));
                nC += gcount(gp, keep);
            }
            j0 += cnt;
        }
        gsync(gp);
    }
    if (nC > 0) {
        flush();
        if (!fits) return false;
    }
    st_cand += s.misc[4];  // every append precedes the last barrier
    if (!changed) return true;
    // write the merged front back (fresh region if it outgrew the old one)
    int off = nbx.x, cap = nbx.y;
    if (nB > cap) {
        if (gp.tid == 0) {
            int nc = 16;
            while (nc < nB) nc <<= 1;
            const unsigned o = atomicAdd(a.pool_top, (unsigned)nc);
            if ((unsigned long long)o + (unsigned)nc > a.pool_cap) {
                atomicOr(a.err, kErrPool);
                s.misc[0] = -1;
            } else {
                s.misc[0] = (int)o;
                s.misc[1] = nc;
            }
        }
        gsync(gp);
        off = s.misc[0];
        cap = s.misc[1];
        gsync(gp);
        if (off < 0) return true;
        lo = 0;  // a fresh region gets the whole front
    }
    float mn = MPAP_INF;
    int nopen = 0, first = nB;
    for (int i = gp.tid; i < nB; i += gp.nt) {
        const float4 L = s.B[i];
        if (i >= lo) a.pool[(size_t)(unsigned)off + i] = L;
        if (lab_open(L)) {
            mn = fminf(mn, L.x);
            ++nopen;
            first = min(first, i);
        }
    }
    // least open cost, open count and first open index in one reduction
    mn = wave_min(mn);
    nopen = wave_sum(nopen);
    first = -wave_max_i(-first);
    const int w = gp.w, nw = gp.nw;
    if (lane_id() == 0) {
        s.e_c[w] = mn;
        s.e_off[w] = nopen;
        s.e_pre[w] = first;
    }
    gsync(gp);
    if (gp.tid == 0) {
        for (int i = 1; i < nw; ++i) {
            mn = fminf(mn, s.e_c[i]);
            nopen += s.e_off[i];
            first = min(first, s.e_pre[i]);
        }
        a.nb[x] = make_int4(off, cap, nB, nopen);
        // first open label: the count and select of the next iteration start there
        reinterpret_cast<int *>(&a.fo[x])[3] = first;
        a.minopen[x] = mn;
    }
    gsync(gp);
    return true;
}

}  // namespace

__global__ void __launch_bounds__(256) k_search_init(SearchArgs a) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < a.n) {
        a.nb[v] = make_int4(0, 0, 0, 0);
        a.minopen[v] = MPAP_INF;
        a.gcnt[v] = 0;
        a.fo[v] = make_int4(0, 0, -1, 0);
        a.mark[v] = -1;
        a.wt[v] = 0;
    }
    if (v == 0) {
        *a.pool_top = 16u * (unsigned)a.nq;
        for (int i = 0; i < 2 * kListRegions; ++i) {
            a.acnt[i] = 0;
            a.mcur[i] = 0;
        }
        *a.bar = 0u;
        *a.err = 0;
        for (int i = 0; i < kOutWords; ++i) a.out[i] = 0;
    }
    for (long long i = v; i < (long long)a.wstat_cap * kTraceWords;
         i += (long long)gridDim.x * blockDim.x)
        a.wstat[i] = 0;
}

// Root label of every query (Alg. 3 first lines): (x_init, 0, 0) open, in its
// own 16-label region.  Runs after k_search_init.
__global__ void __launch_bounds__(256) k_search_roots(SearchArgs a) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.nq) return;
    const int r = a.qroot[q];
    if (r < 0) {  // a query left out of this launch
        a.qlast[q] = -1;
        a.qstop[q] = -2;
        return;
    }
    a.qstop[q] = a.qearly[q] ? -1 : -2;
    a.nb[r] = make_int4(16 * q, 16, 1, 1);
    a.minopen[r] = 0.0f;
    a.pool[(size_t)16 * q] = make_float4(0.f, 0.f, 0.f, __uint_as_float(MPAP_OPEN_BIT));
    a.qlast[q] = 0;
}

// LDS of a merge group from `base`: a front stage of capB labels, a chunk of
// capC candidates, per-thread in-edge tiles of nt entries; spill space (the
// block's, in global memory) for the whole workgroup only.
__device__ __forceinline__ void carve_group(unsigned char *base, const SearchArgs &a, MergeLds &s, int capB,
                            int capC, int nt, bool spill) {
    unsigned char *p = base;
    s.Bl = reinterpret_cast<float4 *>(p);
    p += sizeof(float4) * capB;
    s.C = reinterpret_cast<float4 *>(p);
    p += sizeof(float4) * capC;
    s.e_off = reinterpret_cast<int *>(p);
    p += sizeof(int) * nt;
    s.e_pre = reinterpret_cast<int *>(p);
    p += sizeof(int) * nt;
    s.e_c = reinterpret_cast<float *>(p);
    p += sizeof(float) * nt;
    s.e_d = reinterpret_cast<float *>(p);
    p += sizeof(float) * nt;
    s.u_idx = reinterpret_cast<int *>(p);
    p += sizeof(int) * capC;
    s.u_end = reinterpret_cast<int *>(p);
    p += sizeof(int) * capC;
    s.scan = reinterpret_cast<int *>(p);
    p += sizeof(long long) * 16;
    s.misc = reinterpret_cast<int *>(p);
    p += sizeof(int) * 8;
    s.segcap = max(capB, capC) / 64 + 2;
    s.capB = capB;
    s.capC = capC;
    s.segd = reinterpret_cast<float *>(p);
    p += sizeof(float) * s.segcap;
    s.segm = reinterpret_cast<float *>(p);
    p += sizeof(float) * s.segcap;
    s.bdeadl = p;
    p += capB;
    s.cdead = p;
    s.capG = spill ? a.capG : 0;
    s.Bg0 = spill ? a.spill + (size_t)blockIdx.x * 2 * a.capG : nullptr;
    s.Bg1 = spill ? s.Bg0 + a.capG : nullptr;
    s.bdeadg = spill ? a.spill_flags + (size_t)blockIdx.x * a.capG : nullptr;
    s.B = s.Bl;
    s.bdead = s.bdeadl;
    s.spilled = false;
}

__device__ __forceinline__ void carve_lds(unsigned char *lds, const SearchArgs &a, MergeLds &s) {
    carve_group(lds, a, s, a.capB, a.capC, (int)blockDim.x, true);
}

// kHalves (workgroup-only build): iterations with at least a.halves_min
// targets merge by halves.  kObj: the objective count of every query (2 or
// 3), or 0 when it differs between queries.
template <bool kWaveMerges, bool kHalves, int kObj>
__device__ __forceinline__ void search_body(SearchArgs a) {
    static_assert(!(kWaveMerges && kHalves), "merges by halves are a workgroup-only build");
    extern __shared__ __align__(16) unsigned char lds[];
    // (the merge groups' LDS views are carved where they are used, so that
    // their pointers do not stay live across the loop)

    __shared__ long long red_ll[16];
    // merges by halves: each half's barrier words, and the control words
    // {stop, backed-out target of half 0 and 1, carried claim of half 0 and 1,
    // the next whole-workgroup command}
    __shared__ int hbar[2][8];
    __shared__ int hctl[8];

    const int G = (int)gridDim.x;
    const int b = (int)blockIdx.x;
    const int lo = (int)((long long)b * a.n / G);
    const int hi = (int)((long long)(b + 1) * a.n / G);

    unsigned epoch = 0;
    long long i_step = 0;  // iteration index: query q's threshold is i_step * qdelta[q]
    int wave = 0;          // number of groups expanded so far
    long long abase = a.arena_base;  // arena ids handed out so far
    int it = 0;            // loop trips (parity of the partial sums)
    long long st_merges = 0, st_cand = 0;  // workgroup merges (thread 0 counts)
    long long wv_merges = 0, wv_cand = 0;  // single-wave merges (lane 0 counts)
    // merges by halves: per half {merges, candidates, back-outs} (kept in
    // LDS by each half's first thread, so that they hold no registers)
    __shared__ unsigned long long hstat[2][3];
    if (threadIdx.x < 6) hstat[threadIdx.x / 3][threadIdx.x % 3] = 0;
    int status = kStatusOk;

    const bool tr0 = (b == 0 && threadIdx.x == 0);
    for (;;) {
        const int par = it & 1;
        long long* tr = (wave < a.wstat_cap) ? a.wstat + (size_t)wave * kTraceWords : nullptr;
        if (tr0 && tr) tr[kTrStart] = (long long)wall_clock64();
        if (threadIdx.x == 0 && b == 0) {
            for (int r = 0; r < (kWaveMerges ? 2 : kListRegions); ++r) {
                a.acnt[2 * r + wave_par(wave)] = 0;
                a.mcur[2 * r + wave_par(wave)] = 0;
            }
        }
        if (a.early_any) {
            // Alg. 3's loop condition, per query: the loop ends before a
            // group that holds a plan at a goal node, i.e. when some goal
            // node's least open cost is within this iteration's threshold
            // (every plan kept is within the bound).  One thread per query.
            for (int q = b * (int)blockDim.x + threadIdx.x; q < a.nq;
                 q += G * (int)blockDim.x) {
                if (a.qstop[q] != -1) continue;
                const float T = threshold(i_step, a.qdelta[q]);
                for (int gi = a.qgoff[q]; gi < a.qgoff[q + 1]; ++gi)
                    if (a.minopen[a.goal_list[gi]] <= T) {
                        a.qstop[q] = wave;
                        break;
                    }
            }
            grid_barrier(a.bar, G, epoch, a.err, kErrTimeout, kSpinLimit);
        }
        {
            MergeLds s;
            carve_lds(lds, a, s);
            phase_count(a, i_step, par, lo, hi, s.u_idx, s.scan, red_ll);
        }
        if (tr0 && tr) tr[kTrCountDone] = (long long)wall_clock64();
        grid_barrier(a.bar, G, epoch, a.err, kErrTimeout, kSpinLimit);
        if (tr0 && tr) tr[kTrCounted] = (long long)wall_clock64();

        // every block derives the same decisions from the same partial sums
        // (read by all its threads at once, then reduced)
        long long total = 0, before = 0, open_nodes = 0;
        long long mstep = 0x7fffffffffffffffll;
        for (int q = threadIdx.x; q < G; q += blockDim.x) {
            const long long c = a.part_cnt[par * G + q];
            if (q < b) before += c;
            total += c;
            open_nodes += a.part_open[par * G + q];
            mstep = min(mstep, a.part_step[par * G + q]);
        }
        total = block_sum_ll(total, red_ll);
        before = block_sum_ll(before, red_ll);
        open_nodes = block_sum_ll(open_nodes, red_ll);
        mstep = block_min_ll(mstep, red_ll);
        // (the barrier made the other blocks' writes visible: relaxed loads)
        const int errv = __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (errv != 0) {
            status = kStatusError;
            break;
        }
        if (open_nodes == 0) break;  // P_open is empty
        ++it;
        if (it > 2 * a.max_waves + 64 || (total == 0 && mstep == 0x7fffffffffffffffll)) {
            status = kStatusNoConverge;
            break;
        }
        if (total == 0) {
            // empty group: skip to the first iteration whose group is not
            // empty (the least step that reaches some open label)
            i_step = max(mstep, i_step + 1);
            continue;
        }
        if (wave >= a.max_waves) {
            status = kStatusNoConverge;
            break;
        }
        if (abase + total > a.arena_cap || total > a.F_cap) {
            status = kStatusArena;
            if (b == 0 && threadIdx.x == 0) a.out[kOutNeed] = total;
            break;
        }
        {
            MergeLds s;
            carve_lds(lds, a, s);
            phase_select<kWaveMerges>(a, i_step, wave, abase, before, lo, hi, s.u_idx, s.u_end,
                                      s.scan);
        }
        if (tr0 && tr) tr[kTrSelectDone] = (long long)wall_clock64();
        grid_barrier(a.bar, G, epoch, a.err, kErrTimeout, kSpinLimit);
        if (tr0 && tr) {
            tr[kTrSelected] = (long long)wall_clock64();
            tr[kTrGroup] = total;
        }

        const unsigned wp = wave_par(wave);
        const int na = __hip_atomic_load(&a.acnt[wp], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const long long m0 = (long long)wall_clock64();
        // many small targets: one wave each; few: the workgroups share them
        // (a single wave is slower per merge, so it pays only when the waves
        // of the grid all have several targets)
        const bool by_wave = kWaveMerges && a.wcap > 0 && na >= a.wmin;
        if (by_wave) {
            // small fronts: each wave takes targets itself and merges them in
            // its LDS slice; fronts that outgrow it join the large list
            WaveLds W;
            carve_wave(lds, a, W);
            for (;;) {
                int k = 0;
                if (lane_id() == 0) k = atomicAdd(&a.mcur[wp], 1);
                k = __shfl(k, 0, 64);
                if (k >= na) break;
                const int x = a.alist[k];
                if ((unsigned)x >= (unsigned)a.n) {
                    if (lane_id() == 0) atomicOr(a.err, kErrTarget);
                } else if (wave_merge_node<kObj>(a, x, wave, W, wv_cand)) {
                    ++wv_merges;
                } else if (lane_id() == 0) {
                    const int kb = atomicAdd(&a.acnt[2 + wp], 1);
                    a.alist[a.n + kb] = x;
                }
            }
            __syncthreads();  // the slices are the workgroup's LDS again
            grid_barrier(a.bar, G, epoch, a.err, kErrTimeout, kSpinLimit);
        }
        // merges by halves in this iteration: enough targets for two per workgroup
        const bool halves = kHalves && na >= a.halves_min;
        if constexpr (!kWaveMerges) {
            // weight classes: every target once, by the children queued to it
            // (final after the select barrier; cleared here for the next
            // iteration), appended to its class region (one reservation per
            // class present in a wave)
            const int l = lane_id();
            for (int k0 = b * (int)blockDim.x; k0 < na; k0 += (int)(G * blockDim.x)) {
                const int k = k0 + threadIdx.x;
                int c = -1, x = 0;
                if (k < na) {
                    x = a.alist[k];
                    if ((unsigned)x < (unsigned)a.n) {
                        const int wx = a.wt[x];
                        c = weight_class(wx);
                        // with merges by halves: large fronts and very many
                        // children go to the whole workgroup's regions, the
                        // heaviest to the first
                        if (halves) {
                            const int fz = a.nb[x].z;
                            if (wx > 4 * a.big_children || fz > a.capBh) c = kWeightClasses;
                            else if (wx > a.big_children || fz > a.big_front) c = kWeightClasses + 1;
                        }
                        a.wt[x] = 0;
                    } else {
                        atomicOr(a.err, kErrTarget);
                    }
                }
                uint64_t todo = ballot64(c >= 0);
                while (todo) {
                    const int lead = (int)__ffsll((unsigned long long)todo) - 1;
                    const int cl = __shfl(c, lead, 64);
                    const uint64_t same = ballot64(c == cl);
                    int base = 0;
                    if (l == lead) base = atomicAdd(&a.acnt[2 * (1 + cl) + wp], (int)__popcll(same));
                    base = __shfl(base, lead, 64);
                    if (c == cl) a.alist[(1 + cl) * a.n + base + lanes_below(same)] = x;
                    todo &= ~same;
                }
            }
            grid_barrier(a.bar, G, epoch, a.err, kErrTimeout, kSpinLimit);
        }
        // one workgroup per target, taken dynamically (merges differ widely in
        // cost); the next one is claimed while the current one merges.  Wave
        // build: the large fronts (and the small ones when no wave took them);
        // workgroup-only build: the heaviest weight class first (with merges
        // by halves: the whole workgroup's region first, then the classes by
        // halves)
        int nbig = 0, nsmall = na;
        if constexpr (kWaveMerges) {
            nbig = __hip_atomic_load(&a.acnt[2 + wp], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (by_wave) nsmall = 0;
        }
        int *const cursor = &a.mcur[kWaveMerges ? 2 + wp : wp];
        // thread 0's walk over the class regions (claims only grow); with
        // merges by halves each half's first thread walks on its own
        int cls = kWeightClasses - 1, cbase = 0, ccnt = 0;
        if (!kWaveMerges && (threadIdx.x & (halves ? 511 : 1023)) == 0)
            ccnt = __hip_atomic_load(&a.acnt[2 * (1 + cls) + wp], __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
        // list index of the k-th claim, -1 when none is left
        auto locate = [&](int k) -> int {
            if constexpr (kWaveMerges) {
                return k;  // resolved below
            } else {
                if (k >= na) return -1;
                while (cls > 0 && k >= cbase + ccnt) {
                    cbase += ccnt;
                    --cls;
                    ccnt = __hip_atomic_load(&a.acnt[2 * (1 + cls) + wp], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
                }
                return k < cbase + ccnt ? (1 + cls) * a.n + (k - cbase) : -1;
            }
        };
        // Whole-workgroup merges come from one loop (one call site per
        // build): thread 0 claims and hands out the next target, or -2 (run
        // the merges by halves) or -1 (done).  With merges by halves: first
        // the whole workgroup's region, then the halves; a half that backs
        // out of a target (its front outgrew the half's stage) stops both
        // halves after their current merges, the whole workgroup merges the
        // target, and the halves go on.
        // the whole workgroup's regions rb (heavy) and rb + 1 as one list
        const int rb = 1 + kWeightClasses;
        const int nw0 = halves ? __hip_atomic_load(&a.acnt[2 * rb + wp], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT)
                               : 0;
        const int nwhole = halves ? nw0 + __hip_atomic_load(&a.acnt[2 * (rb + 1) + wp],
                                                            __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT)
                                  : 0;
        int *const wcur = &a.mcur[2 * rb + wp];
        // thread 0: 0 whole-workgroup region, 1 after the halves, 2 no halves
        int phase = halves ? 0 : 2;
        int next = -1;
        if (threadIdx.x == 0) next = phase == 0 ? atomicAdd(wcur, 1) : locate(atomicAdd(cursor, 1));
        // (the half and the wave index are uniform in a wave: read from the
        // first lane, so that the half's LDS views stay in scalar registers)
        // (merges by halves run in 1024-thread workgroups: halves of 512)
        const int h = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 9);
        if (threadIdx.x < 8) hctl[threadIdx.x] = threadIdx.x == 0 ? 0 : -1;
        __syncthreads();
        for (;;) {
            if (threadIdx.x == 0) {
                int cmd = -1;
                for (;;) {
                    int x = -1;
                    if (phase == 0) {
                        if (next >= nwhole) {
                            phase = 1;
                            cmd = -2;
                            break;
                        }
                        x = a.alist[(size_t)(next < nw0 ? rb : rb + 1) * a.n +
                                    (next < nw0 ? next : next - nw0)];
                        next = atomicAdd(wcur, 1);
                    } else if (phase == 1) {
                        if (hctl[1] >= 0) {
                            x = hctl[1];
                            hctl[1] = -1;
                        } else if (hctl[2] >= 0) {
                            x = hctl[2];
                            hctl[2] = -1;
                        } else if (hctl[0] != 0) {
                            hctl[0] = 0;
                            cmd = -2;
                            break;
                        } else {
                            break;  // done
                        }
                    } else {
                        const int idx = next;
                        if (kWaveMerges ? idx >= nsmall + nbig : idx < 0) break;
                        next = locate(atomicAdd(cursor, 1));
                        x = kWaveMerges ? (idx < nsmall ? a.alist[idx] : a.alist[a.n + (idx - nsmall)])
                                        : a.alist[idx];
                    }
                    if ((unsigned)x < (unsigned)a.n) {
                        cmd = x;
                        break;
                    }
                    atomicOr(a.err, kErrTarget);
                }
                hctl[5] = cmd;
            }
            __syncthreads();
            const int cmd = hctl[5];
            __syncthreads();
            if (cmd == -1) break;
            if (cmd >= 0) {
                MergeLds s;
                carve_lds(lds, a, s);
                Grp<false> gw = whole_group();
                // (the wave-first build and the halves builds for two or
                // either objective count keep the single-read survivor step:
                // the four-read one needs more registers than they leave)
                merge_node<!kWaveMerges && (!kHalves || kObj == 3), kObj>(a, cmd, wave, s, gw, st_cand);
                ++st_merges;
                continue;
            }
            // cmd == -2: the merges by halves, heaviest class first
            if constexpr (kHalves) {
                Grp<true> gh{(int)threadIdx.x & 511, 512,
                             __builtin_amdgcn_readfirstlane(((int)threadIdx.x >> 6) & 7), 8, hbar[h],
                             0, a.err, 0};
                MergeLds sh;
                carve_group(lds + (size_t)h * a.half_lds, a, sh, a.capBh, a.capCh, 512, false);
                if (threadIdx.x < 16) hbar[threadIdx.x >> 3][threadIdx.x & 7] = 0;
                __syncthreads();
                int hnext = -1;
                if (gh.tid == 0) {
                    hnext = hctl[3 + h] >= 0 ? hctl[3 + h] : locate(atomicAdd(cursor, 1));
                    hctl[3 + h] = -1;
                }
                for (;;) {
                    if (gh.tid == 0) {
                        if (__hip_atomic_load(&hctl[0], __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_WORKGROUP) != 0) {
                            hctl[3 + h] = hnext;  // claimed, not merged: carried over
                            hnext = -2;
                        }
                        if (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
                            kErrTimeout)
                            hnext = -1;  // a barrier wait gave up: the search ends with an error
                        sh.misc[2] = hnext;
                    }
                    gsync(gh);
                    const int idx = sh.misc[2];
                    gsync(gh);
                    if (idx < 0) break;
                    if (gh.tid == 0) hnext = locate(atomicAdd(cursor, 1));
                    const int x = a.alist[idx];
                    long long cand = 0;
                    if ((unsigned)x >= (unsigned)a.n) {
                        if (gh.tid == 0) atomicOr(a.err, kErrTarget);
                    } else if (merge_node<kObj == 3, kObj>(a, x, wave, sh, gh, cand)) {
                        if (gh.tid == 0) {
                            hstat[h][0] += 1;
                            hstat[h][1] += (unsigned long long)cand;
                        }
                    } else if (gh.tid == 0) {
                        hctl[1 + h] = x;
                        hstat[h][2] += 1;
                        __hip_atomic_store(&hctl[0], 1, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                }
                __syncthreads();
            }
        }
        if (threadIdx.x == 0 && tr) {
            const long long dm = (long long)wall_clock64() - m0;
            atomicMax((unsigned long long *)&tr[kTrMaxMerge], (unsigned long long)dm);
            atomicAdd((unsigned long long *)&tr[kTrSumMerge], (unsigned long long)dm);
        }
        grid_barrier(a.bar, G, epoch, a.err, kErrTimeout, kSpinLimit);
        if (tr0 && tr) {
            tr[kTrMerged] = (long long)wall_clock64();
            tr[kTrTargets] = na + nbig;
        }

        abase += total;
        ++wave;
        ++i_step;
    }
    if (lane_id() == 0) {
        const bool t0 = threadIdx.x == 0;
        atomicAdd((unsigned long long *)&a.out[kOutMerges],
                  (unsigned long long)(wv_merges + (t0 ? st_merges : 0)));
        atomicAdd((unsigned long long *)&a.out[kOutCandidates],
                  (unsigned long long)(wv_cand + (t0 ? st_cand : 0)));
    }
    if (kHalves && threadIdx.x < 2) {
        const unsigned long long *hs = hstat[threadIdx.x];
        if (hs[0] | hs[2]) {
            atomicAdd((unsigned long long *)&a.out[kOutMerges], hs[0]);
            atomicAdd((unsigned long long *)&a.out[kOutCandidates], hs[1]);
            atomicAdd((unsigned long long *)&a.out[kOutHalfMerges], hs[0]);
            atomicAdd((unsigned long long *)&a.out[kOutBackouts], hs[2]);
        }
    }
    if (threadIdx.x == 0) {
        if (b == 0) {
            a.out[kOutWaves] = wave;
            a.out[kOutLabels] = abase;
            a.out[kOutStatus] = status;
        }
    }
}

// The builds of the persistent search: with single-wave merges for
// iterations with many small targets (large batches); the workgroup path
// only; and the workgroup path with merges by halves (two targets at once per
// workgroup in iterations with enough of them); each for queries of two
// objectives, of three, or of either (decided per query).  Each build gets
// its own register allocation.
__global__ void __launch_bounds__(1024) k_search(SearchArgs a) { search_body<false, false, 0>(a); }
__global__ void __launch_bounds__(1024) k_search_o2(SearchArgs a) {
    search_body<false, false, 2>(a);
}
__global__ void __launch_bounds__(1024) k_search_o3(SearchArgs a) {
    search_body<false, false, 3>(a);
}
__global__ void __launch_bounds__(1024) k_search_halves(SearchArgs a) {
    search_body<false, true, 0>(a);
}
__global__ void __launch_bounds__(1024) k_search_halves_o2(SearchArgs a) {
    search_body<false, true, 2>(a);
}
__global__ void __launch_bounds__(1024) k_search_halves_o3(SearchArgs a) {
    search_body<false, true, 3>(a);
}
__global__ void __launch_bounds__(1024) k_search_wave(SearchArgs a) {
    search_body<true, false, 0>(a);
}
__global__ void __launch_bounds__(1024) k_search_wave_o2(SearchArgs a) {
    search_body<true, false, 2>(a);
}

__global__ void __launch_bounds__(256) k_count_front(SearchArgs a) {
    // front labels X = sum_v |P(v)| and useful relaxations R = sum_v |P(v)| outdeg(v)
    __shared__ long long red[16];
    long long s = 0, r = 0;
    int mx = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) {
        const long long k = a.nb[v].z;
        s += k;
        r += k * (a.optr[v + 1] - a.optr[v]);
        mx = max(mx, (int)k);
    }
    s = block_sum_ll(s, red);
    r = block_sum_ll(r, red);
    mx = wave_max_i(mx);
    if (threadIdx.x == 0) {
        atomicAdd((unsigned long long *)&a.out[kOutFront], (unsigned long long)s);
        atomicAdd((unsigned long long *)&a.out[kOutRelax], (unsigned long long)r);
    }
    if (lane_id() == 0)
        atomicMax((unsigned long long *)&a.out[kOutMaxFront], (unsigned long long)mx);
}

// Plans still open when the early stop ended a query's loop are part of
// P_candidates if their head is a goal node.  Each such plan gets an arena id
// after the expanded ones, in query, goal-list and bucket order (so ids are
// deterministic), and its meta word becomes that id; the plan stays in its
// bucket.  Two passes over the queries: count (and check the arena's room),
// then assign.
__global__ void __launch_bounds__(1024) k_close_stopped(SearchArgs a) {
    __shared__ int scan[16];
    const long long base = a.out[kOutLabels];
    long long total = 0;
    for (int pass = 0; pass < 2; ++pass) {
        long long carry = 0;
        for (int q0 = 0; q0 < a.nq; q0 += (int)blockDim.x) {
            const int q = q0 + (int)threadIdx.x;
            const bool stopped = q < a.nq && a.qstop[q] >= 0;
            int cnt = 0;
            if (stopped)
                for (int gi = a.qgoff[q]; gi < a.qgoff[q + 1]; ++gi) {
                    const int4 nbv = a.nb[a.goal_list[gi]];
                    for (int k = 0; k < nbv.z; ++k)
                        cnt += lab_open(a.pool[(size_t)(unsigned)nbv.x + k]) ? 1 : 0;
                }
            int tot;
            const int ex = block_excl_scan(cnt, scan, &tot);
            if (pass == 1 && cnt > 0) {
                long long id = base + carry + ex;
                for (int gi = a.qgoff[q]; gi < a.qgoff[q + 1]; ++gi) {
                    const int x = a.goal_list[gi];
                    const int4 nbv = a.nb[x];
                    for (int k = 0; k < nbv.z; ++k) {
                        const size_t slot = (size_t)(unsigned)nbv.x + k;
                        const float4 L = a.pool[slot];
                        if (!lab_open(L)) continue;
                        a.arena[id] = make_int2(x, lab_parent(L));
                        reinterpret_cast<int *>(&a.pool[slot])[3] = (int)id;
                        ++id;
                    }
                }
            }
            carry += tot;
        }
        if (pass == 0) {
            total = carry;
            if (base + total > a.arena_cap) {
                if (threadIdx.x == 0) {
                    a.out[kOutStatus] = kStatusArena;
                    a.out[kOutNeed] = total;
                }
                return;
            }
        }
    }
    if (threadIdx.x == 0) a.out[kOutClosed] = total;
}

// ----------------------------------------------------------- goal front (a7)
// P_candidates of Alg. 3 kept whole: per query, the weak-Pareto minimum of the
// labels of all its goal nodes, in lexicographic (c, d, m) order, built with
// the same sorted merge as the search (goal nodes in ascending order, so of
// equal vectors the one at the smallest goal node is kept).  One workgroup per
// query (looping if there are more queries than workgroups).
__global__ void __launch_bounds__(1024) k_goal_front(SearchArgs a, GoalArgs g) {
    extern __shared__ __align__(16) unsigned char lds[];
    if (*(volatile int *)g.overflow) return;  // regions did not fit (k_goal_bound)
    MergeLds s;
    carve_lds(lds, a, s);
    for (int q = blockIdx.x; q < g.nq; q += gridDim.x) {
        s.B = s.Bl;
        s.bdead = s.bdeadl;
        s.spilled = false;
        int nB = 0, glo = 0;
        for (int gi = g.qgoff[q]; gi < g.qgoff[q + 1]; ++gi) {
            const int4 nbv = a.nb[g.goal_list[gi]];
            for (int c0 = 0; c0 < nbv.z; c0 += a.capC) {
                const int nC = min(a.capC, nbv.z - c0);
                for (int i = threadIdx.x; i < nC; i += blockDim.x)
                    s.C[i] = a.pool[(size_t)(unsigned)nbv.x + c0 + i];
                if (threadIdx.x == 0) {
                    s.misc[6] = 0;  // merge_chunk's append counters start at zero
                    s.misc[7] = 0;
                }
                __syncthreads();
                Grp<false> gw = whole_group();
                merge_chunk<false>(s, gw, nB, nC, a.near_scan, a.qnobj[q] >= 3, glo, a.err, false);
            }
        }
        const long long o = g.lab_off[q];
        if (nB > g.lab_cap[q]) {
            if (threadIdx.x == 0) atomicOr(g.overflow, 1);
            nB = g.lab_cap[q];
        }
        for (int i = threadIdx.x; i < nB; i += blockDim.x) {
            const float4 L = s.B[i];
            g.out_lab[o + i] = L;
            g.out_node[o + i] = a.arena[__float_as_int(L.w)].x;
        }
        if (threadIdx.x == 0) g.out_count[q] = nB;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(1024) k_goal_bound(SearchArgs a, GoalArgs g, long long cap,
                                                    long long *total) {
    __shared__ long long wsum[16];
    const int l = lane_id(), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    long long carry = 0;
    for (int q0 = 0; q0 < g.nq; q0 += blockDim.x) {
        const int q = q0 + threadIdx.x;
        long long b = 0;
        if (q < g.nq)
            for (int gi = g.qgoff[q]; gi < g.qgoff[q + 1]; ++gi) b += a.nb[g.goal_list[gi]].z;
        const long long incl = wave_incl_scan_add(b);
        if (l == 63) wsum[w] = incl;
        __syncthreads();
        long long before = 0, all = 0;
        for (int i = 0; i < nw; ++i) {
            before += i < w ? wsum[i] : 0;
            all += wsum[i];
        }
        if (q < g.nq) {
            g.lab_off[q] = carry + before + incl - b;
            g.lab_cap[q] = (int)min(b, 0x7fffffffll);
        }
        carry += all;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *total = carry;
        if (carry > cap) atomicOr(g.overflow, 1);
    }
}

__global__ void __launch_bounds__(256) k_goal_pack(GoalArgs g, float4 *plab, int *pnode,
                                                   long long pcap) {
    __shared__ long long red[8];
    if (*(volatile int *)g.overflow) return;
    for (int q = blockIdx.x; q < g.nq; q += gridDim.x) {
        long long o = 0;
        for (int i = threadIdx.x; i < q; i += blockDim.x) o += g.out_count[i];
        o = block_sum_ll(o, red);
        const int k = g.out_count[q];
        if (o + k > pcap) {
            if (threadIdx.x == 0) atomicOr(g.overflow, 2);
            continue;
        }
        const long long src = g.lab_off[q];
        for (int i = threadIdx.x; i < k; i += blockDim.x) {
            plab[o + i] = g.out_lab[src + i];
            pnode[o + i] = g.out_node[src + i];
        }
    }
}

// Re-walk the plan of each label with the analytic per-edge drift (the check
// of a search run on the learned surrogate's drift): thread i follows the
// parent chain of label lab[i] back to its root, then folds cost, drift
// (bound on the pre-reset drift, relocalisation) and max drift forward.
// With sur (the searched values of the labels) the thread also decides the
// judge: feasible, and drift and max drift within tol of the analytic ones
// relative to max(analytic, 1e-3 beta), compared in float64 -> pass[i].
__global__ void __launch_bounds__(256) k_rescore(const int2 *arena, const int *optr,
                                                 const int *ocol, const float *ocost,
                                                 const float *odrift, const uint8_t *nflag,
                                                 const int *lab, const float *beta,
                                                 const int *nobj, int n, int *path, int maxlen,
                                                 float4 *out, int *err, const float4 *sur,
                                                 float tol, uint8_t *pass) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int *pth = path + (size_t)i * maxlen;
    int len = 0;
    int id = lab[i];
    while (id >= 0 && len < maxlen) {
        const int2 r = arena[id];
        pth[len++] = r.x;
        id = r.y;
    }
    if (id >= 0) {
        atomicOr(err, 1);
        out[i] = make_float4(MPAP_INF, MPAP_INF, MPAP_INF, 0.f);
        if (pass) pass[i] = 0;
        return;
    }
    float c = 0.f, d = 0.f, m = 0.f;
    bool ok = true;
    for (int k = len - 1; k > 0; --k) {
        const int u = pth[k], v = pth[k - 1];
        int lo = optr[u], hi = optr[u + 1];
        while (lo < hi) {  // targets of a row are sorted
            const int mid = (lo + hi) >> 1;
            if (ocol[mid] < v) lo = mid + 1; else hi = mid;
        }
        if (lo >= optr[u + 1] || ocol[lo] != v) {
            atomicOr(err, 2);
            ok = false;
            break;
        }
        c = c + ocost[lo];
        const float dpre = d + odrift[lo];
        ok = ok && (dpre <= beta[i]);
        d = (nflag[v] & 1u) ? 0.0f : dpre;
        m = (nobj[i] >= 3) ? fmaxf(m, dpre) : 0.0f;
    }
    out[i] = make_float4(c, d, m, ok ? 1.f : 0.f);
    if (pass) {
        const float4 s = sur[i];
        const double floor = 1e-3 * (double)beta[i];
        const double ed = fabs((double)s.y - (double)d) / fmax((double)d, floor);
        const double em = fabs((double)s.z - (double)m) / fmax((double)m, floor);
        pass[i] = (ok && ed <= (double)tol && em <= (double)tol) ? 1 : 0;
    }
}
