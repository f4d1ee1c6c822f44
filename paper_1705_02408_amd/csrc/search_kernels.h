// Kernel argument blocks and launch-facing constants of the search kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// status / error bits written by the device
constexpr int kStatusOk = 0;
constexpr int kStatusError = 1;       // see the err word
constexpr int kStatusNoConverge = 2;  // wave cap reached
constexpr int kStatusArena = 3;       // arena or frontier capacity too small

constexpr int kErrBucket = 1;   // a front outgrew the LDS staging capacity
constexpr int kErrPool = 2;     // bucket pool exhausted
constexpr int kErrTimeout = 4;  // a grid or half-workgroup barrier wait exceeded its bound
constexpr int kErrTarget = 8;   // a queued merge target is not a node (internal error)

// Merge targets of a workgroup-only launch are ordered by expected work (the
// children queued to them): class 0 below kWeightClassBase children, class c
// from kWeightClassBase * 2^(c-1) on, the last class open-ended.  Heavier
// classes are merged first, so the longest merges of an iteration start early.
constexpr int kWeightClasses = 10;
constexpr int kWeightClassBase = 128;
// Target list regions of n entries each: all targets, one per weight class,
// and (with merges by halves) two of targets the whole workgroup merges: the
// heavy ones (first), then the rest.
constexpr int kListRegions = 3 + kWeightClasses;

// device output words
constexpr int kOutWaves = 0;
constexpr int kOutLabels = 1;
constexpr int kOutMerges = 2;
constexpr int kOutCandidates = 3;
constexpr int kOutStatus = 4;
constexpr int kOutFront = 5;
constexpr int kOutRelax = 6;
constexpr int kOutNeed = 7;  // group size that did not fit (arena / frontier)
constexpr int kOutMaxFront = 8;
constexpr int kOutClosed = 9;  // open goal plans given arena ids at an early stop
constexpr int kOutHalfMerges = 10;  // merges done by half workgroups
constexpr int kOutBackouts = 11;    // targets a half backed out of (merged again whole)
constexpr int kOutWords = 12;

// per-wave trace words (device clock ticks, 100 MHz wall clock)
constexpr int kTraceWords = 10;
constexpr int kTrStart = 0;      // start of the count phase
constexpr int kTrCounted = 1;    // after the count barrier
constexpr int kTrSelected = 2;   // after the select barrier
constexpr int kTrMerged = 3;     // after the merge barrier
constexpr int kTrGroup = 4;      // group size
constexpr int kTrTargets = 5;    // merge targets
constexpr int kTrMaxMerge = 6;   // longest per-block merge phase (ticks)
constexpr int kTrSumMerge = 7;   // sum over blocks of merge-phase ticks
constexpr int kTrCountDone = 8;  // block 0 finished its count work
constexpr int kTrSelectDone = 9; // block 0 finished its select work

struct SearchArgs {
    // graph (device)
    int n;
    const int *rptr;      // in-edge CSR row pointers [n+1]
    const int *rsrc;      // in-edge source node [E]
    const float *rcost;   // in-edge cost [E]
    const float *rdrift;  // in-edge drift increment [E]
    const int *optr;      // out-edge CSR row pointers [n+1]
    const int *ocol;      // out-edge target [E]
    const uint8_t *nflag; // bit 0: relocalise on arrival; bit 1: goal
    // queries: the roadmap is the disjoint union of nq query roadmaps, query q
    // owning nodes [qoff[q], qoff[q+1]); each has its own bound, objective
    // count, root and group-threshold step (query q's group of iteration i
    // holds its open labels of cost <= i * qdelta[q])
    int nq;
    const int *qoff;     // [nq+1]
    const float *qbeta;  // [nq]
    const int *qnobj;    // [nq]
    const int *qroot;    // [nq] global node id of x_init
    const int *qheur;    // [nq] 1: drift from the learned surrogate (sdrift)
    const float *sdrift; // surrogate drift, in-edge order (the roadmap is symmetric)
    int *qlast;          // [nq] last wave with a group label of the query
    const float *qdelta; // [nq] lambda * r_n of the query
    // the early stop of Alg. 3's loop condition (per query): the loop of a
    // query with qearly[q] = 1 ends before the first group that holds a plan
    // at one of its goal nodes (goal_list[qgoff[q] .. qgoff[q+1]))
    const int *qgoff;      // [nq+1]
    const int *goal_list;  // goal nodes, global ids, query by query
    const int *qearly;     // [nq] 1: early stop, 0: until the query's P_open is empty
    int *qstop;            // [nq] -2: no early stop; -1: running; >= 0: stopped after
                           // that many expanded groups
    int early_any;         // some query has qearly = 1
    int max_waves;
    int near_scan;       // bucket labels tested per candidate before the full scan
    int capB;  // LDS staging capacity of a front (labels)
    int capC;  // candidate chunk (labels), multiple of the block size
    int nblocks;
    // state
    float4 *pool;
    unsigned long long pool_cap;
    unsigned *pool_top;
    int4 *nb;          // per node {pool offset, capacity, count, 0}
    float *minopen;    // per node least cost of an open label (+inf: none)
    int *gcnt;         // per node group size of the current iteration
    int4 *fo;          // per node {frontier offset, count, wave, first open label index}
    int *mark;         // per node last wave it was queued as merge target (wave build)
    int *wt;           // per node children queued to it this iteration (workgroup-only
                       // build; zero between iterations)
    int *alist;        // merge targets of the current wave, kListRegions regions of n:
                       // wave build: fronts of at most wcap labels in region 0 (merged
                       // by one wave), larger ones in region 1; workgroup-only build:
                       // every target in region 0, then by weight class c in region 1+c,
                       // with merges by halves the whole workgroup's in regions
                       // 1+kWeightClasses (heavy) and 2+kWeightClasses
    int *acnt;         // [2 kListRegions] target count of region r at [2 r + wave parity]
    int *mcur;         // [2 kListRegions] next target to merge, same layout
    int wcap;          // largest front merged by a single wave (0: none)
    int wmin;          // single-wave merges in iterations with at least wmin small targets
    int wslice;        // LDS bytes of one wave's slice in single-wave merges
    // merges by halves (workgroup-only build, 1024-thread workgroups): each
    // half of a workgroup merges its own targets in its half of the LDS
    // (half_lds bytes from the start of the dynamic LDS, a front stage of
    // capBh labels and a chunk of capCh); targets with fronts above
    // big_front labels or more than big_children children queued go to the
    // whole workgroup first, those above capBh labels or 4 big_children
    // children before the others
    int halves;        // 1: merges by halves (the k_search_halves build)
    int capBh, capCh, half_lds;
    int big_front, big_children;
    int halves_min;    // least merge targets of an iteration that merges by halves
    float4 *F;         // frontier labels of the current wave
    long long F_cap;
    int2 *arena;       // per expanded label {node, parent id}
    long long arena_cap;
    long long arena_base;  // ids already in the arena when the launch starts (a re-search
                           // that continues from an earlier result's labels); 0 otherwise
    long long *part_cnt;   // [2][nblocks]
    long long *part_open;  // [2][nblocks]
    long long *part_step;  // [2][nblocks] least iteration index with a non-empty group
    unsigned *bar;
    int *err;
    long long *out;    // [kOutWords]
    float4 *spill;        // per-block spill space for fronts beyond capB [nblocks][2][capG]
    uint8_t *spill_flags; // [nblocks][capG]
    int capG;
    long long *wstat;  // per-wave trace [wstat_cap][kTraceWords] (block-0 clock)
    int wstat_cap;
};

// Goal fronts of all queries: query q's goal nodes are
// goal_list[qgoff[q] .. qgoff[q+1]); its front goes to out_lab[lab_off[q] ..)
// (room for lab_cap[q] labels) with the goal node of each label.
struct GoalArgs {
    int nq;
    const int *qgoff;      // [nq+1]
    const int *goal_list;
    long long *lab_off;    // [nq] region of query q in out_lab/out_node
    int *lab_cap;          // [nq] its size
    float4 *out_lab;
    int *out_node;
    int *out_count;        // [nq]
    int *overflow;
};

__global__ void k_search_init(SearchArgs a);
// analytic re-walk of labels' plans (surrogate check): out = {c, d, m, feasible};
// with sur (nullable) also the judge's per-label decision pass[i]
__global__ void k_rescore(const int2 *arena, const int *optr, const int *ocol,
                          const float *ocost, const float *odrift, const uint8_t *nflag,
                          const int *lab, const float *beta, const int *nobj, int n, int *path,
                          int maxlen, float4 *out, int *err, const float4 *sur, float tol,
                          uint8_t *pass);
__global__ void k_search_roots(SearchArgs a);
// builds of the persistent search (_o2 / _o3: every query has two / three
// objectives; without: decided per query)
__global__ void k_search(SearchArgs a);
__global__ void k_search_o2(SearchArgs a);
__global__ void k_search_o3(SearchArgs a);
__global__ void k_search_halves(SearchArgs a);  // with merges by halves
__global__ void k_search_halves_o2(SearchArgs a);
__global__ void k_search_halves_o3(SearchArgs a);
__global__ void k_search_wave(SearchArgs a);  // with single-wave merges
__global__ void k_search_wave_o2(SearchArgs a);
__global__ void k_count_front(SearchArgs a);
// After a search with early stops: the plans still open at the goal nodes of
// every stopped query get arena ids (after the expanded ones) so that goal
// fronts name walkable witnesses.  One workgroup of 1024 threads.
__global__ void k_close_stopped(SearchArgs a);
__global__ void k_goal_front(SearchArgs a, GoalArgs g);
// per-query goal-front regions: lab_cap[q] = sum of the front sizes of the
// query's goal nodes (a bound on its goal front), lab_off = exclusive scan;
// *total = the sum; overflow |= 1 when it exceeds cap (then k_goal_front does
// nothing).  One block.
__global__ void k_goal_bound(SearchArgs a, GoalArgs g, long long cap, long long *total);
// goal fronts packed densely in query order: query q's out_count[q] labels go
// to plab/pnode at sum_{j<q} out_count[j]; overflow |= 2 beyond pcap
__global__ void k_goal_pack(GoalArgs g, float4 *plab, int *pnode, long long pcap);
