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
constexpr int kErrTimeout = 4;  // grid barrier wait exceeded its bound

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
constexpr int kOutWords = 10;

// per-wave trace words (device clock ticks, 100 MHz wall clock)
constexpr int kTraceWords = 8;
constexpr int kTrStart = 0;      // start of the count phase
constexpr int kTrCounted = 1;    // after the count barrier
constexpr int kTrSelected = 2;   // after the select barrier
constexpr int kTrMerged = 3;     // after the merge barrier
constexpr int kTrGroup = 4;      // group size
constexpr int kTrTargets = 5;    // merge targets
constexpr int kTrMaxMerge = 6;   // longest per-block merge phase (ticks)
constexpr int kTrSumMerge = 7;   // sum over blocks of merge-phase ticks

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
    // parameters
    float beta;
    float delta;  // lambda * r_n
    int nobj;
    int root;
    int max_waves;
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
    int4 *fo;          // per node {frontier offset, count, wave, 0}
    int *mark;         // per node last wave it was queued as merge target
    int *alist;        // merge targets of the current wave [n]
    int *acnt;         // [2] target counts by wave parity
    int *mcur;         // [2] next target to merge, by wave parity
    float4 *F;         // frontier labels of the current wave
    long long F_cap;
    int2 *arena;       // per expanded label {node, parent id}
    long long arena_cap;
    long long *part_cnt;   // [2][nblocks]
    long long *part_open;  // [2][nblocks]
    float *part_min;       // [2][nblocks]
    unsigned *bar;
    int *err;
    long long *out;    // [kOutWords]
    long long *wstat;  // per-wave trace [wstat_cap][kTraceWords] (block-0 clock)
    int wstat_cap;
};

struct GoalArgs {
    int n_goal;
    const int *goal_list;
    const int4 *nb;
    const float4 *pool;
    float4 *lab;       // gathered goal labels [cap]
    int *lab_node;     // [cap]
    uint8_t *dead;     // [cap]
    int cap;
    int *n_lab;
    float4 *out_lab;   // goal front, lexicographic order [cap]
    int *out_node;     // [cap]
    int *out_count;
};

__global__ void k_search_init(SearchArgs a);
__global__ void k_search(SearchArgs a);
__global__ void k_count_front(SearchArgs a);
__global__ void k_goal_gather(GoalArgs g);
__global__ void k_goal_dominance(GoalArgs g);
__global__ void k_goal_emit(GoalArgs g);
