// Kernels of the double-integrator roadmap (position and velocity in 3D):
// minimum-energy fixed-time steering costs, selection of each state's
// cheapest reachable targets, and the drift increment along each trajectory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

constexpr int kSteerThreads = 256;
constexpr int kSteerMaxWidth = 1024;  // candidates ranked per selection round
constexpr int kSteerMaxSteps = 255;   // check steps per trajectory (K + 1 <= 256 points)
constexpr int kSteerMaxOut = 64;      // out-degree limit
constexpr int kSteerMaxBoxes = 4096;

struct SteerArgs {
    int n;
    const float *pos;  // [n][3]
    const float *vel;  // [n][3]
    int nbox;
    const float *blo;  // [nbox][3]
    const float *bhi;
    int nblob;
    const float *mu;   // [nblob][3]
    const float *sig;
    const float *amp;
    float T;           // steering time
    int K;             // check steps (K + 1 points)
    int k_out;         // out-degree
};

// Per source u (one block each): the first k_out reachable targets in
// ascending (J, id) order -> nbr[u * k_out + i], ncost (J), ncnt[u].
// *err |= 1 when more than the ranking buffer's worth of candidates share one
// steering cost (the selection cannot order them).
__global__ void k_steer_select(SteerArgs a, int *nbr, float *ncost, int *ncnt, int *err);
// rows of the CSR, each sorted by target id
__global__ void k_steer_compact(int n, int k_out, const int *row_ptr, const int *nbr,
                                const float *ncost, const int *ncnt, int *col, float *cost);
// drift increment and polyline length of every edge (one wave per source row)
__global__ void k_traj_drift(SteerArgs a, const int *row_ptr, const int *col, float *drift,
                             float *elen);
// surrogate inputs of every edge along its trajectory, and the 8-point base
__global__ void k_traj_features(SteerArgs a, const int *row_ptr, const int *col,
                                const float *elen, uint16_t *X, float *base);
