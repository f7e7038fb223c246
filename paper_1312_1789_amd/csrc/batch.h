// batch.h -- device-side plan and launch arguments of the batched form (many
// independent clusters in one step sequence).  Not part of the public C-ABI.
#pragma once

#include "internal.h"

namespace nb {

constexpr int kBatchITileMax = 256;   // largest i-tile: active rows per work item
constexpr int64_t kBatchMaxRows = int64_t(1) << 22;   // items aimed for in one step x i-tile, at most
constexpr int kBatchMaxPerWG = 32;     // most items aimed for per persistent workgroup
constexpr int kBatchSchedBlock = 1024;  // particles per scheduling block
constexpr int kXcds = 8;                // XCDs of the device: work queues of the persistent force kernel

// The work of the cluster of one rank (plan order) in a step, written by
// the plan for the persistent force kernel: one 64-byte load per work item.
struct BatchRank {
    int64_t i0, i1;   // its work items [i0, i1)
    int64_t base;     // first particle
    int64_t jc;       // j-range per split
    int64_t poff;     // offset of its split partials (doubles)
    int64_t aoff;     // offset of its active list
    int32_t nn, na;   // particles, active rows
    int32_t sp, c;    // j-splits, cluster index
};
static_assert(sizeof(BatchRank) == 64, "one 64-byte record per rank");

// Written by the plan kernel of every batched step and read by the kernels
// after it.  Arrays sized n_clusters + 1 (the last entry of a scanned array
// holds its total).
struct BatchPlan {
    int64_t t_end;              // clusters whose next time exceeds this do not step
    int64_t n_live;             // clusters that stepped in the last plan
    int64_t pad[6];
    int64_t *nact;              // [nc]   active particles per cluster
    int64_t *aoff;              // [nc+1] offsets of the clusters' active lists
    int64_t *ioff;              // [nc+1] first work item of each cluster rank
    int64_t *poff;              // [nc+1] offsets of the clusters' split partials (doubles)
    int64_t *jchunk;            // [nc]   j-range per split
    int32_t *split;             // [nc]   j-splits per cluster
    int64_t *tcur;              // [nc]   time of the cluster's last completed step
    BatchRank *rank;            // [nc]   work of each cluster rank
    // items taken from each XCD's eighth of the step's items (one 64-byte
    // line per counter); reset by the plan
    unsigned queue[kXcds * 16];
};

struct BatchCounters {
    int64_t steps;
    int64_t sum_n_act;
    int64_t interactions;
    unsigned long long underflow;
    unsigned long long nonfinite;
    int64_t pad[3];
};

// Everything a batched launch needs; all pointers are device addresses inside
// the batch workspace except the state, which the caller passes per call.
struct BatchLaunch {
    int nc;                     // clusters
    int nb;                     // scheduling blocks per cluster (largest cluster / 1024, rounded up)
    int nblk;                   // scheduling blocks of all clusters
    const int32_t *blk;         // [nblk][2] (cluster, block) of each
    int64_t n;                  // particles in all clusters
    const int64_t *off;         // [nc+1] cluster offsets
    const int32_t *ord;         // [nc]   clusters by decreasing size
    int32_t *cid;               // [n]    cluster of each particle
    int64_t *tnext;             // [nc]   next block time of each cluster
    int64_t *bmin;              // [nc][nb]
    int32_t *bcnt;              // [nc][nb]
    BatchPlan *plan;
    BatchCounters *ctr;
    int32_t *act;               // [n] concatenated active lists
    double *part;               // split partials
    double *force;              // [12][n] step forces by active row
    double eps2;
    int64_t n_hard;             // per cluster; every pair is unsoftened when eps2 == 0
    int force_grid;             // workgroups of the persistent force kernel
    int per_wg;                 // work items aimed for per persistent workgroup
    int k_items;                // items aimed for in one step: min(force_grid * per_wg, kBatchMaxRows / itile)
    int itile;                  // active rows per work item: 64 or 256
};

hipError_t batch_cid(const BatchLaunch &L, hipStream_t s);
hipError_t batch_schedule(const BatchLaunch &L, const nbody_state &st, int all_active, int order, hipStream_t s);
hipError_t batch_predict(const BatchLaunch &L, const nbody_state &st, int order, int precision, void *rec,
                         hipStream_t s);
// Reset the work queues (a second force pass on the same plan).
hipError_t batch_requeue(const BatchLaunch &L, hipStream_t s);
hipError_t batch_force(const BatchLaunch &L, int order, int precision, const void *rec, hipStream_t s);
hipError_t batch_reduce(const BatchLaunch &L, int order, double *o0, double *o1, double *o2, double *o3,
                        hipStream_t s);
hipError_t batch_correct(const BatchLaunch &L, const nbody_config &c, const nbody_state &st, hipStream_t s);
// Workgroups of the persistent force kernel (i-tile itile) that fit on the
// device at once.
int batch_force_resident(int order, int precision, int itile, int device);

}  // namespace nb
