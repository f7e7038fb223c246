// batch.hip -- many independent clusters advanced together: every call of a
// batched step gives each cluster one block step of its own (its own t_next
// and active set), with a fixed sequence of launches whose grids do not
// depend on the data, so one step can be captured in a HIP graph and
// replayed without the host.
//
// Sequence of one batched step:
//   k_b_min / k_b_count  per (cluster, 1024-particle block): next-time minima,
//                        the cluster's t_next, active counts;
//   k_b_plan             one block: active offsets, j-splits and work items
//                        per cluster (largest clusters first), counters, and
//                        the reset of the work queues;
//   k_b_compact          ordered active lists;
//   k_b_predict          every particle to its cluster's t_next;
//   k_b_force            persistent: workgroups take (cluster, i-tile, j-split)
//                        items from per-XCD queues until all are empty;
//   k_b_reduce           split partials summed in split order;
//   k_b_correct          corrector, interpolation and new steps.
// Method as in the single-system kernels (paper: Abstract; Sec. "Codes
// description"): Hermite block steps of order 4, 6 or 8 and direct-summation
// softened gravity with its derivatives (Nitadori & Makino 2008).
#include <climits>

#include "batch.h"
#include "hermite.h"
#include "pairwise.h"

namespace nb {
namespace {

constexpr int kBBlock = kBatchSchedBlock;
constexpr int kBTile = 32;   // records per LDS tile of the one-wave force workgroups
constexpr int kBThreads = 256;  // threads per scheduling block (4 particles each)

__device__ __forceinline__ int64_t b_next(const int64_t *t_tick, const int32_t *level, int64_t i)
{
    return t_tick[i] + (int64_t(1) << (kLevelMax - level[i]));
}

// Block b of cluster c covers [off[c] + b*kBBlock, min(off[c] + (b+1)*kBBlock, off[c+1])); the
// launch has one workgroup per such block, (c, b) = blk[2x], blk[2x + 1].
// Also clears the cluster's active count, which k_b_count accumulates.
__global__ void __launch_bounds__(kBThreads)
k_b_min(const int64_t *__restrict__ off, const int64_t *__restrict__ t_tick, const int32_t *__restrict__ level,
        int nb, const int32_t *__restrict__ blk, int64_t *__restrict__ bmin, BatchPlan *__restrict__ pl)
{
    __shared__ int64_t sm[kBThreads];
    const int c = blk[2 * blockIdx.x], b = blk[2 * blockIdx.x + 1];
    if (b == 0 && threadIdx.x == 0) pl->nact[c] = 0;
    const int64_t lo = off[c] + int64_t(b) * kBBlock, hi = off[c + 1];
    int64_t mn = INT64_MAX;
    for (int k = 0; k < kBBlock / kBThreads; ++k) {
        const int64_t i = lo + int64_t(k) * kBThreads + threadIdx.x;
        if (i < hi && i < lo + kBBlock) {
            const int64_t t = b_next(t_tick, level, i);
            mn = t < mn ? t : mn;
        }
    }
    sm[threadIdx.x] = mn;
    __syncthreads();
    for (int s = kBThreads / 2; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s && sm[threadIdx.x + s] < sm[threadIdx.x]) sm[threadIdx.x] = sm[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) bmin[int64_t(c) * nb + b] = sm[0];
}

// Cluster minimum (from the block minima), then this block's active count,
// also added into the cluster's count (integer atomics: the total does not
// depend on their order).  all_active != 0 marks every particle active
// (initialisation).
__global__ void __launch_bounds__(kBThreads)
k_b_count(const int64_t *__restrict__ off, const int64_t *__restrict__ t_tick, const int32_t *__restrict__ level,
          int nb, const int32_t *__restrict__ blk, const int64_t *__restrict__ bmin, int all_active,
          BatchPlan *__restrict__ pl, int64_t *__restrict__ tnext, int32_t *__restrict__ bcnt)
{
    __shared__ int64_t sm[kBThreads];
    __shared__ int cnt[kBThreads];
    const int c = blk[2 * blockIdx.x], b = blk[2 * blockIdx.x + 1];
    const int nbc = int((off[c + 1] - off[c] + kBBlock - 1) / kBBlock);   // the cluster's blocks
    int64_t mn = INT64_MAX;
    for (int k = threadIdx.x; k < nbc; k += kBThreads) {
        const int64_t v = bmin[int64_t(c) * nb + k];
        mn = v < mn ? v : mn;
    }
    sm[threadIdx.x] = mn;
    __syncthreads();
    for (int s = kBThreads / 2; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s && sm[threadIdx.x + s] < sm[threadIdx.x]) sm[threadIdx.x] = sm[threadIdx.x + s];
        __syncthreads();
    }
    // initialisation: every particle at t = 0; otherwise clusters past t_end rest
    const int64_t tn = all_active ? 0 : sm[0];
    const bool live = all_active || tn <= pl->t_end;
    const int64_t lo = off[c] + int64_t(b) * kBBlock, hi = off[c + 1];
    int k0 = 0;
    for (int k = 0; k < kBBlock / kBThreads; ++k) {
        const int64_t i = lo + int64_t(k) * kBThreads + threadIdx.x;
        if (live && i < hi && i < lo + kBBlock && (all_active || b_next(t_tick, level, i) == tn)) ++k0;
    }
    cnt[threadIdx.x] = k0;
    __syncthreads();
    for (int s = kBThreads / 2; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s) cnt[threadIdx.x] += cnt[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        bcnt[int64_t(c) * nb + b] = cnt[0];
        if (cnt[0] > 0) atomicAdd(reinterpret_cast<unsigned long long *>(&pl->nact[c]), (unsigned long long)cnt[0]);
        if (b == 0) tnext[c] = tn;
    }
}

// Exclusive scan of v[0..n) in one block (chunks of kBThreads, running carry).
__device__ void block_scan(int64_t *v, int n, int64_t *sh)
{
    int64_t carry = 0;
    for (int c0 = 0; c0 < n; c0 += kBThreads) {
        const int c = c0 + threadIdx.x;
        const int64_t x = c < n ? v[c] : 0;
        sh[threadIdx.x] = x;
        __syncthreads();
        for (int o = 1; o < kBThreads; o <<= 1) {
            const int64_t add = int(threadIdx.x) >= o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += add;
            __syncthreads();
        }
        if (c < n) v[c] = carry + sh[threadIdx.x] - x;
        carry += sh[kBThreads - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) v[n] = carry;
    __syncthreads();
}

// Sum over the block of one value per thread (the result is returned to
// every thread).
__device__ int64_t block_sum(int64_t v, int64_t *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int st = kBThreads / 2; st > 0; st >>= 1) {
        if (int(threadIdx.x) < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    const int64_t r = sh[0];
    __syncthreads();
    return r;
}

// The plan of one batched step (one block).  For every cluster: active
// offset, j-splits and work items.  Items are sized by cost: the step's
// padded work W = sum_c tiles_c * itile * N_c is cut into about k_items items
// of W / k_items pair evaluations each (a cluster's j-range is split into s_c
// pieces of at least 128), so no item is much longer than the average and the
// persistent kernel ends evenly.  Items are numbered in the cluster order
// ord[] (largest clusters first).  Bound used for the partial buffer:
// s_c <= itile N_c k_items / W + 1, so sum_c s_c a_c <= itile k_items + n.
// Also resets the work queues and adds the step's interactions to the counters.
__global__ void __launch_bounds__(kBThreads)
k_b_plan(int nc, const int64_t *__restrict__ off, const int32_t *__restrict__ ord, const int64_t *__restrict__ tnext,
         BatchPlan *__restrict__ pl, int ncomp, int k_items, int itile, BatchCounters *__restrict__ ctr)
{
    __shared__ int64_t sh[kBThreads];
    int64_t w = 0, inter = 0, live = 0;
    for (int c = threadIdx.x; c < nc; c += kBThreads) {
        const int64_t a = pl->nact[c], nn = off[c + 1] - off[c];
        pl->aoff[c] = a;
        if (a > 0) pl->tcur[c] = tnext[c];
        w += (a + itile - 1) / itile * itile * nn;
        inter += a * nn;
        live += a > 0 ? 1 : 0;
    }
    const int64_t W = block_sum(w, sh);
    inter = block_sum(inter, sh);
    live = block_sum(live, sh);
    const int64_t w_item = W / k_items + 1;
    block_scan(pl->aoff, nc, sh);
    // splits, items (in rank order), partial rows (in cluster order)
    for (int r = threadIdx.x; r < nc; r += kBThreads) {
        const int c = ord[r];
        const int64_t na = pl->nact[c], nn = off[c + 1] - off[c];
        const int64_t tiles = (na + itile - 1) / itile;
        int64_t sp = (int64_t(itile) * nn + w_item - 1) / w_item;
        const int64_t sp_max = nn / kMixedChunk > 1 ? nn / kMixedChunk : 1;   // pieces of at least one FP32 chunk
        sp = sp < 1 ? 1 : (sp > sp_max ? sp_max : sp);
        int64_t jc = (nn + sp - 1) / sp;
        jc = (jc + kMixedChunk - 1) / kMixedChunk * kMixedChunk;
        sp = (nn + jc - 1) / jc;
        pl->split[c] = int32_t(sp);
        pl->jchunk[c] = jc;
        pl->ioff[r] = tiles * sp;
        pl->poff[c] = sp * na * ncomp;
    }
    __syncthreads();
    block_scan(pl->ioff, nc, sh);
    block_scan(pl->poff, nc, sh);
    for (int r = threadIdx.x; r < nc; r += kBThreads) {
        const int c = ord[r];
        BatchRank d;
        d.i0 = pl->ioff[r];
        d.i1 = pl->ioff[r + 1];
        d.base = off[c];
        d.jc = pl->jchunk[c];
        d.poff = pl->poff[c];
        d.aoff = pl->aoff[c];
        d.nn = int32_t(off[c + 1] - off[c]);
        d.na = int32_t(pl->nact[c]);
        d.sp = pl->split[c];
        d.c = c;
        pl->rank[r] = d;
    }
    if (threadIdx.x < kXcds) pl->queue[threadIdx.x * 16] = 0u;
    if (threadIdx.x == 0) {
        pl->n_live = live;
        ctr->interactions += inter;
        ctr->sum_n_act += pl->aoff[nc];
        ctr->steps += 1;
    }
}

// Ordered active lists: block (b, c) writes its actives after those of the
// cluster's earlier blocks, at aoff[c] + sum of bcnt[c][0 .. b).
__global__ void __launch_bounds__(kBThreads)
k_b_compact(const int64_t *__restrict__ off, const int64_t *__restrict__ t_tick, const int32_t *__restrict__ level,
            int nb, const int32_t *__restrict__ blk, const int64_t *__restrict__ tnext,
            const int32_t *__restrict__ bcnt, int all_active, const BatchPlan *__restrict__ pl,
            int32_t *__restrict__ act)
{
    __shared__ int s[kBThreads];
    __shared__ int64_t sb[kBThreads];
    constexpr int PER = kBBlock / kBThreads;
    const int c = blk[2 * blockIdx.x], b = blk[2 * blockIdx.x + 1];
    int64_t before = 0;
    for (int k = threadIdx.x; k < b; k += kBThreads) before += bcnt[int64_t(c) * nb + k];
    const int64_t block_off = pl->aoff[c] + block_sum(before, sb);
    const int64_t lo = off[c] + int64_t(b) * kBBlock, hi = off[c + 1];
    const int64_t tn = tnext[c];
    const bool live = pl->nact[c] > 0;
    const int64_t base = lo + int64_t(threadIdx.x) * PER;
    int flags[PER];
    int k0 = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int64_t i = base + k;
        flags[k] = (live && i < hi && (all_active || b_next(t_tick, level, i) == tn)) ? 1 : 0;
        k0 += flags[k];
    }
    s[threadIdx.x] = k0;
    __syncthreads();
    for (int o = 1; o < kBThreads; o <<= 1) {
        const int add = int(threadIdx.x) >= o ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    int64_t pos = block_off + s[threadIdx.x] - k0;
#pragma unroll
    for (int k = 0; k < PER; ++k)
        if (flags[k]) act[pos++] = int32_t(base + k);
}

__device__ __forceinline__ int find_cluster(const int64_t *__restrict__ off, int nc, int64_t i)
{
    int lo = 0, hi = nc;   // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void __launch_bounds__(256)
k_b_cid(const int64_t *__restrict__ off, int nc, int64_t n, int32_t *__restrict__ cid)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) cid[i] = find_cluster(off, nc, i);
}

template <int P, int PREC>
__global__ void __launch_bounds__(256)
k_b_predict(int64_t n, const int32_t *__restrict__ cid, const int64_t *__restrict__ tnext,
            const BatchPlan *__restrict__ pl,
            const double *__restrict__ m, const double *__restrict__ x, const double *__restrict__ v,
            const double *__restrict__ d0, const double *__restrict__ d1, const double *__restrict__ d2,
            const double *__restrict__ d3, const double *__restrict__ d4, const double *__restrict__ d5,
            const int64_t *__restrict__ t_tick, void *__restrict__ rec_out)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = cid[i];
    if (pl->nact[c] == 0) return;   // resting cluster: its records are not read
    const double dt = double(tnext[c] - t_tick[i]) * (1.0 / double(kTicksPerUnit));
    const double *ds[6] = {d0, d1, d2, d3, d4, d5};
    predict_one<P, PREC>(n, i, dt, m, x, v, ds, rec_out);
}

// One work item of a 64-lane workgroup: the rows of one i-tile against the
// j-range [j0, j1) of its cluster (cluster particles [base, base + nn), the
// first nh unsoftened).  The 64 lanes form R = 64 / JS groups of JS
// consecutive lanes; group r holds the tile's rows r and r + R (two rows per
// lane, so one record read from LDS serves two rows) and lane sl of the group
// takes j0 + sl, j0 + sl + JS, ... .  The JS lanes' sums are folded with a
// fixed butterfly and lane sl = 0 stores the group's rows.  A tile of `rows`
// active rows takes the largest JS (at most 64 and the tile length) with
// 2R >= rows, so a cluster's last, partly filled tile leaves at most half of
// its lanes idle (b_item_rows).
template <class Pol, int P, int JS, int TILE>
__device__ __forceinline__ void b_item(const typename Pol::Rec *__restrict__ rec, const int32_t *__restrict__ al,
                                       int64_t na, int64_t row0, int64_t base, int64_t nn, int64_t nh, int64_t j0,
                                       int64_t j1, typename Pol::ET e2, typename Pol::Rec (*tile)[TILE],
                                       double *__restrict__ dst)
{
    using Rec = typename Pol::Rec;
    using Part = typename Pol::Part;
    using ET = typename Pol::ET;
    static_assert(!Pol::kWithPot, "the batched force sums no potential");
    static_assert(TILE % JS == 0, "tile shape");
    constexpr int R = 64 / JS;
    constexpr int NV = 3 * (P / 2);
    constexpr int PIECES = int(sizeof(Rec) / 16);       // 16-byte pieces per record
    constexpr int PER_T = (TILE * PIECES + 63) / 64;     // pieces each lane moves per tile
    typedef uint4 __attribute__((may_alias)) piece_t;
    const int lane = int(threadIdx.x);
    const int r = lane / JS, sl = lane % JS;
    typename Pol::I ip[2];
    int64_t iidx[2];
    double acc[2][NV];
    Part pt[2][13];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int64_t q0 = row0 + r + k * R;
        const int64_t q = q0 < na ? q0 : na - 1;   // padding rows recompute the last row; never stored
        const int64_t ia = al[q];
        iidx[k] = (ia >= base && ia < base + nn) ? ia : base;
        ip[k] = Pol::load(rec[iidx[k]]);
#pragma unroll
        for (int c = 0; c < NV; ++c) acc[k][c] = 0.0;
    }
    // unsoftened pairs among the cluster's first nh particles: this lane's j
    // of [j0, min(j1, base + nh)), each added into FP64 on its own
    const int64_t jh1 = j1 < base + nh ? j1 : base + nh;
    for (int64_t j = j0 + sl; j < jh1; j += JS) {
        const Rec rj = rec[j];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            Part ph[13];
#pragma unroll
            for (int c = 0; c < 13; ++c) zero_part(ph[c]);
            const ET el = (iidx[k] - base < nh) ? ET(0) : e2;
            Pol::template pair<true>(ip[k], rj, el, j != iidx[k], ph);
#pragma unroll
            for (int c = 0; c < NV; ++c) acc[k][c] += to_double(ph[c]);
        }
    }
    // the softened rest through double-buffered LDS tiles; slots of the last
    // tile past j1 hold zero records (mass 0), which add exact zeros, as does
    // the row's own particle (zero separation, softened r^2 > 0)
    const int64_t js0 = j0 > base + nh ? j0 : base + nh;
    piece_t pre[PER_T];
    auto fetch = [&](int64_t jt) {
        const piece_t *src = reinterpret_cast<const piece_t *>(rec + jt);
        const int64_t avail = (j1 - jt) * PIECES;
#pragma unroll
        for (int k = 0; k < PER_T; ++k) {
            const int pc = lane + k * 64;
            if (pc < avail && pc < TILE * PIECES) pre[k] = src[pc];
            else pre[k] = piece_t{0u, 0u, 0u, 0u};
        }
    };
    if (js0 < j1) fetch(js0);
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int c = 0; c < 13; ++c) zero_part(pt[k][c]);
    // every tile is taken whole (IT records per lane): the slots of the last
    // tile past j1 hold zero records.  The FP32 sums are added into FP64
    // every kChunk / TILE tiles (kChunk consecutive j of the range).
    constexpr int IT = TILE / JS;
    constexpr int FL = Pol::kChunk > 0 ? Pol::kChunk / TILE : (1 << 30);
    static_assert(Pol::kChunk % TILE == 0, "whole tiles per FP32 chunk");
    int since = 0;   // tiles since the last flush
    int buf = 0;
    for (int64_t jt = js0; jt < j1; jt += TILE) {
        piece_t *tw = reinterpret_cast<piece_t *>(tile[buf]);
#pragma unroll
        for (int k = 0; k < PER_T; ++k)
            if (lane + k * 64 < TILE * PIECES) tw[lane + k * 64] = pre[k];
        __syncthreads();   // tile ready; the other buffer is no longer read
        if (jt + TILE < j1) fetch(jt + TILE);
        const Rec *tr = tile[buf] + sl;
#pragma unroll 8
        for (int u = 0; u < IT; ++u) {
            const Rec rj = tr[u * JS];
#pragma unroll
            for (int k = 0; k < 2; ++k) Pol::template pair<false>(ip[k], rj, e2, true, pt[k]);
        }
        if (++since == FL) {
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int c = 0; c < NV; ++c) {
                    acc[k][c] += to_double(pt[k][c]);
                    zero_part(pt[k][c]);
                }
            since = 0;
        }
        buf ^= 1;
    }
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int c = 0; c < NV; ++c) acc[k][c] += to_double(pt[k][c]);
    // fold the group's JS lanes (consecutive lanes: xor offsets below JS stay in the group)
#pragma unroll
    for (int m = JS / 2; m > 0; m >>= 1)
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int c = 0; c < NV; ++c) acc[k][c] += __shfl_xor(acc[k][c], m, 64);
    if (sl == 0) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int64_t q0 = row0 + r + k * R;
            if (q0 < na)
#pragma unroll
                for (int c = 0; c < NV; ++c) dst[int64_t(c) * na + q0] = acc[k][c];
        }
    }
}

// b_item with the largest lane group JS (at most 64 and the tile length)
// whose 2 * 64 / JS rows hold the tile's `rows` active rows.
template <class Pol, int P, int TILE, int ROWS>
__device__ __forceinline__ void b_item_rows(int rows, const typename Pol::Rec *__restrict__ rec,
                                            const int32_t *__restrict__ al, int64_t na, int64_t row0, int64_t base,
                                            int64_t nn, int64_t nh, int64_t j0, int64_t j1, typename Pol::ET e2,
                                            typename Pol::Rec (*tile)[TILE], double *__restrict__ dst)
{
    constexpr int J2 = 2 < TILE ? 2 : TILE, J4 = 4 < TILE ? 4 : TILE, J8 = 8 < TILE ? 8 : TILE;
    constexpr int J16 = 16 < TILE ? 16 : TILE, J32 = 32 < TILE ? 32 : TILE, J64 = 64 < TILE ? 64 : TILE;
    if (ROWS == 128 && rows > 64) b_item<Pol, P, 1, TILE>(rec, al, na, row0, base, nn, nh, j0, j1, e2, tile, dst);
    else if (rows > 32) b_item<Pol, P, J2, TILE>(rec, al, na, row0, base, nn, nh, j0, j1, e2, tile, dst);
    else if (rows > 16) b_item<Pol, P, J4, TILE>(rec, al, na, row0, base, nn, nh, j0, j1, e2, tile, dst);
    else if (rows > 8) b_item<Pol, P, J8, TILE>(rec, al, na, row0, base, nn, nh, j0, j1, e2, tile, dst);
    else if (rows > 4) b_item<Pol, P, J16, TILE>(rec, al, na, row0, base, nn, nh, j0, j1, e2, tile, dst);
    else if (rows > 2) b_item<Pol, P, J32, TILE>(rec, al, na, row0, base, nn, nh, j0, j1, e2, tile, dst);
    else b_item<Pol, P, J64, TILE>(rec, al, na, row0, base, nn, nh, j0, j1, e2, tile, dst);
}

// Persistent force kernel.  The step's items (in cluster rank order: item
// = cluster ord[rank], i-tile, j-split) form 8 contiguous ranges, one per
// XCD, each with its own queue counter.  The dispatcher places workgroup g on
// XCD g mod 8: a workgroup takes items from its own XCD's range (a few
// clusters, whose j records that XCD's L2 then holds), then from the other
// ranges in turn, and leaves when all eight are empty.  Each counter is
// shared by an eighth of the workgroups only.  Every wave reaches the exit:
// the counters only grow.  Tiles of ROWS = 64 or 128 rows run as one wave
// with two rows per lane (b_item); 256-row tiles as four waves with one row
// per lane.

// Waves per SIMD the register allocation of k_b_force aims for: the
// one-wave workgroups of the FP32 pair arithmetic (MIXED) at orders 4 and 6
// fit 3 without spills (otherwise the compiler's own choice).
template <class Pol, int P, int BLOCK>
constexpr int b_waves() { return (BLOCK == 64 && sizeof(typename Pol::Part) == 4 && P <= 6) ? 3 : 1; }

// One work item: the i-tile and j-split `local` of the cluster described by d.
template <class Pol, int P, int BLOCK, int TILE, int ROWS>
__device__ __forceinline__ void b_run(const BatchRank &d, int64_t local, const typename Pol::Rec *__restrict__ rec,
                                      const int32_t *__restrict__ act, typename Pol::ET e2, int64_t n_hard, int ncomp,
                                      double *__restrict__ part, typename Pol::Rec (*tile)[TILE])
{
    const uint32_t lq = uint32_t(local), sp = uint32_t(d.sp);
    const int64_t tile_i = lq / sp, split = lq % sp;
    const int64_t na = d.na, base = d.base, nn = d.nn, jc = d.jc;
    const int64_t j0 = base + split * jc;
    const int64_t j1 = (split + 1) * jc < nn ? base + (split + 1) * jc : base + nn;
    const int64_t nh = n_hard < nn ? n_hard : nn;
    double *dst = part + d.poff + split * ncomp * na;
    const int32_t *al = act + d.aoff;
    if constexpr (BLOCK == 64) {
        const int64_t row0 = tile_i * ROWS;
        const int64_t rows = na - row0 < ROWS ? na - row0 : ROWS;
        b_item_rows<Pol, P, TILE, ROWS>(int(rows), rec, al, na, row0, base, nn, nh, j0, j1, e2, tile, dst);
    } else {
        // this lane's active row
        const int64_t q0 = tile_i * BLOCK + threadIdx.x;
        const int64_t q = q0 < na ? q0 : na - 1;
        typename Pol::I ip[1];
        int64_t iidx[1];
        double acc[1][13];
        const int64_t ia = al[q];
        iidx[0] = (ia >= base && ia < base + nn) ? ia : base;
        ip[0] = Pol::load(rec[iidx[0]]);
#pragma unroll
        for (int cc = 0; cc < 13; ++cc) acc[0][cc] = 0.0;
        hard_pairs<Pol, 1>(rec, j0, (j1 < base + nh) ? j1 : base + nh, base, nh, e2, ip, iidx, acc);
        const int64_t js0 = (j0 > base + nh) ? j0 : base + nh;
        lds_tiles<Pol, 1, BLOCK, 2, TILE>(rec, js0, j1, e2, ip, iidx, tile, acc);
        if (q0 < na) {
#pragma unroll
            for (int cc = 0; cc < 3 * (P / 2); ++cc) dst[int64_t(cc) * na + q0] = acc[0][cc];
        }
    }
}

__device__ __forceinline__ int64_t wave_uniform(uint32_t v) { return int64_t(uint32_t(__builtin_amdgcn_readfirstlane(v))); }

template <class Pol, int P, int BLOCK, int TILE, int ROWS>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(b_waves<Pol, P, BLOCK>())))
k_b_force(const typename Pol::Rec *__restrict__ rec, int nc, const int32_t *__restrict__ act,
          BatchPlan *__restrict__ pl, double eps2, int64_t n_hard, int ncomp, double *__restrict__ part)
{
    using Rec = typename Pol::Rec;
    using ET = typename Pol::ET;
    __shared__ Rec tile[2][TILE];
    __shared__ uint32_t s_take;
    const ET e2 = ET(eps2);
    const BatchRank *__restrict__ rk = pl->rank;
    const int64_t total = rk[nc - 1].i1;
    // a step with fewer items than workgroups: the first `total` workgroups
    // (spread over the XCDs) take them all, the others leave at once
    if (int64_t(blockIdx.x) >= total) return;
    const int x0 = int(blockIdx.x) % kXcds;
    const int64_t ahead = 2 * ((int64_t(gridDim.x) + kXcds - 1) / kXcds);   // two items per workgroup of an XCD
    for (int v = 0; v < kXcds; ++v) {
        const int xr = (x0 + v) % kXcds;
        const int64_t r0 = total * xr / kXcds, len = total * (xr + 1) / kXcds - r0;
        uint32_t *q = &pl->queue[xr * 16];
        // the first item of this range; an exhausted range is seen with a
        // load, without adding to its counter
        __syncthreads();   // the previous item's tiles and s_take are no longer read
        if (threadIdx.x == 0) {
            const uint32_t seen = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_take = seen >= uint32_t(len) ? uint32_t(len) : atomicAdd(q, 1u);
        }
        __syncthreads();
        int64_t take = wave_uniform(s_take);   // scalar: the cluster, ranges and loop bounds stay in SGPRs
        if (take >= len) continue;
        // rank of the item's cluster: rk[lo].i0 <= item < rk[lo].i1; the
        // items a workgroup takes from one range only increase
        int lo = 0;
        {
            int hi = nc;
            while (hi - lo > 1) {
                const int mid = (lo + hi) / 2;
                if (rk[mid].i0 <= r0 + take) lo = mid; else hi = mid;
            }
        }
        for (;;) {
            const int64_t item = r0 + take;
            while (rk[lo].i1 <= item) ++lo;
            const BatchRank d = rk[lo];
            // one wave, far from the range's end: the next item is claimed
            // now and its number read after this one, so the atomic's latency
            // is not waited for (near the end a claimed item would wait for
            // this one while other workgroups idle)
            const bool early = BLOCK == 64 && take + ahead < len;
            uint32_t nxt = 0u;
            if (early && threadIdx.x == 0) nxt = atomicAdd(q, 1u);
            b_run<Pol, P, BLOCK, TILE, ROWS>(d, item - d.i0, rec, act, e2, n_hard, ncomp, part, tile);
            if (early) {
                take = wave_uniform(nxt);
            } else {
                __syncthreads();   // the item's tiles and s_take are no longer read
                if (threadIdx.x == 0) s_take = atomicAdd(q, 1u);
                __syncthreads();
                take = wave_uniform(s_take);
            }
            if (take >= len) break;
        }
    }
}

// Row r of the concatenated active list: sum of its cluster's split partials
// into outputs [3][stride] (acc, jerk, snap, crackle).  A group of kRedLanes
// consecutive lanes owns a row (its cluster found through the row's particle):
// for every component, lane l adds splits l, l + kRedLanes, ... in order,
// then the group folds its sums with a fixed butterfly (the order depends
// only on the cluster's split count).
constexpr int kRedLanes = 16;

template <int P>
__global__ void __launch_bounds__(256)
k_b_reduce(int nc, int64_t n, const BatchPlan *__restrict__ pl, const int32_t *__restrict__ act,
           const int32_t *__restrict__ cid, int ncomp, const double *__restrict__ part, double *__restrict__ o0,
           double *__restrict__ o1, double *__restrict__ o2, double *__restrict__ o3, int64_t stride)
{
    constexpr int NV = 3 * (P / 2);
    const int64_t total = pl->aoff[nc];
    const int l = int(threadIdx.x) % kRedLanes;
    const int64_t groups = int64_t(gridDim.x) * blockDim.x / kRedLanes;
    double *outs[4] = {o0, o1, o2, o3};
    // the lanes of a group share r, so they run the same iterations and their
    // exchanges (within the group) always find their partners active
    for (int64_t r = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kRedLanes; r < total; r += groups) {
        const int64_t i = act[r];
        const int c = (i >= 0 && i < n) ? cid[i] : 0;
        const int64_t na = pl->nact[c], q = r - pl->aoff[c];
        if (q < 0 || q >= na) continue;   // never for a consistent plan; the whole group skips together
        const double *src = part + pl->poff[c];
        const int sp = pl->split[c];
        double s[NV];
#pragma unroll
        for (int cc = 0; cc < NV; ++cc) s[cc] = 0.0;
        for (int k = l; k < sp; k += kRedLanes)
#pragma unroll
            for (int cc = 0; cc < NV; ++cc) s[cc] += src[(int64_t(k) * ncomp + cc) * na + q];
#pragma unroll
        for (int m = kRedLanes / 2; m > 0; m >>= 1)
#pragma unroll
            for (int cc = 0; cc < NV; ++cc) s[cc] += __shfl_xor(s[cc], m, 64);
        // lane l of the group stores component l
#pragma unroll
        for (int cc = 0; cc < NV; ++cc) {
            double *o = outs[cc / 3];
            if (l == cc % kRedLanes && o) o[(cc % 3) * stride + r] = s[cc];
        }
    }
}

template <int P>
__global__ void __launch_bounds__(256)
k_b_correct(int64_t n, int nc, const int32_t *__restrict__ act, const int32_t *__restrict__ cid,
            const int64_t *__restrict__ tnext, const BatchPlan *__restrict__ pl, double *__restrict__ x,
            double *__restrict__ v, double *__restrict__ d0, double *__restrict__ d1, double *__restrict__ d2,
            double *__restrict__ d3, double *__restrict__ d4, double *__restrict__ d5, int64_t *__restrict__ t_tick,
            int32_t *__restrict__ level, const double *__restrict__ force, double eta, int rule, int k_min, int k_max,
            BatchCounters *__restrict__ ctr)
{
    const int64_t total = pl->aoff[nc];
    double *dst[6] = {d0, d1, d2, d3, d4, d5};
    const double *fnew[4] = {force, force + 3 * n, force + 6 * n, force + 9 * n};
    for (int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < total; r += int64_t(gridDim.x) * blockDim.x) {
        const int64_t i = act[r];
        if (i < 0 || i >= n) continue;
        const int fl = correct_one<P>(n, i, tnext[cid[i]], fnew, n, r, x, v, dst, t_tick, level, eta, rule, k_min, k_max);
        if (fl & 2) atomicAdd(&ctr->underflow, 1ull);
        if (fl & 1) atomicAdd(&ctr->nonfinite, 1ull);
    }
}

// Work queues back to empty (a second force pass on the same plan).
__global__ void k_b_requeue(BatchPlan *__restrict__ pl)
{
    if (threadIdx.x < kXcds) pl->queue[threadIdx.x * 16] = 0u;
}

unsigned nblk(int64_t n, int b) { return unsigned((n + b - 1) / b); }

// Workgroups of the grid-stride kernels whose work is bounded by the step's
// active count (at most n rows): enough to fill the chip, few enough that a
// step with a small active set does not pay for launching idle workgroups.
constexpr unsigned kStrideGrid = 2048;

template <class Pol, int P>
hipError_t force_p(const BatchLaunch &L, const void *rec, hipStream_t s)
{
    const auto *r = static_cast<const typename Pol::Rec *>(rec);
    if (L.itile == 64)
        hipLaunchKernelGGL((k_b_force<Pol, P, 64, kBTile, 64>), dim3(L.force_grid), dim3(64), 0, s, r, L.nc, L.act,
                           L.plan, L.eps2, L.n_hard, 3 * (P / 2), L.part);
    else if (L.itile == 128)
        hipLaunchKernelGGL((k_b_force<Pol, P, 64, kBTile, 128>), dim3(L.force_grid), dim3(64), 0, s, r, L.nc, L.act,
                           L.plan, L.eps2, L.n_hard, 3 * (P / 2), L.part);
    else
        hipLaunchKernelGGL((k_b_force<Pol, P, 256, 128, 256>), dim3(L.force_grid), dim3(256), 0, s, r, L.nc, L.act,
                           L.plan, L.eps2, L.n_hard, 3 * (P / 2), L.part);
    return hipGetLastError();
}

template <int P>
hipError_t force_prec(int precision, const BatchLaunch &L, const void *rec, hipStream_t s)
{
    if (precision == NBODY_MIXED) return force_p<PolMx<P, false>, P>(L, rec, s);
    if (precision == NBODY_DS) return force_p<PolDS<P, false>, P>(L, rec, s);
    return force_p<PolF64<P, false>, P>(L, rec, s);
}

template <int P>
hipError_t reduce_p(const BatchLaunch &L, double *o0, double *o1, double *o2, double *o3, hipStream_t s)
{
    const unsigned g = nblk(L.n * kRedLanes, 256);
    hipLaunchKernelGGL((k_b_reduce<P>), dim3(g < kStrideGrid ? g : kStrideGrid), dim3(256), 0, s, L.nc, L.n, L.plan,
                       L.act, L.cid, 3 * (P / 2), L.part, o0, o1, o2, o3, L.n);
    return hipGetLastError();
}

}  // namespace

hipError_t batch_requeue(const BatchLaunch &L, hipStream_t s)
{
    hipLaunchKernelGGL(k_b_requeue, dim3(1), dim3(64), 0, s, L.plan);
    return hipGetLastError();
}

template <class Pol, int P>
int resident_p(int itile, int device)
{
    int per_cu = 0, cus = 0;
    const hipError_t e = itile == 64
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_b_force<Pol, P, 64, kBTile, 64>, 64, 0)
        : itile == 128 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_b_force<Pol, P, 64, kBTile, 128>, 64, 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_b_force<Pol, P, 256, 128, 256>, 256, 0);
    if (e != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
    return per_cu * cus;
}

template <int P>
int resident_prec(int precision, int itile, int device)
{
    if (precision == NBODY_MIXED) return resident_p<PolMx<P, false>, P>(itile, device);
    if (precision == NBODY_DS) return resident_p<PolDS<P, false>, P>(itile, device);
    return resident_p<PolF64<P, false>, P>(itile, device);
}

int batch_force_resident(int order, int precision, int itile, int device)
{
    if (order == 4) return resident_prec<4>(precision, itile, device);
    if (order == 6) return resident_prec<6>(precision, itile, device);
    return resident_prec<8>(precision, itile, device);
}

hipError_t batch_cid(const BatchLaunch &L, hipStream_t s)
{
    hipLaunchKernelGGL(k_b_cid, dim3(nblk(L.n, 256)), dim3(256), 0, s, L.off, L.nc, L.n, L.cid);
    return hipGetLastError();
}

hipError_t batch_schedule(const BatchLaunch &L, const nbody_state &st, int all_active, int order, hipStream_t s)
{
    const dim3 g(unsigned(L.nblk));   // the clusters' scheduling blocks, flat
    hipLaunchKernelGGL(k_b_min, g, dim3(kBThreads), 0, s, L.off, st.t_tick, st.level, L.nb, L.blk, L.bmin, L.plan);
    hipLaunchKernelGGL(k_b_count, g, dim3(kBThreads), 0, s, L.off, st.t_tick, st.level, L.nb, L.blk, L.bmin,
                       all_active, L.plan, L.tnext, L.bcnt);
    hipLaunchKernelGGL(k_b_plan, dim3(1), dim3(kBThreads), 0, s, L.nc, L.off, L.ord, L.tnext, L.plan,
                       3 * (order / 2), L.k_items, L.itile, L.ctr);
    hipLaunchKernelGGL(k_b_compact, g, dim3(kBThreads), 0, s, L.off, st.t_tick, st.level, L.nb, L.blk, L.tnext,
                       L.bcnt, all_active, L.plan, L.act);
    return hipGetLastError();
}

hipError_t batch_predict(const BatchLaunch &L, const nbody_state &st, int order, int precision, void *rec,
                         hipStream_t s)
{
    const unsigned g = nblk(L.n, 256);
#define NB_BP(P, PREC)                                                                                       \
    hipLaunchKernelGGL((k_b_predict<P, PREC>), dim3(g), dim3(256), 0, s, L.n, L.cid, L.tnext, L.plan, st.m, st.x, st.v, \
                       st.d[0], st.d[1], st.d[2], st.d[3], st.d[4], st.d[5], st.t_tick, rec)
#define NB_BP_P(P)                                          \
    if (precision == NBODY_FP64) NB_BP(P, NBODY_FP64);     \
    else NB_BP(P, NBODY_MIXED)
    if (order == 4) { NB_BP_P(4); }
    else if (order == 6) { NB_BP_P(6); }
    else { NB_BP_P(8); }
#undef NB_BP_P
#undef NB_BP
    return hipGetLastError();
}

hipError_t batch_force(const BatchLaunch &L, int order, int precision, const void *rec, hipStream_t s)
{
    if (order == 4) return force_prec<4>(precision, L, rec, s);
    if (order == 6) return force_prec<6>(precision, L, rec, s);
    return force_prec<8>(precision, L, rec, s);
}

hipError_t batch_reduce(const BatchLaunch &L, int order, double *o0, double *o1, double *o2, double *o3,
                        hipStream_t s)
{
    if (order == 4) return reduce_p<4>(L, o0, o1, o2, o3, s);
    if (order == 6) return reduce_p<6>(L, o0, o1, o2, o3, s);
    return reduce_p<8>(L, o0, o1, o2, o3, s);
}

hipError_t batch_correct(const BatchLaunch &L, const nbody_config &c, const nbody_state &st, hipStream_t s)
{
    const unsigned g0 = nblk(L.n, 256);
    const unsigned g = g0 < kStrideGrid ? g0 : kStrideGrid;
#define NB_BC(P)                                                                                              \
    hipLaunchKernelGGL((k_b_correct<P>), dim3(g), dim3(256), 0, s, L.n, L.nc, L.act, L.cid, L.tnext, L.plan,     \
                       st.x, st.v, st.d[0], st.d[1], st.d[2], st.d[3], st.d[4], st.d[5], st.t_tick, st.level,    \
                       L.force, c.eta, dt_rule_of(c), int(c.k_min), int(c.k_max), L.ctr)
    if (c.order == 4) NB_BC(4);
    else if (c.order == 6) NB_BC(6);
    else NB_BC(8);
#undef NB_BC
    return hipGetLastError();
}

}  // namespace nb
