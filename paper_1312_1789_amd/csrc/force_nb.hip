// force_nb.hip -- the pairwise force split by neighbour spheres, with the
// neighbour lists (the Ahmad & Cohen 1973 scheme of the paper's second code,
// NBODY6++GPU, Sec. "Results": the GPU evaluates the force from the distant
// particles and the neighbour lists; the near, fast-changing part is summed
// over the list on its own shorter steps).
//
// For active particle i with neighbour radius squared h2[q], particle j != i
// is a neighbour when its unsoftened squared distance is below h2[q]; the
// kernel tests r^2 + eps_ij^2 < h2[q] + eps_ij^2 in its own precision, on the
// sum the pair term forms anyway.  Acceleration and jerk (the terms of the 4th-order
// scheme, softened as in the full force) are summed over the other particles
// (regular part) and over the neighbours (irregular part); the neighbour list
// holds their indices in increasing order.
//
// Kernel 1, grid (i-tiles of kNbBlock rows, j-splits): each lane holds one
// active row and walks its split in increasing j, adding the pair terms of
// the non-neighbours (the neighbours are masked out of the same FMA sequence
// as the full force) and appending the neighbours to its split's part of the
// list.  The j below n_hard (unsoftened when i is hard too) are taken one by
// one with their checks; the rest streams through LDS tiles of kNbBlock
// records with no per-pair index test: the self pair (difference zero, r^2 =
// eps^2 > 0) either is a neighbour, and is dropped at the append, or adds
// exact zeros to the regular part.  Kernel 2, one wave per
// row: the regular partial sums added in split order, the split lists
// concatenated, and the irregular part summed over the list (lanes take
// every 64th entry, then a fixed butterfly).  A row whose list was cut at
// max_nb gets NaN for its irregular part.
#include "pairwise.h"

namespace nb {
namespace {

constexpr int kNbBlock = 128;

// One pair of the regular sum: the differences, the softened r^2 + eps_ij^2,
// the neighbour test r^2 + eps_ij^2 < h^2 + eps_ij^2 (the unsoftened test,
// written on the sum the pair term forms anyway), and the pair's order-4
// terms added when j is valid and not a neighbour.  Returns whether j is a
// neighbour.  hh_e = h^2 + eps_ij^2 for the pair's softening.
__device__ __forceinline__ bool nb_pair(const typename PolF64<4, false>::I &i, const RecF64<4> &j, double el,
                                        double hh_e, bool valid, double *A)
{
    const double dx = j.x - i.x, dy = j.y - i.y, dz = j.z - i.z;
    const double wx = j.vx - i.vx, wy = j.vy - i.vy, wz = j.vz - i.vz;
    const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, el)));
    const bool is_nb = valid && r2 < hh_e;
    const bool ok = valid && !is_nb;
    const double rinv = rsqrt64(ok ? r2 : 1.0);
    const double mr = ok ? j.m * rinv : 0.0;
    core_fma<4, false, double>(dx, dy, dz, wx, wy, wz, 0, 0, 0, 0, 0, 0, mr, rinv * rinv, A);
    return is_nb;
}

// The pair of the LDS-tile loop: softened (eps2 > 0, so r^2 > 0), no
// validity test (the self pair is handled as stated above).
__device__ __forceinline__ bool nb_pair_soft(const typename PolF64<4, false>::I &i, const RecF64<4> &j, double e2,
                                             double hh_e, double *A)
{
    const double dx = j.x - i.x, dy = j.y - i.y, dz = j.z - i.z;
    const double wx = j.vx - i.vx, wy = j.vy - i.vy, wz = j.vz - i.vz;
    const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, e2)));
    const bool is_nb = r2 < hh_e;
    const double rinv = rsqrt64(r2);
    const double mr = is_nb ? 0.0 : j.m * rinv;
    core_fma<4, false, double>(dx, dy, dz, wx, wy, wz, 0, 0, 0, 0, 0, 0, mr, rinv * rinv, A);
    return is_nb;
}

__device__ __forceinline__ bool nb_pair_soft(const typename DSIn<4>::I &i, const RecDS<4> &j, float e2, float hh_e,
                                             float *A)
{
    const float dx = (j.xh - i.xh) + (j.xl - i.xl);
    const float dy = (j.yh - i.yh) + (j.yl - i.yl);
    const float dz = (j.zh - i.zh) + (j.zl - i.zl);
    const float wx = (j.vxh - i.vxh) + (j.vxl - i.vxl);
    const float wy = (j.vyh - i.vyh) + (j.vyl - i.vyl);
    const float wz = (j.vzh - i.vzh) + (j.vzl - i.vzl);
    const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, e2)));
    const bool is_nb = r2 < hh_e;
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float mr = is_nb ? 0.0f : j.m * rinv;
    core_fma<4, false, float>(dx, dy, dz, wx, wy, wz, 0, 0, 0, 0, 0, 0, mr, rinv * rinv, A);
    return is_nb;
}

__device__ __forceinline__ bool nb_pair(const typename DSIn<4>::I &i, const RecDS<4> &j, float el, float hh_e,
                                        bool valid, float *A)
{
    const float dx = (j.xh - i.xh) + (j.xl - i.xl);
    const float dy = (j.yh - i.yh) + (j.yl - i.yl);
    const float dz = (j.zh - i.zh) + (j.zl - i.zl);
    const float wx = (j.vxh - i.vxh) + (j.vxl - i.vxl);
    const float wy = (j.vyh - i.vyh) + (j.vyl - i.vyl);
    const float wz = (j.vzh - i.vzh) + (j.vzl - i.vzl);
    const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, el)));
    const bool is_nb = valid && r2 < hh_e;
    const bool ok = valid && !is_nb;
    const float rinv = __builtin_amdgcn_rsqf(ok ? r2 : 1.0f);
    const float mr = ok ? j.m * rinv : 0.0f;
    core_fma<4, false, float>(dx, dy, dz, wx, wy, wz, 0, 0, 0, 0, 0, 0, mr, rinv * rinv, A);
    return is_nb;
}

template <class Pol>
__global__ void __launch_bounds__(kNbBlock)
k_force_nb(const typename Pol::Rec *__restrict__ rec, int64_t n, const int32_t *__restrict__ act, int64_t n_act,
           const double *__restrict__ h2, double eps2, int64_t n_hard, int64_t j_chunk, int max_nb,
           double *__restrict__ part, int32_t *__restrict__ seg_cnt, int32_t *__restrict__ seg)
{
    using Rec = typename Pol::Rec;
    using ET = typename Pol::ET;
    using Part = typename Pol::Part;
    const int64_t q = int64_t(blockIdx.x) * kNbBlock + threadIdx.x;
    const int split = blockIdx.y;
    const int64_t j0 = int64_t(split) * j_chunk;
    const int64_t j1 = (j0 + j_chunk < n) ? j0 + j_chunk : n;   // j0 < n for every split
    const bool row = q < n_act;
    const int64_t qq = row ? q : n_act - 1;   // padding lanes recompute the last row; never stored
    const int64_t ia = act[qq];
    const int64_t i = (ia >= 0 && ia < n) ? ia : 0;
    const typename Pol::I ip = Pol::load(rec[i]);
    const ET e2 = ET(eps2);
    const ET hh_e = ET(h2[qq] + eps2), hh_0 = ET(h2[qq]);   // h^2 + eps_ij^2 for soft and hard pairs
    const bool i_hard = i < n_hard;
    double acc[13];
    Part p[13];
#pragma unroll
    for (int c = 0; c < 13; ++c) {
        acc[c] = 0.0;
        zero_part(p[c]);
    }
    static_assert(Pol::kChunk == 0 || Pol::kChunk == kNbBlock, "one FP32 chunk per tile");
    int cnt = 0;
    int32_t *my_seg = seg + (int64_t(split) * n_act + qq) * max_nb;
    // j below n_hard: each pair's terms added into FP64 on their own
    const int64_t jh1 = j1 < n_hard ? j1 : n_hard;
    for (int64_t j = j0; j < jh1; ++j) {
        const Rec rj = rec[j];
        Part ph[13];
#pragma unroll
        for (int c = 0; c < 13; ++c) zero_part(ph[c]);
        const bool is_nb = nb_pair(ip, rj, i_hard ? ET(0) : e2, i_hard ? hh_0 : hh_e, j != i, ph);
        if (is_nb) {
            if (row && cnt < max_nb) my_seg[cnt] = int32_t(j);
            ++cnt;
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] += to_double(ph[c]);
    }
    // the rest (softened pairs) through LDS tiles; the FP32 sums are flushed
    // after every tile (one chunk)
    __shared__ Rec tile[kNbBlock];
    const int64_t js0 = j0 > n_hard ? j0 : n_hard;
    for (int64_t jt = js0; jt < j1; jt += kNbBlock) {
        const int64_t jl = jt + threadIdx.x;
        if (jl < j1) tile[threadIdx.x] = rec[jl];
        __syncthreads();
        const int m = j1 - jt < kNbBlock ? int(j1 - jt) : kNbBlock;
        for (int u = 0; u < m; ++u) {
            const Rec rj = tile[u];
            if (nb_pair_soft(ip, rj, e2, hh_e, p)) {
                const int64_t j = jt + u;
                if (j != i) {
                    if (row && cnt < max_nb) my_seg[cnt] = int32_t(j);
                    ++cnt;
                }
            }
        }
        flush<Part, 1>(&p, &acc);
        __syncthreads();
    }
    if (!row) return;
    // split-fastest: the finishing kernel's lanes read consecutive splits
    const int n_split = int(gridDim.y);
#pragma unroll
    for (int c = 0; c < 6; ++c) part[(int64_t(c) * n_act + q) * n_split + split] = acc[c];
    seg_cnt[q * n_split + split] = cnt;
}

// One 64-lane workgroup per active row: for each of the 6 regular
// components, lane l adds the row's partial sums of splits l, l + 64, ... in
// order and a fixed butterfly folds the lanes; all lanes copy the splits'
// neighbour lists one after the other (increasing j, at most max_nb entries);
// then lane l adds the irregular terms of list entries l, l + 64, ... and the
// lanes' sums are folded with a fixed butterfly.
template <class Pol>
__global__ void __launch_bounds__(64)
k_nb_finish(const typename Pol::Rec *__restrict__ rec, int64_t n, const int32_t *__restrict__ act, int64_t n_act,
            double eps2, int64_t n_hard, int n_split, int max_nb, const double *__restrict__ part,
            const int32_t *__restrict__ seg_cnt, const int32_t *__restrict__ seg, double *__restrict__ acc_irr,
            double *__restrict__ jrk_irr, double *__restrict__ acc_reg, double *__restrict__ jrk_reg,
            int32_t *__restrict__ nb_count, int32_t *__restrict__ nb_list)
{
    using ET = typename Pol::ET;
    using Part = typename Pol::Part;
    const int64_t q = blockIdx.x;
    const int l = int(threadIdx.x);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        // the loads of eight of this lane's splits in flight together, added in split order
        const double *src = part + (int64_t(c) * n_act + q) * n_split;
        double s = 0.0;
        int sp = l;
        for (; sp + 7 * 64 < n_split; sp += 8 * 64) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = src[sp + u * 64];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; sp < n_split; sp += 64) s += src[sp];
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) s += __shfl_xor(s, m, 64);
        if (l == 0) (c < 3 ? acc_reg : jrk_reg)[(c % 3) * n_act + q] = s;
    }
    // the lists: 64 splits at a time, lane l taking split s0 + l; a prefix sum
    // over the lanes places each split's entries after those of the splits
    // before it, and at most max_nb entries are kept in all.  The counts of
    // up to kNbPass passes are loaded together first (one memory round trip
    // for them instead of one per pass).
    constexpr int kNbPass = 16;
    int64_t total = 0;
    int written = 0;
    int cnts[kNbPass];
    for (int s0 = 0; s0 < n_split; s0 += 64) {
        const int pass = (s0 / 64) % kNbPass;
        if (pass == 0) {
#pragma unroll
            for (int k = 0; k < kNbPass; ++k) {
                const int spk = s0 + 64 * k + l;
                cnts[k] = spk < n_split ? seg_cnt[q * n_split + spk] : 0;
            }
        }
        const int sp = s0 + l;
        int c = 0;
#pragma unroll
        for (int k = 0; k < kNbPass; ++k) c = k == pass ? cnts[k] : c;
        const int stored = c < max_nb ? c : max_nb;
        int incl = stored;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(incl, o, 64);
            if (l >= o) incl += t;
        }
        const int base = written + (incl - stored);
        const int room = max_nb - base;
        const int take = room <= 0 ? 0 : (stored < room ? stored : room);
        const int32_t *src = seg + (int64_t(sp < n_split ? sp : 0) * n_act + q) * max_nb;
        for (int k = 0; k < take; ++k) nb_list[q * max_nb + base + k] = src[k];
        const int all = __shfl(incl, 63, 64);
        written = written + all < max_nb ? written + all : max_nb;
        int64_t cs = c;
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) cs += __shfl_xor(cs, m, 64);
        total += cs;
    }
    if (l == 0) nb_count[q] = int32_t(total);
    __syncthreads();   // the row's list is complete in memory
    const int64_t ia = act[q];
    const int64_t i = (ia >= 0 && ia < n) ? ia : 0;
    const typename Pol::I ip = Pol::load(rec[i]);
    const ET e2 = ET(eps2);
    const bool i_hard = i < n_hard;
    double acc[13];
    Part p[13];
#pragma unroll
    for (int c = 0; c < 13; ++c) {
        acc[c] = 0.0;
        zero_part(p[c]);
    }
    for (int k = l; k < written; k += 64) {   // at most 64 terms per lane: one FP32 chunk
        const int64_t j = nb_list[q * max_nb + k];
        Pol::template pair<true>(ip, rec[j], (i_hard && j < n_hard) ? ET(0) : e2, true, p);
    }
    flush<Part, 1>(&p, &acc);
#pragma unroll
    for (int m = 32; m > 0; m >>= 1)
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] += __shfl_xor(acc[c], m, 64);
    if (l < 6) {
        const double v = total > written ? __builtin_nan("") : acc[l];   // a cut list: no irregular part
        (l < 3 ? acc_irr : jrk_irr)[(l % 3) * n_act + q] = v;
    }
}

template <class Pol>
hipError_t run_nb(const NbArgs &a, hipStream_t s, int n_split, int64_t j_chunk)
{
    const unsigned tiles = unsigned((a.n_act + kNbBlock - 1) / kNbBlock);
    double *part = a.scratch;
    int32_t *seg_cnt = reinterpret_cast<int32_t *>(part + int64_t(n_split) * 6 * a.n_act);
    int32_t *seg = seg_cnt + int64_t(n_split) * a.n_act;
    hipLaunchKernelGGL((k_force_nb<Pol>), dim3(tiles, unsigned(n_split)), dim3(kNbBlock), 0, s,
                       static_cast<const typename Pol::Rec *>(a.rec), a.n, a.act, a.n_act, a.h2, a.eps2, a.n_hard,
                       j_chunk, a.max_nb, part, seg_cnt, seg);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_nb_finish<Pol>), dim3(unsigned(a.n_act)), dim3(64), 0, s,
                       static_cast<const typename Pol::Rec *>(a.rec), a.n, a.act, a.n_act, a.eps2, a.n_hard, n_split,
                       a.max_nb, part, seg_cnt, seg, a.acc_irr, a.jrk_irr, a.acc_reg, a.jrk_reg, a.nb_count,
                       a.nb_list);
    return hipGetLastError();
}

}  // namespace

// Bytes of scratch one (split, row) pair needs: 6 partial sums, a count and
// max_nb list entries.
int64_t nb_scratch_per_row(int max_nb) { return 6 * 8 + 4 + 4 * int64_t(max_nb); }

int nb_split(int64_t n, int64_t n_act, int max_nb, int64_t scratch_bytes, int n_split_req)
{
    const int64_t tiles = (n_act + kNbBlock - 1) / kNbBlock;
    // about 4096 workgroups of 128 lanes (8 waves per SIMD; the kernel fits
    // 6 at a time), splits of at least one tile, and what the scratch holds
    int64_t sp = n_split_req > 0 ? n_split_req : (4096 + tiles - 1) / tiles;
    const int64_t by_n = (n + kNbBlock - 1) / kNbBlock;
    const int64_t by_scratch = scratch_bytes / (nb_scratch_per_row(max_nb) * (n_act > 0 ? n_act : 1));
    if (sp > by_n) sp = by_n;
    if (sp > by_scratch) sp = by_scratch;
    if (sp > 65535) sp = 65535;
    return int(sp);   // 0: the scratch cannot hold one split
}

hipError_t launch_force_nb(int precision, const NbArgs &a, int n_split, hipStream_t s, int *used_split)
{
    // split length: whole tiles of kNbBlock j (a multiple of the MIXED chunk)
    int64_t j_chunk = (a.n + n_split - 1) / n_split;
    j_chunk = (j_chunk + kNbBlock - 1) / kNbBlock * kNbBlock;
    const int sp = int((a.n + j_chunk - 1) / j_chunk);
    if (used_split) *used_split = sp;
    if (precision == NBODY_MIXED) return run_nb<PolMx<4, false>>(a, s, sp, j_chunk);
    return run_nb<PolF64<4, false>>(a, s, sp, j_chunk);
}

}  // namespace nb
