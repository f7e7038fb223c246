// force.hip -- the O(n_act * n) pairwise force kernels (acceleration, jerk,
// snap, crackle, potential) for gfx950, in FP64, MIXED and DS arithmetic.
//
// Direct summation of softened gravity over all j != i (paper: Abstract,
// where correlations between distant particles rule out approximations), with
// the time derivatives a Hermite scheme of order 4, 6 or 8 needs (paper:
// Sec. "Codes description").  Derivative recursion: Nitadori & Makino (2008).
//
// Launch shape: grid (i-tiles, j-splits).  A lane holds NI active particles
// in registers and the block walks its split's j range; the j records reach
// the lanes either through wave-uniform scalar loads (kernel A) or through
// LDS tiles (kernel B).  For active sets smaller than a wavefront, kernel C
// spreads each active row over several lanes instead.  With one split the
// kernel writes the final FP64 sums; with several, each split writes its
// partial sums and a second kernel adds them in a fixed order.
#include "pairwise.h"

namespace nb {
namespace {

// --------------------------------------------------------------------------
// Pieces shared by both force kernels.  blockIdx.x: i-tile of blockDim.x * NI
// active particles (lane t holds rows t, t + blockDim.x, ...); blockIdx.y:
// j-split [split * j_chunk, min(n, (split+1) * j_chunk)).  Pairs with both
// indices below n_hard are unsoftened and their self pair is masked; above
// n_hard the self pair is evaluated with eps2 > 0 (its acceleration and
// derivatives are exactly zero, every difference being zero), except in the
// kernels that also sum the potential, which mask it by index.
//
// Partial sums of launches with more than kSplitFastestAbove splits are
// stored split-fastest, part[component][row][split], so that the lanes
// reducing one output read consecutive splits; with fewer splits (one lane
// or four per output) row-fastest, part[split][component][row], so that a
// workgroup's stores are coalesced.
constexpr int kSplitFastestAbove = 32;

template <class Pol, int P, int NI>
__device__ __forceinline__ void store_rows(int64_t n_act, int64_t row0, int split, int n_split,
                                           double (*acc)[13], double *__restrict__ o_acc,
                                           double *__restrict__ o_jrk, double *__restrict__ o_snp,
                                           double *__restrict__ o_crk, double *__restrict__ o_pot,
                                           double *__restrict__ part)
{
    constexpr int NV = 3 * (P / 2);
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int64_t q = row0 + int64_t(k) * blockDim.x;
        if (q >= n_act) continue;
        const double pot = acc[k][kPot];
        if (n_split == 1) {
            double *outs[4] = {o_acc, o_jrk, o_snp, o_crk};
#pragma unroll
            for (int c = 0; c < NV; ++c) {
                double *o = outs[c / 3];
                if (o) o[(c % 3) * n_act + q] = acc[k][c];
            }
            if (Pol::kWithPot && o_pot) o_pot[q] = -pot;
        } else if (n_split > kSplitFastestAbove) {
            double *base = part + q * n_split + split;
            const int64_t cs = n_act * n_split;
#pragma unroll
            for (int c = 0; c < NV; ++c) base[c * cs] = acc[k][c];
            if (Pol::kWithPot) base[NV * cs] = -pot;
        } else {
            constexpr int NC = NV + 1;
            double *base = part + int64_t(split) * NC * n_act;
#pragma unroll
            for (int c = 0; c < NV; ++c) base[int64_t(c) * n_act + q] = acc[k][c];
            if (Pol::kWithPot) base[int64_t(NV) * n_act + q] = -pot;
        }
    }
}

// Kernel A (scalar j path): every lane walks the same j range, so each j
// record is read with a wave-uniform address into SGPRs and feeds the VALU
// directly.  Suits FP64 arithmetic, which issues at one wave instruction per
// four cycles whatever the operand source.
template <class Pol, int P, int NI>
__global__ void __launch_bounds__(256)
k_force(const typename Pol::Rec *__restrict__ rec, int64_t n, const int32_t *__restrict__ act, int64_t n_act,
        double eps2, int64_t n_hard, int64_t j_chunk, int n_split, double *__restrict__ o_acc,
        double *__restrict__ o_jrk, double *__restrict__ o_snp, double *__restrict__ o_crk,
        double *__restrict__ o_pot, double *__restrict__ part)
{
    using Rec = typename Pol::Rec;
    using Part = typename Pol::Part;
    using ET = typename Pol::ET;
    const ET e2 = ET(eps2);
    const int64_t row0 = int64_t(blockIdx.x) * blockDim.x * NI + threadIdx.x;
    const int split = blockIdx.y;
    const int64_t j0 = int64_t(split) * j_chunk;
    const int64_t j1 = (j0 + j_chunk < n) ? j0 + j_chunk : n;

    typename Pol::I ip[NI];
    int64_t iidx[NI];
    double acc[NI][13];
    load_rows<Pol, NI>(rec, n, act, n_act, row0, ip, iidx, acc);
    hard_pairs<Pol, NI>(rec, j0, (j1 < n_hard) ? j1 : n_hard, 0, n_hard, e2, ip, iidx, acc);

    const int64_t js0 = (j0 > n_hard) ? j0 : n_hard;
    constexpr int64_t CH = Pol::kChunk > 0 ? Pol::kChunk : (int64_t(1) << 40);
    Part p[NI][13];
#pragma unroll
    for (int k = 0; k < NI; ++k)
#pragma unroll
        for (int c = 0; c < 13; ++c) zero_part(p[k][c]);
    for (int64_t jc = js0; jc < j1; jc += CH) {
        const int cnt = int(((jc + CH < j1) ? jc + CH : j1) - jc);   // <= n <= 2^26
#pragma unroll 2
        for (int u = 0; u < cnt; ++u) {
            const int64_t j = jc + u;
            const Rec rj = rec[j];
#pragma unroll
            for (int k = 0; k < NI; ++k) {
                // the self pair adds nothing to a, jerk, ...; only the potential needs it masked
                if constexpr (Pol::kWithPot) Pol::template pair<true>(ip[k], rj, e2, j != iidx[k], p[k]);
                else Pol::template pair<false>(ip[k], rj, e2, true, p[k]);
            }
        }
        flush<Part, NI>(p, acc);
    }
    store_rows<Pol, P, NI>(n_act, row0, split, n_split, acc, o_acc, o_jrk, o_snp, o_crk,
                           o_pot, part);
}

// Kernel B (LDS j path): the block stages BLOCK j records at a time in LDS
// (double-buffered, the next tile's global loads in flight during the
// current tile's arithmetic) and every lane reads them with same-address
// (broadcast) LDS loads into VGPRs.  All VALU operands are then VGPRs, which
// lets FP32 instructions of two waves on a SIMD issue together -- about twice
// the FP32 rate of SGPR-operand instructions on gfx950.  The FP32 chunk
// boundaries are those of kernel A, so both give identical bits.
template <class Pol, int P, int NI, int BLOCK, int UNROLL, int TILE>
__global__ void __launch_bounds__(BLOCK)
k_force_lds(const typename Pol::Rec *__restrict__ rec, int64_t n, const int32_t *__restrict__ act, int64_t n_act,
            double eps2, int64_t n_hard, int64_t j_chunk, int n_split, double *__restrict__ o_acc,
            double *__restrict__ o_jrk, double *__restrict__ o_snp, double *__restrict__ o_crk,
            double *__restrict__ o_pot, double *__restrict__ part)
{
    using Rec = typename Pol::Rec;
    using ET = typename Pol::ET;
    __shared__ Rec tile[2][TILE];
    const ET e2 = ET(eps2);
    const int64_t row0 = int64_t(blockIdx.x) * BLOCK * NI + threadIdx.x;
    const int split = blockIdx.y;
    const int64_t j0 = int64_t(split) * j_chunk;
    const int64_t j1 = (j0 + j_chunk < n) ? j0 + j_chunk : n;

    typename Pol::I ip[NI];
    int64_t iidx[NI];
    double acc[NI][13];
    load_rows<Pol, NI>(rec, n, act, n_act, row0, ip, iidx, acc);
    hard_pairs<Pol, NI>(rec, j0, (j1 < n_hard) ? j1 : n_hard, 0, n_hard, e2, ip, iidx, acc);

    const int64_t js0 = (j0 > n_hard) ? j0 : n_hard;
    lds_tiles<Pol, NI, BLOCK, UNROLL, TILE>(rec, js0, j1, e2, ip, iidx, tile, acc);
    store_rows<Pol, P, NI>(n_act, row0, split, n_split, acc, o_acc, o_jrk, o_snp, o_crk,
                           o_pot, part);
}

// Kernel C (wave j-split, for active sets smaller than a wavefront): a
// 64-lane workgroup holds R active rows, each on JS = 64 / R lanes; lane s of
// a row takes j = j0 + s, j0 + s + JS, ... of the split's range, with vector
// loads (the JS lanes of a row read consecutive records; the rows share
// them).  The row's JS partial sums are then folded with a fixed cross-lane
// butterfly, so a workgroup's serial work is 1/JS of kernels A and B and the
// result is the same for every run.  Hard pairs (both indices below n_hard)
// and the self pair are handled per pair.
template <class Pol, int P, int R>
__global__ void __launch_bounds__(64)
k_force_ws(const typename Pol::Rec *__restrict__ rec, int64_t n, const int32_t *__restrict__ act, int64_t n_act,
           double eps2, int64_t n_hard, int64_t j_chunk, int n_split, double *__restrict__ o_acc,
           double *__restrict__ o_jrk, double *__restrict__ o_snp, double *__restrict__ o_crk,
           double *__restrict__ o_pot, double *__restrict__ part)
{
    using Rec = typename Pol::Rec;
    using Part = typename Pol::Part;
    using ET = typename Pol::ET;
    constexpr int JS = 64 / R;
    constexpr int NV = 3 * (P / 2);
    const ET e2 = ET(eps2);
    const int lane = int(threadIdx.x);
    const int r = lane / JS, sl = lane % JS;
    const int64_t q = int64_t(blockIdx.x) * R + r;
    const int split = blockIdx.y;
    const int64_t j0 = int64_t(split) * j_chunk;
    const int64_t j1 = (j0 + j_chunk < n) ? j0 + j_chunk : n;
    const int64_t qq = q < n_act ? q : n_act - 1;   // padding rows recompute the last row; never stored
    const int64_t ia = act[qq];
    const int64_t i = (ia >= 0 && ia < n) ? ia : 0;
    const typename Pol::I ip = Pol::load(rec[i]);
    const bool i_hard = i < n_hard;
    double acc[13];
    Part p[13];
#pragma unroll
    for (int c = 0; c < 13; ++c) {
        acc[c] = 0.0;
        zero_part(p[c]);
    }
    constexpr int CH = Pol::kChunk > 0 ? Pol::kChunk : (1 << 30);
    int since = 0;
    int64_t j = j0 + sl;
    Rec nxt = rec[j < j1 ? j : j1 - 1];
    for (; j < j1; j += JS) {
        const Rec rj = nxt;
        nxt = rec[j + JS < j1 ? j + JS : j1 - 1];
        const ET el = (i_hard && j < n_hard) ? ET(0) : e2;
        Pol::template pair<true>(ip, rj, el, j != i, p);
        if (++since == CH) {
            flush<Part, 1>(&p, &acc);
            since = 0;
        }
    }
    flush<Part, 1>(&p, &acc);
    // fold the JS lanes of the row (lanes r*JS .. r*JS + JS - 1)
#pragma unroll
    for (int m = JS / 2; m > 0; m >>= 1)
#pragma unroll
        for (int c = 0; c < 13; ++c) acc[c] += __shfl_xor(acc[c], m, 64);
    if (sl != 0 || q >= n_act) return;
    if (n_split == 1) {
        double *outs[4] = {o_acc, o_jrk, o_snp, o_crk};
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            double *o = outs[c / 3];
            if (o) o[(c % 3) * n_act + q] = acc[c];
        }
        if (Pol::kWithPot && o_pot) o_pot[q] = -acc[kPot];
    } else {
        // split-fastest partial sums: the reduction's lanes then read
        // consecutive splits of one output
        double *base = part + q * n_split + split;
        const int64_t cs = n_act * n_split;
#pragma unroll
        for (int c = 0; c < NV; ++c) base[c * cs] = acc[c];
        if (Pol::kWithPot) base[NV * cs] = -acc[kPot];
    }
}

// Sum of the j-split partial results.  A group of L lanes (L = 1, 4, 16 or
// 64, consecutive lanes of one wavefront) owns one output value: lane l adds
// splits l, l + L, l + 2L, ... in order, then the group folds its L sums with
// a fixed butterfly of cross-lane exchanges.  The order depends only on
// n_split and L, so reruns are bitwise identical.  Layouts: SF = false,
// part[split][component][row] (kernels A and B with at most
// kSplitFastestAbove splits: a workgroup's lanes write consecutive rows);
// SF = true, part[component][row][split] (kernels A and B with more splits,
// and the wave j-split kernels: a group's lanes read consecutive splits).
template <int P, int L, bool SF>
__global__ void __launch_bounds__(256)
k_reduce(const double *__restrict__ part, int64_t n_act, int n_split, double *__restrict__ o_acc,
         double *__restrict__ o_jrk, double *__restrict__ o_snp, double *__restrict__ o_crk,
         double *__restrict__ o_pot)
{
    constexpr int NV = 3 * (P / 2);
    constexpr int NC = NV + 1;
    const int64_t g = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / L;   // output index
    const int l = int(threadIdx.x) % L;
    const bool valid = g < n_act * NC;
    const int64_t gg = valid ? g : 0;
    const int c = int(gg / n_act);
    const int64_t q = gg - int64_t(c) * n_act;
    double s = 0.0;
    if (valid) {
        // the loads of eight splits are issued together (one memory round
        // trip instead of eight); the values are still added in split order
        const double *src = SF ? part + (int64_t(c) * n_act + q) * n_split : part + int64_t(c) * n_act + q;
        const int64_t step = SF ? 1 : int64_t(NC) * n_act;
        int sp = l;
        for (; sp + 7 * L < n_split; sp += 8 * L) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = src[int64_t(sp + u * L) * step];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; sp < n_split; sp += L) s += src[int64_t(sp) * step];
    }
#pragma unroll
    for (int m = L / 2; m > 0; m >>= 1) s += __shfl_xor(s, m, 64);
    if (!valid || l != 0) return;
    if (c == NV) {
        if (o_pot) o_pot[q] = s;
        return;
    }
    double *outs[4] = {o_acc, o_jrk, o_snp, o_crk};
    double *o = outs[c / 3];
    if (o) o[(c % 3) * n_act + q] = s;
}

template <int P, bool SF>
hipError_t launch_reduce(const ForceArgs &a, int n_split, hipStream_t s)
{
    const int64_t outs = a.n_act * (3 * (P / 2) + 1);
    // lanes per output: enough that each lane adds at most about 8 splits
    const int L = n_split <= 8 ? 1 : n_split <= 32 ? 4 : n_split <= 128 ? 16 : 64;
    const unsigned blocks = unsigned((outs * L + 255) / 256);
#define NB_RED(LL) hipLaunchKernelGGL((k_reduce<P, LL, SF>), dim3(blocks), dim3(256), 0, s, a.part, a.n_act, n_split, \
                                      a.out[0], a.out[1], a.out[2], a.out[3], a.out[4])
    if (L == 1) NB_RED(1);
    else if (L == 4) NB_RED(4);
    else if (L == 16) NB_RED(16);
    else NB_RED(64);
#undef NB_RED
    return hipGetLastError();
}

struct Shape {
    int ni, block, n_split, jpath;
    int64_t j_chunk;
};

template <class Pol, int P, int NI>
hipError_t run(const ForceArgs &a, hipStream_t s, const Shape &sh)
{
    const int64_t per_block = int64_t(sh.block) * NI;
    const int64_t tiles = (a.n_act + per_block - 1) / per_block;
    const dim3 grid{unsigned(tiles), unsigned(sh.n_split), 1u};
    const auto *rec = static_cast<const typename Pol::Rec *>(a.rec);
#define NB_FORCE_ARGS rec, a.n, a.act, a.n_act, a.eps2, a.n_hard, sh.j_chunk, sh.n_split, a.out[0], a.out[1], \
                      a.out[2], a.out[3], a.out[4], a.part
    if (sh.jpath == 3) {
        // rows per wave for the active set: 1, 4 or 16
        const int rw = a.n_act <= 1 ? 1 : (a.n_act <= 4 ? 4 : 16);
        const dim3 g3{unsigned((a.n_act + rw - 1) / rw), unsigned(sh.n_split), 1u};
        if (rw == 1) hipLaunchKernelGGL((k_force_ws<Pol, P, 1>), g3, dim3(64), 0, s, NB_FORCE_ARGS);
        else if (rw == 4) hipLaunchKernelGGL((k_force_ws<Pol, P, 4>), g3, dim3(64), 0, s, NB_FORCE_ARGS);
        else hipLaunchKernelGGL((k_force_ws<Pol, P, 16>), g3, dim3(64), 0, s, NB_FORCE_ARGS);
    } else if (sh.jpath == 1) {
        hipLaunchKernelGGL((k_force<Pol, P, NI>), grid, dim3(sh.block), 0, s, NB_FORCE_ARGS);
    } else if (sh.block == 64) {
        hipLaunchKernelGGL((k_force_lds<Pol, P, NI, 64, 2, 64>), grid, dim3(64), 0, s, NB_FORCE_ARGS);
    } else if (sh.block == 128) {
        hipLaunchKernelGGL((k_force_lds<Pol, P, NI, 128, 2, 128>), grid, dim3(128), 0, s, NB_FORCE_ARGS);
    } else {
        hipLaunchKernelGGL((k_force_lds<Pol, P, NI, 256, 2, 128>), grid, dim3(256), 0, s, NB_FORCE_ARGS);
    }
#undef NB_FORCE_ARGS
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || sh.n_split == 1) return e;
    if (sh.jpath == 3 || sh.n_split > kSplitFastestAbove) return launch_reduce<P, true>(a, sh.n_split, s);
    return launch_reduce<P, false>(a, sh.n_split, s);
}

template <class Pol, int P>
hipError_t run_ni(const ForceArgs &a, hipStream_t s, const Shape &sh)
{
    if (sh.ni == 2 && sh.jpath != 3) return run<Pol, P, 2>(a, s, sh);
    return run<Pol, P, 1>(a, s, sh);
}

template <int P, bool POT>
hipError_t run_pot(int precision, const ForceArgs &a, hipStream_t s, const Shape &sh)
{
    switch (precision) {
    case NBODY_MIXED: return run_ni<PolMx<P, POT>, P>(a, s, sh);
    case NBODY_DS: return run_ni<PolDS<P, POT>, P>(a, s, sh);
    default: return run_ni<PolF64<P, POT>, P>(a, s, sh);
    }
}

// The potential is accumulated only when it is asked for.
template <int P>
hipError_t run_prec(int precision, const ForceArgs &a, hipStream_t s, const Shape &sh)
{
    return a.out[4] ? run_pot<P, true>(precision, a, s, sh) : run_pot<P, false>(precision, a, s, sh);
}

}  // namespace

int record_bytes(int order, int precision)
{
    if (precision == NBODY_FP64) return order == 4 ? 64 : order == 6 ? 80 : 112;
    return order == 8 ? 80 : 64;
}

// Number of j-splits: enough waves to cover every SIMD several times when the
// active set is small, bounded by the partial-sum scratch and by keeping at
// least 256 j per split.
int auto_split(int64_t n, int64_t n_act, int ni, int block, int64_t part_rows)
{
    const int64_t per_block = int64_t(block) * ni;
    const int64_t tiles = (n_act + per_block - 1) / per_block;
    const int64_t waves = tiles * (block / 64);
    const int64_t target_waves = 256 * 4 * 8;   // CUs x SIMDs x waves per SIMD
    int64_t sp = (target_waves + waves - 1) / waves;
    const int64_t max_by_n = n / kMixedChunk > 0 ? n / kMixedChunk : 1;   // splits of at least one FP32 chunk
    const int64_t max_by_part = part_rows / (n_act > 0 ? n_act : 1);
    if (sp > max_by_n) sp = max_by_n;
    if (sp > max_by_part) sp = max_by_part;
    if (sp > 65535) sp = 65535;
    return sp < 1 ? 1 : int(sp);
}

int auto_split_path(int64_t n, int64_t n_act, int ni, int block, int jpath, int64_t part_rows)
{
    if (jpath != 3) return auto_split(n, n_act, ni, block, part_rows);
    // kernel C: one 64-lane workgroup per 1, 4 or 16 rows and split.  Split
    // counts giving about 512, 1024 and 2048 workgroups were the fastest on
    // MI355X (n = 2^17 and 2^20, orders 6 and 8, with and without the
    // predictor inside): shorter splits cost more in per-workgroup set-up and
    // in the split reduction than they add in parallelism.
    const int64_t rw = n_act <= 1 ? 1 : (n_act <= 4 ? 4 : 16);
    const int64_t tiles = (n_act + rw - 1) / rw;
    const int64_t target = rw == 1 ? 512 : (rw == 4 ? 1024 : 2048);
    int64_t sp = (target + tiles - 1) / tiles;
    const int64_t max_by_n = n / kMixedChunk > 0 ? n / kMixedChunk : 1;
    const int64_t max_by_part = part_rows / (n_act > 0 ? n_act : 1);
    if (sp > max_by_n) sp = max_by_n;
    if (sp > max_by_part) sp = max_by_part;
    if (sp > 65535) sp = 65535;
    return sp < 1 ? 1 : int(sp);
}

void split_shape(int64_t n, int64_t n_act, int n_split_req, int ni, int block, int jpath, int64_t part_rows,
                 int *n_split, int64_t *j_chunk)
{
    int sp = n_split_req > 0 ? n_split_req : auto_split_path(n, n_act, ni, block, jpath, part_rows);
    if (n_act > 0 && int64_t(sp) * n_act > part_rows) sp = int(part_rows / n_act);
    if (sp < 1) sp = 1;
    // split length: a multiple of the MIXED chunk so chunks never straddle splits
    int64_t jc = (n + sp - 1) / sp;
    jc = (jc + kMixedChunk - 1) / kMixedChunk * kMixedChunk;
    *j_chunk = jc;
    *n_split = int((n + jc - 1) / jc);
}

hipError_t launch_split_reduce_sf(int order, const ForceArgs &a, int n_split, hipStream_t s)
{
    if (order == 4) return launch_reduce<4, true>(a, n_split, s);
    if (order == 6) return launch_reduce<6, true>(a, n_split, s);
    return launch_reduce<8, true>(a, n_split, s);
}

hipError_t launch_force(int order, int precision, const ForceArgs &a, hipStream_t s, UsedShape *used)
{
    Shape sh{};
    sh.ni = (a.ni == 2) ? 2 : 1;
    sh.block = (a.block == 64 || a.block == 128) ? a.block : 256;
    // j path: FP64 reads j records from SGPRs, the FP32 modes from LDS
    sh.jpath = a.jpath >= 1 && a.jpath <= 3 ? a.jpath : (precision == NBODY_FP64 ? 1 : 2);
    split_shape(a.n, a.n_act, a.n_split, sh.ni, sh.block, sh.jpath, a.part_rows, &sh.n_split, &sh.j_chunk);
    if (used) *used = UsedShape{sh.jpath == 3 ? 1 : sh.ni, sh.jpath == 3 ? 64 : sh.block, sh.n_split, sh.jpath};
    switch (order) {
    case 4: return run_prec<4>(precision, a, s, sh);
    case 6: return run_prec<6>(precision, a, s, sh);
    default: return run_prec<8>(precision, a, s, sh);
    }
}

}  // namespace nb
