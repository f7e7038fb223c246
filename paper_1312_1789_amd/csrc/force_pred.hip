// force_pred.hip -- the wave j-split force kernel with the j-particle
// predictor folded into its j loads, for block steps with few active
// particles.
//
// Each block step predicts every particle to the block time and then sums the
// force on the active ones over all of them (paper: Sec. "Codes
// description").  With few active particles the separate predictor pass
// (read the stored state, write a record) and the force pass (read the
// records back) are both bound by HBM traffic over all n particles.  Here
// each workgroup predicts the j-particles of its split itself as it walks
// them: the stored state is read once, no record is written or read.
//
// The arithmetic is the predictor's (predict_state) and the pair term's
// (Pol::pair), and every lane visits its j-particles in the order of the
// unfused wave j-split kernel, with the same FP32 chunk boundaries, so the
// results equal, bit for bit, those of the predictor followed by that kernel.
#include <type_traits>

#include "hermite.h"
#include "pairwise.h"

namespace nb {
namespace {

// R active rows per 64-lane workgroup, JS = 64 / R lanes per row; lane
// (r, sl) takes j = j0 + sl, j0 + sl + JS, ... of the split [j0, j1).  The
// workgroup walks its split in tiles of 64: lane l predicts j-particle
// jt + l (its stored state was loaded one tile ahead) into LDS, and row r's
// lanes then take the tile's j-particles sl, sl + JS, ..., sl + (R-1) JS.
// With one row per workgroup (JS = 64) a lane's own prediction is its only
// j-particle of the tile, and the record stays in registers.
template <class Pol, int P, int PREC, int R>
__global__ void __launch_bounds__(64)
k_force_wsp(PredIn in, int64_t n, const int32_t *__restrict__ act, int64_t n_act, double eps2, int64_t n_hard,
            int64_t j_chunk, int n_split, double *__restrict__ o_acc, double *__restrict__ o_jrk,
            double *__restrict__ o_snp, double *__restrict__ o_crk, double *__restrict__ o_pot,
            double *__restrict__ part)
{
    using Rec = typename Pol::Rec;
    using Part = typename Pol::Part;
    using ET = typename Pol::ET;
    static_assert(std::is_same<Rec, typename PredRec<P, PREC>::type>::value, "record type of the precision");
    constexpr int JS = 64 / R;
    constexpr int NV = 3 * (P / 2);
    constexpr double kInvTick = 1.0 / double(kTicksPerUnit);
    const ET e2 = ET(eps2);
    const int lane = int(threadIdx.x);
    const int r = lane / JS, sl = lane % JS;
    const int64_t q = int64_t(blockIdx.x) * R + r;
    const int split = blockIdx.y;
    const int64_t j0 = int64_t(split) * j_chunk;
    const int64_t j1 = (j0 + j_chunk < n) ? j0 + j_chunk : n;   // j0 < n for every split
    const int64_t qq = q < n_act ? q : n_act - 1;   // padding rows recompute the last row; never stored
    const int64_t ia = act[qq];
    const int64_t i = (ia >= 0 && ia < n) ? ia : 0;
    const typename Pol::I ip = Pol::load(predict_state<P, PREC>(load_pstate<P>(n, i, in.m, in.x, in.v, in.d),
                                                                double(in.t - in.t_tick[i]) * kInvTick));
    const bool i_hard = i < n_hard;
    double acc[13];
    Part p[13];
#pragma unroll
    for (int c = 0; c < 13; ++c) {
        acc[c] = 0.0;
        zero_part(p[c]);
    }
    constexpr int CH = Pol::kChunk > 0 ? Pol::kChunk : (1 << 30);
    static_assert(CH % R == 0, "chunk length a multiple of the rows per workgroup");
    int since = 0;
    __shared__ Rec tile[R > 1 ? 64 : 1];
    // stored state of this lane's first j-particle (lanes past j1 take j1 - 1,
    // whose record is never used)
    int64_t jn = j0 + lane < j1 ? j0 + lane : j1 - 1;
    PState<P> nx = load_pstate<P>(n, jn, in.m, in.x, in.v, in.d);
    int64_t tn = in.t_tick[jn];
    for (int64_t jt = j0; jt < j1; jt += 64) {
        const PState<P> cur = nx;
        const int64_t tc = tn;
        jn = jt + 64 + lane < j1 ? jt + 64 + lane : j1 - 1;   // next tile, loaded during this one
        nx = load_pstate<P>(n, jn, in.m, in.x, in.v, in.d);
        tn = in.t_tick[jn];
        const Rec mine = predict_state<P, PREC>(cur, double(in.t - tc) * kInvTick);
        const int cnt = j1 - jt < 64 ? int(j1 - jt) : 64;
        if constexpr (R == 1) {
            if (lane < cnt) {
                const int64_t j = jt + lane;
                const ET el = (i_hard && j < n_hard) ? ET(0) : e2;
                Pol::template pair<true>(ip, mine, el, j != i, p);
                if (++since == CH) {
                    flush<Part, 1>(&p, &acc);
                    since = 0;
                }
            }
        } else {
            tile[lane] = mine;
            __syncthreads();
            // A full tile without the row's own particle and without hard
            // pairs needs no per-pair checks; the chunk counter then moves by
            // R at once (the chunk length is a multiple of R, and only the
            // split's last tile can be partial, so the flushes fall on the
            // same pairs as with per-pair counting).  Not with the potential:
            // without the self-pair select the compiler may fuse m_j / r into
            // the potential sum as one FMA, which rounds differently.
            const bool plain = !Pol::kWithPot && cnt == 64 && (i < jt || i >= jt + 64) && !(i_hard && jt < n_hard);
            if (plain) {
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const Rec rj = tile[sl + k * JS];
                    Pol::template pair<false>(ip, rj, e2, true, p);
                }
                since += R;
                if (since == CH) {
                    flush<Part, 1>(&p, &acc);
                    since = 0;
                }
            } else {
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const int u = sl + k * JS;
                    if (u < cnt) {
                        const int64_t j = jt + u;
                        const Rec rj = tile[u];
                        const ET el = (i_hard && j < n_hard) ? ET(0) : e2;
                        Pol::template pair<true>(ip, rj, el, j != i, p);
                        if (++since == CH) {
                            flush<Part, 1>(&p, &acc);
                            since = 0;
                        }
                    }
                }
            }
            __syncthreads();
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
        // split-fastest partial sums, as the unfused wave j-split kernel
        double *base = part + q * n_split + split;
        const int64_t cs = n_act * n_split;
#pragma unroll
        for (int c = 0; c < NV; ++c) base[c * cs] = acc[c];
        if (Pol::kWithPot) base[NV * cs] = -acc[kPot];
    }
}

template <class Pol, int P, int PREC>
hipError_t run(const ForceArgs &a, const PredIn &in, hipStream_t s, int n_split, int64_t j_chunk)
{
    // rows per workgroup for the active set: 1, 4 or 16 (as the unfused kernel)
    const int rw = a.n_act <= 1 ? 1 : (a.n_act <= 4 ? 4 : 16);
    const dim3 grid{unsigned((a.n_act + rw - 1) / rw), unsigned(n_split), 1u};
#define NB_WSP(RR) hipLaunchKernelGGL((k_force_wsp<Pol, P, PREC, RR>), grid, dim3(64), 0, s, in, a.n, a.act, a.n_act, \
                                      a.eps2, a.n_hard, j_chunk, n_split, a.out[0], a.out[1], a.out[2], a.out[3],  \
                                      a.out[4], a.part)
    if (rw == 1) NB_WSP(1);
    else if (rw == 4) NB_WSP(4);
    else NB_WSP(16);
#undef NB_WSP
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n_split == 1) return e;
    return launch_split_reduce_sf(P, a, n_split, s);
}

template <int P, bool POT>
hipError_t run_pot(int precision, const ForceArgs &a, const PredIn &in, hipStream_t s, int n_split, int64_t jc)
{
    switch (precision) {
    case NBODY_MIXED: return run<PolMx<P, POT>, P, NBODY_MIXED>(a, in, s, n_split, jc);
    case NBODY_DS: return run<PolDS<P, POT>, P, NBODY_DS>(a, in, s, n_split, jc);
    default: return run<PolF64<P, POT>, P, NBODY_FP64>(a, in, s, n_split, jc);
    }
}

template <int P>
hipError_t run_prec(int precision, const ForceArgs &a, const PredIn &in, hipStream_t s, int n_split, int64_t jc)
{
    return a.out[4] ? run_pot<P, true>(precision, a, in, s, n_split, jc)
                    : run_pot<P, false>(precision, a, in, s, n_split, jc);
}

}  // namespace

hipError_t launch_force_pred(int order, int precision, const ForceArgs &a, const PredIn &in, hipStream_t s,
                             UsedShape *used)
{
    int n_split = 1;
    int64_t j_chunk = 0;
    split_shape(a.n, a.n_act, a.n_split, 1, 64, 3, a.part_rows, &n_split, &j_chunk);
    if (used) *used = UsedShape{1, 64, n_split, 3};
    switch (order) {
    case 4: return run_prec<4>(precision, a, in, s, n_split, j_chunk);
    case 6: return run_prec<6>(precision, a, in, s, n_split, j_chunk);
    default: return run_prec<8>(precision, a, in, s, n_split, j_chunk);
    }
}

}  // namespace nb
