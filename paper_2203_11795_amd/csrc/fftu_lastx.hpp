// k_lastx: the innermost dimension's Superstep-0 FFTs, Superstep 0's twiddle,
// Superstep 1 (the one all-to-all) and Superstep 2 (the length-p FFTs) of
// Algorithm 2.3 (arXiv 2203.11795) in one pass over HBM.
//
// Superstep 0 is a d-D FFT per block and its dimensions may be taken in any
// order (eq. (1.3)), so the other local dimensions run first as ordinary passes
// and the innermost one comes last. A workgroup takes the same RW consecutive
// rows (lines along the innermost dimension, fixed k_1 .. k_{d-1}) of every one of
// the P blocks: P RW lines of m_d contiguous elements, which is all the sources
// of RW m_d consecutive local indices k. It transforms the lines in registers
// and LDS (the k_line contiguous layout), transposes through LDS so that each
// thread holds, for one k, the sources of the exchange's register dimensions,
// and finishes as k_exchange does: twiddle by prod_l omega_{n_l}^{k_l s'_l},
// the length-p_l DFTs, and the scatter to V^(r)[t + k' q] (Theorem 2.1).
//
// The tile is 2^LOGNT threads x E elements, E = 2^LOGR the register sources per
// thread of the exchange and the elements per thread of the line plan alike.
// complex128 goes through LDS as two rounds of doubles.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fftu_device.hpp"
#include "fftu_exchange.hpp"
#include "fftu_internal.hpp"
#include "fftu_line.hpp"

namespace fftu {

template <int LOGL, int LOGR, int LOGH, int LOGNT>
struct LastxShape {
    using PL = LinePlan<LOGL, lastx_loge(LOGL, LOGR)>;
    static constexpr int LOGP = LOGR + LOGH;
    static constexpr int LOGW = LOGNT - PL::LOGTPL;   // lines per tile: P x RW
    static constexpr int LOGRW = LOGW - LOGP;         // rows per tile
    static constexpr int LOGK = LOGRW + LOGL;         // local indices per tile
    static constexpr int L = 1 << LOGL;
    static constexpr int LP = L + PL::TPL;            // LDS row of the transpose: L + L/32 swizzled words, padded
    static constexpr int PITCH = L + L / 16 + 1;      // LDS row of the line stages (see lidx)
    static constexpr int WORDS = (1 << LOGW) * (LP > PITCH ? LP : PITCH);   // 8-byte LDS words
};

// 512 threads: two workgroups per CU, 4 waves per SIMD, at most 128 VGPRs. 1024
// threads: one workgroup of 16 waves per CU, the same register bound. MUL: every
// output is multiplied by lx.ex.mul at its position (convolution); the multipliers
// are all loaded before the stores, so the 512-thread bound leaves the compiler up
// to 256 VGPRs. TL: the exchange's twiddles come from an LDS copy of the omega
// table, placed after the work area (the planner takes it when two 512-thread
// workgroups per CU still fit).
// One tile of k_lastx; MULM is the exchange's store mode (exchange_store: 1 plain,
// 2 the pointwise product, 3 the signs under lx.ex.sign_mask).
template <typename T, int LOGL, int NR, int LPR, int NH, int LPH, int MULM, bool TL, int LOGNT>
__device__ __forceinline__ void lastx_tile(const cx<T> *__restrict__ in, cx<T> *__restrict__ out, const LastxDesc &lx,
                                           const cx<T> *__restrict__ table)
{
    constexpr int LOGR = NR * LPR, LOGH = NH * LPH;
    constexpr int NT = 1 << LOGNT;
    using S = LastxShape<LOGL, LOGR, LOGH, LOGNT>;
    using PL = typename S::PL;
    static_assert(lastx_split_ok(LOGL, NR, LPR, NH, LPH, LOGNT), "k_lastx: no such split");
    static_assert(PL::LOGE == LOGR && S::LOGRW >= 0, "k_lastx: the line plan and the exchange split disagree");
    static_assert(lastx_lds_bytes(LOGL, PL::LOGE, sizeof(cx<T>), LOGNT) == S::L * sizeof(cx<T>) + S::WORDS * 8,
                  "k_lastx: LDS size");
    constexpr int R = 1 << LOGR;
    constexpr int H = 1 << LOGH;
    constexpr int KG = (NT / 64) / H;
    static_assert(KG * 64 == (1 << S::LOGK), "k_lastx: one tile is KG groups of 64 local indices");

    extern __shared__ unsigned char smem_raw[];
    cx<T> *tw = reinterpret_cast<cx<T> *>(smem_raw);
    unsigned char *work = smem_raw + S::L * sizeof(cx<T>);
    const int tid = threadIdx.x;
    line_twiddles<T, LOGL>(tw, table, lx.ex.g.lognmax, tid);
    cx<T> *ttab = reinterpret_cast<cx<T> *>(work + S::WORDS * 8);
    if constexpr (TL)
        for (int e = tid; e < (1 << lx.ex.g.lognmax); e += NT) ttab[e] = table[e];

    // line layout: thread (w, j) holds line w = s RW + row, register m <-> position j + TPL m
    const int j = tid & (PL::TPL - 1);
    const int w = tid >> PL::LOGTPL;
    const int s = w >> S::LOGRW;
    const int row = w & ((1 << S::LOGRW) - 1);
    // exchange layout: thread (grp, hw, lane) holds, for the sources (hw, jj), jj in [R],
    // tile index i = grp 64 + lane taken as (row, r_d, t_d) with t_d fastest, i.e. the local
    // index k_d = r_d + p_d t_d of that row, so that consecutive lanes store consecutive t_d
    // (runs of q_d elements in one destination block)
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int hw = wv & (H - 1);
    const int grp = wv >> LOGH;
    const int lpd = lx.ex.g.logp[lx.ex.g.d - 1];
    const int i = grp * 64 + lane;
    const int f = (((i & (S::L - 1)) & ((S::L >> lpd) - 1)) << lpd) + ((i & (S::L - 1)) >> (LOGL - lpd));
    const int kk = (i & ~(S::L - 1)) + f;
    // LDS word of line position x: x + x / 32 keeps reads at a stride of p_d on distinct banks
    const int rd = ((hw << LOGR) << S::LOGRW) * S::LP + (kk >> LOGL) * S::LP + f + (f >> 5);

    const int logM = lx.ex.g.logmstride[0] + lx.ex.g.logm[0];
    {
        const int64_t tile = blockIdx.x;   // one tile per workgroup (the launcher checks the grid)
        cx<T> v[PL::E];
        if constexpr (lastx_staged_load(LOGL, PL::LOGE, sizeof(cx<T>))) {
            // a thread's run of a line (TPL elements) is under 128 bytes: read the tile's
            // RW L contiguous elements of each block linearly instead (64 consecutive
            // elements per wave instruction) and hand each thread its line positions
            // through LDS, as k_line's staged layout does
            cx<T> r[PL::E];
#pragma unroll
            for (int c = 0; c < PL::E; ++c) {
                const int e = tid + c * NT;
                r[c] = conj_if(get(&in[(int64_t(e >> S::LOGK) << logM) + (tile << S::LOGK) + (e & ((1 << S::LOGK) - 1))]),
                               lx.conj_in);
            }
            // element e is position e mod L of line e / L
            auto at = [&](int e) { return lidx<kLineContig>(e & (S::L - 1), e >> LOGL, S::PITCH); };
            auto mine = [&](int m) { return lidx<kLineContig>(j + m * PL::TPL, w, S::PITCH); };
            if constexpr (sizeof(T) == 8) {
                T *ld = reinterpret_cast<T *>(work);
#pragma unroll
                for (int c = 0; c < PL::E; ++c) ld[at(tid + c * NT)] = r[c].x;
                __syncthreads();
#pragma unroll
                for (int m = 0; m < PL::E; ++m) v[m].x = ld[mine(m)];
                __syncthreads();
#pragma unroll
                for (int c = 0; c < PL::E; ++c) ld[at(tid + c * NT)] = r[c].y;
                __syncthreads();
#pragma unroll
                for (int m = 0; m < PL::E; ++m) v[m].y = ld[mine(m)];
            } else {
                cx<T> *ld = reinterpret_cast<cx<T> *>(work);
#pragma unroll
                for (int c = 0; c < PL::E; ++c) ld[at(tid + c * NT)] = r[c];
                __syncthreads();
#pragma unroll
                for (int m = 0; m < PL::E; ++m) v[m] = ld[mine(m)];
            }
            __syncthreads();   // the gathers are done before line_stages reuses the area
        } else {
            const int64_t base = (int64_t(s) << logM) + (((tile << S::LOGRW) + row) << LOGL);
#pragma unroll
            for (int m = 0; m < PL::E; ++m) v[m] = conj_if(get(&in[base + j + m * PL::TPL]), lx.conj_in);
            __syncthreads();   // the omega_L table is in LDS
        }

        line_stages<T, LOGL, kLineContig, PL::LOGE>(v, j, w, S::PITCH, static_cast<void *>(work), tw, true);

        // transpose: element (s, row, x) to LDS word (s RW + row) LP + x + x / 32, read back
        // as (hw R + jj, kk); the register index is the row of R LP RW words
        cx<T> u[R];
        auto wr = [&](int m) {
            const int x = j + m * PL::TPL;
            return w * S::LP + x + (x >> 5);
        };
        __syncthreads();
        if constexpr (sizeof(T) == 8) {
            T *ld = reinterpret_cast<T *>(work);
#pragma unroll
            for (int m = 0; m < PL::E; ++m) ld[wr(m)] = v[m].x;
            __syncthreads();
#pragma unroll
            for (int jj = 0; jj < R; ++jj) u[jj].x = ld[rd + (jj << S::LOGRW) * S::LP];
            __syncthreads();
#pragma unroll
            for (int m = 0; m < PL::E; ++m) ld[wr(m)] = v[m].y;
            __syncthreads();
#pragma unroll
            for (int jj = 0; jj < R; ++jj) u[jj].y = ld[rd + (jj << S::LOGRW) * S::LP];
        } else {
            cx<T> *ld = reinterpret_cast<cx<T> *>(work);
#pragma unroll
            for (int m = 0; m < PL::E; ++m) ld[wr(m)] = v[m];
            __syncthreads();
#pragma unroll
            for (int jj = 0; jj < R; ++jj) u[jj] = ld[rd + (jj << S::LOGRW) * S::LP];
        }

        exchange_core<T, NR, LPR, NH, LPH, NT, false, MULM>(
            out, lx.ex, TL ? ttab : table, work, (tile << S::LOGK) + kk, tid,
            [&](int jj, int, int64_t, bool) { return u[jj]; });
    }
}

template <typename T, int LOGL, int NR, int LPR, int NH, int LPH, bool MUL, bool TL, int LOGNT>
__global__ __launch_bounds__(1 << LOGNT, (MUL && LOGNT == 9) ? 2 : 4) void k_lastx(const cx<T> *__restrict__ in,
                                                                      cx<T> *__restrict__ out, const LastxDesc lx,
                                                                      const cx<T> *__restrict__ table)
{
    lastx_tile<T, LOGL, NR, LPR, NH, LPH, MUL ? 2 : 1, TL, LOGNT>(in, out, lx, table);
}

// k_lastx with every output negated by the parity of its buffer index under
// lx.ex.sign_mask (no product; MUL is false, kept so that the name lists the same
// arguments): the last kernel of a transform whose result is wanted with signs.
template <typename T, int LOGL, int NR, int LPR, int NH, int LPH, bool MUL, bool TL, int LOGNT>
__global__ __launch_bounds__(1 << LOGNT, 4) void k_lastx_sign(const cx<T> *__restrict__ in, cx<T> *__restrict__ out,
                                                              const LastxDesc lx, const cx<T> *__restrict__ table)
{
    static_assert(!MUL, "k_lastx_sign: no product");
    lastx_tile<T, LOGL, NR, LPR, NH, LPH, 3, TL, LOGNT>(in, out, lx, table);
}

namespace lastx_detail {

template <typename T, int LOGL, int NR, int LPR, int NH, int LPH, int LOGNT>
hipError_t go_nt(const void *in, void *out, const LastxDesc &lx, const void *table, hipStream_t stream)
{
    if (lx.tiles < 1 || lx.tiles > lastx_max_tiles(LOGNT)) return hipErrorInvalidValue;
    const uint32_t blocks = uint32_t(lx.tiles);
    const dim3 threads(1u << LOGNT);
    const cx<T> *a = static_cast<const cx<T> *>(in), *tab = static_cast<const cx<T> *>(table);
    cx<T> *b = static_cast<cx<T> *>(out);
    const uint32_t base = lastx_lds_bytes(LOGL, lastx_loge(LOGL, NR * LPR), sizeof(cx<T>), LOGNT);
    if (lx.ex.sign_mask != 0) {
        if (lx.ex.mul) return hipErrorInvalidValue;   // signs and a product are not combined
        if (lx.table_lds) {
            if constexpr (LOGNT == kLastxLogThreads) {
                if (lx.lds_bytes != base + (uint32_t(sizeof(cx<T>)) << lx.ex.g.lognmax)) return hipErrorInvalidValue;
                hipLaunchKernelGGL((k_lastx_sign<T, LOGL, NR, LPR, NH, LPH, false, true, LOGNT>), dim3(blocks), threads,
                                   lx.lds_bytes, stream, a, b, lx, tab);
            } else {
                return hipErrorInvalidValue;
            }
        } else {
            if (lx.lds_bytes != base) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_lastx_sign<T, LOGL, NR, LPR, NH, LPH, false, false, LOGNT>), dim3(blocks), threads,
                               lx.lds_bytes, stream, a, b, lx, tab);
        }
    } else if (lx.ex.mul) {
        if (lx.lds_bytes != base) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_lastx<T, LOGL, NR, LPR, NH, LPH, true, false, LOGNT>), dim3(blocks), threads,
                           lx.lds_bytes, stream, a, b, lx, tab);
    } else if (lx.table_lds) {
        if constexpr (LOGNT == kLastxLogThreads) {
            if (lx.lds_bytes != base + (uint32_t(sizeof(cx<T>)) << lx.ex.g.lognmax)) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_lastx<T, LOGL, NR, LPR, NH, LPH, false, true, LOGNT>), dim3(blocks), threads,
                               lx.lds_bytes, stream, a, b, lx, tab);
        } else {
            return hipErrorInvalidValue;
        }
    } else {
        if (lx.lds_bytes != base) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_lastx<T, LOGL, NR, LPR, NH, LPH, false, false, LOGNT>), dim3(blocks), threads,
                           lx.lds_bytes, stream, a, b, lx, tab);
    }
    return hipGetLastError();
}

template <typename T, int LOGL, int NR, int LPR, int NH, int LPH>
hipError_t go(const void *in, void *out, const LastxDesc &lx, const void *table, hipStream_t stream)
{
    if constexpr (lastx_split_ok(LOGL, NR, LPR, NH, LPH, kLastxLogThreads)) {
        if (lx.lognt == kLastxLogThreads) return go_nt<T, LOGL, NR, LPR, NH, LPH, kLastxLogThreads>(in, out, lx, table, stream);
    } else if constexpr (lastx_split_needs_1024(LOGL, NR, LPR, NH, LPH)) {
        if (lx.lognt == kLastxMaxLogThreads)
            return go_nt<T, LOGL, NR, LPR, NH, LPH, kLastxMaxLogThreads>(in, out, lx, table, stream);
    }
    return hipErrorInvalidValue;
}

template <typename T, int LOGL, int NR, int LPR>
hipError_t waves(const void *in, void *out, const LastxDesc &lx, const void *table, hipStream_t stream)
{
    const ExchangeDesc &ex = lx.ex;
    if (ex.nh == 0) return go<T, LOGL, NR, LPR, 0, 0>(in, out, lx, table, stream);
    if (ex.nh == 1 && ex.lph == 1) return go<T, LOGL, NR, LPR, 1, 1>(in, out, lx, table, stream);
    if (ex.nh == 1 && ex.lph == 2) return go<T, LOGL, NR, LPR, 1, 2>(in, out, lx, table, stream);
    if (ex.nh == 2 && ex.lph == 1) return go<T, LOGL, NR, LPR, 2, 1>(in, out, lx, table, stream);
    return hipErrorInvalidValue;
}

template <typename T, int LOGL>
hipError_t regs(const void *in, void *out, const LastxDesc &lx, const void *table, hipStream_t stream)
{
    const ExchangeDesc &ex = lx.ex;
    if constexpr (line_loge(LOGL) == 3) {
        if (ex.nr == 3 && ex.lpr == 1) return waves<T, LOGL, 3, 1>(in, out, lx, table, stream);
        if constexpr (lastx_loge(LOGL, 4) == 4) {   // lines of 64 as 16 elements per thread
            if (ex.nr == 4 && ex.lpr == 1) return waves<T, LOGL, 4, 1>(in, out, lx, table, stream);
            if (ex.nr == 2 && ex.lpr == 2) return waves<T, LOGL, 2, 2>(in, out, lx, table, stream);
        }
    } else if constexpr (line_loge(LOGL) == 4) {
        if (ex.nr == 4 && ex.lpr == 1) return waves<T, LOGL, 4, 1>(in, out, lx, table, stream);
        if (ex.nr == 2 && ex.lpr == 2) return waves<T, LOGL, 2, 2>(in, out, lx, table, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace lastx_detail

// Host launcher for one element type (instantiated in fftu_lastx_f32.hip / fftu_lastx_f64.hip).
template <typename T>
hipError_t launch_lastx_t(const void *in, void *out, const LastxDesc &lx, const void *table, hipStream_t stream)
{
    if (lx.ex.g.conj_in != 0) return hipErrorInvalidValue;
    switch (lx.logl) {
    case 5: return lastx_detail::regs<T, 5>(in, out, lx, table, stream);
    case 6: return lastx_detail::regs<T, 6>(in, out, lx, table, stream);
    case 7: return lastx_detail::regs<T, 7>(in, out, lx, table, stream);
    case 8: return lastx_detail::regs<T, 8>(in, out, lx, table, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_lastx_f32(const void *in, void *out, const LastxDesc &lx, const void *table, hipStream_t stream);
hipError_t launch_lastx_f64(const void *in, void *out, const LastxDesc &lx, const void *table, hipStream_t stream);

}  // namespace fftu
