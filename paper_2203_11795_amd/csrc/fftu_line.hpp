// k_line device code (one tile at a time), shared by the k_line kernels and the
// persistent batch kernel. See fftu_line.hip for the description of the pass.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fftu_device.hpp"
#include "fftu_internal.hpp"

namespace fftu {


// LDS index of position x of line w. Strided layout: line positions are rows of W
// (lanes run over w); contiguous layouts: one row per line, one pad element per 16
// so that radix-16 scatters (stride 16) spread over the banks.
template <int MODE>
__device__ __forceinline__ int lidx(int x, int w, int pitch)
{
    return MODE == kLineStrided ? x * pitch + w : w * pitch + x + (x >> 4);
}

// Exchange of a line through LDS between radix stage S and S+1: stage S's
// outputs are written at their Stockham positions and the next stage's inputs
// (register m <-> position j + TPL m) are read back. complex128 lines go through
// LDS as two rounds of doubles (real parts, then imaginary parts) so that a tile
// needs 8 bytes of LDS per element; complex64 lines go in one round.
template <typename T, int LOGL, int S, int MODE, int LOGE = line_loge(LOGL), typename V, typename GET>
__device__ __forceinline__ void line_scatter(const cx<T> (&v)[1 << LOGE], int j, int w, int pitch,
                                             V *lds, GET get)
{
    using PL = LinePlan<LOGL, LOGE>;
    constexpr int LR = PL::lr(S), R = 1 << LR, LNS = PL::lns(S), NB = PL::E / R;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        const int jj = j + c * PL::TPL;
        const int ob = ((jj >> LNS) << (LNS + LR)) + (jj & ((1 << LNS) - 1));
#pragma unroll
        for (int r = 0; r < R; ++r) lds[lidx<MODE>(ob + (r << LNS), w, pitch)] = get(v[c + r * NB]);
    }
}

template <typename T, int LOGL, int MODE, int LOGE = line_loge(LOGL), typename V, typename PUT>
__device__ __forceinline__ void line_gather(cx<T> (&v)[1 << LOGE], int j, int w, int pitch,
                                            const V *lds, PUT put)
{
    using PL = LinePlan<LOGL, LOGE>;
#pragma unroll
    for (int m = 0; m < PL::E; ++m) put(v[m], lds[lidx<MODE>(j + m * PL::TPL, w, pitch)]);
}

template <typename T, int LOGL, int S, int MODE, int LOGE = line_loge(LOGL)>
__device__ __forceinline__ void line_exchange(cx<T> (&v)[1 << LOGE], int j, int w, int pitch,
                                              void *smem, bool active)
{
    if constexpr (sizeof(T) == 8) {
        T *lds = static_cast<T *>(smem);
        if (active) line_scatter<T, LOGL, S, MODE, LOGE>(v, j, w, pitch, lds, [](const cx<T> &a) { return a.x; });
        __syncthreads();
        if (active) line_gather<T, LOGL, MODE, LOGE>(v, j, w, pitch, lds, [](cx<T> &a, T b) { a.x = b; });
        __syncthreads();
        if (active) line_scatter<T, LOGL, S, MODE, LOGE>(v, j, w, pitch, lds, [](const cx<T> &a) { return a.y; });
        __syncthreads();
        if (active) line_gather<T, LOGL, MODE, LOGE>(v, j, w, pitch, lds, [](cx<T> &a, T b) { a.y = b; });
    } else {
        cx<T> *lds = static_cast<cx<T> *>(smem);
        if (active) line_scatter<T, LOGL, S, MODE, LOGE>(v, j, w, pitch, lds, [](const cx<T> &a) { return a; });
        __syncthreads();
        if (active) line_gather<T, LOGL, MODE, LOGE>(v, j, w, pitch, lds, [](cx<T> &a, cx<T> b) { a = b; });
    }
}

template <typename T, int LOGL, int MODE, int LOGE = line_loge(LOGL)>
__device__ __forceinline__ void line_stages(cx<T> (&v)[1 << LOGE], int j, int w, int pitch,
                                            void *smem, const cx<T> *tw, bool active)
{
    using PL = LinePlan<LOGL, LOGE>;
    if (active) line_compute<T, LOGL, 0, LOGE>(v, j, tw);
    if constexpr (PL::NS > 1) {
        line_exchange<T, LOGL, 0, MODE, LOGE>(v, j, w, pitch, smem, active);
        if (active) line_compute<T, LOGL, 1, LOGE>(v, j, tw);
    }
    if constexpr (PL::NS > 2) {
        __syncthreads();
        line_exchange<T, LOGL, 1, MODE, LOGE>(v, j, w, pitch, smem, active);
        if (active) line_compute<T, LOGL, 2, LOGE>(v, j, tw);
    }
}

// One tile of a k_line pass: W lines (see the layouts above) with pd.threads
// working threads; threads with tid >= pd.threads (a larger workgroup) only join
// the barriers. tw holds omega_L^e, e in [L]; lds is the tile's LDS. CO: the
// results are stored device-coherently (see put()). SIGN: every loaded element is
// negated where its buffer index has an odd number of bits under pd.sign_mask.
template <typename T, int LOGL, int MODE, bool CO = false, bool SIGN = false>
__device__ __forceinline__ void line_tile(const cx<T> *in, cx<T> *out, const PassDesc &pd, const cx<T> *tw,
                                          cx<T> *lds, int64_t t, int tid)
{
    using PL = LinePlan<LOGL>;
    const int W = 1 << pd.logW;
    const int pitch = pd.lw;
    const bool active = tid < pd.threads;
    int j, w;
    if constexpr (MODE == kLineStrided) {
        w = tid & (W - 1);
        j = tid >> pd.logW;
    } else {
        j = tid & (PL::TPL - 1);
        w = tid >> PL::LOGTPL;
    }
    const T scale = static_cast<T>(pd.scale);
    auto sign_of = [&](int64_t idx, cx<T> a) {
        if constexpr (SIGN) {
            if (__popcll(uint64_t(idx) & pd.sign_mask) & 1) a = {-a.x, -a.y};
        }
        return a;
    };
    cx<T> v[PL::E];
    int64_t base;      // global offset of element 0 of this thread's line
    int64_t xstride;   // global distance between consecutive line elements
    if constexpr (MODE == kLineStrided) {
        // line u = t W + w of the (A, B) lines: outer block u / B, column u mod B (a tile
        // may span several outer blocks when B < W)
        const int64_t u = (t << pd.logW) + w;
        base = (u >> pd.logB) * pd.GB + (u & ((int64_t(1) << pd.logB) - 1));
        xstride = int64_t(1) << pd.logB;
    } else {
        base = ((t << pd.logW) + w) << LOGL;
        xstride = 1;
    }

    if constexpr (MODE == kLineStaged) {
        // the tile is W L contiguous elements: W / B outer blocks of L rows of B columns
        const int64_t tbase = (t << pd.logW) << LOGL;
        const int lb = pd.logB, bm = (1 << lb) - 1;
        // W L = threads * E: every working thread * E: every working thread moves E elements, all loads issued first
        if (active) {
            cx<T> r[PL::E];
#pragma unroll
            for (int c = 0; c < PL::E; ++c) r[c] = get<CO>(&in[tbase + tid + c * pd.threads]);
            if constexpr (SIGN) {
#pragma unroll
                for (int c = 0; c < PL::E; ++c) r[c] = sign_of(tbase + tid + c * pd.threads, r[c]);
            }
#pragma unroll
            for (int c = 0; c < PL::E; ++c) {
                const int e = tid + c * pd.threads;
                lds[lidx<MODE>((e >> lb) & (PL::L - 1), ((e >> (lb + LOGL)) << lb) | (e & bm), pitch)] =
                    conj_if(r[c], pd.conj_in);
            }
        }
        __syncthreads();
        if (active) line_gather<T, LOGL, MODE>(v, j, w, pitch, lds, [](cx<T> &a, cx<T> b) { a = b; });
        __syncthreads();
    } else if (active) {
#pragma unroll
        for (int m = 0; m < PL::E; ++m) v[m] = conj_if(get<CO>(&in[base + int64_t(j + m * PL::TPL) * xstride]), pd.conj_in);
        if constexpr (SIGN) {
#pragma unroll
            for (int m = 0; m < PL::E; ++m) v[m] = sign_of(base + int64_t(j + m * PL::TPL) * xstride, v[m]);
        }
    }

    line_stages<T, LOGL, MODE>(v, j, w, pitch, static_cast<void *>(lds), tw, active);

#pragma unroll
    for (int m = 0; m < PL::E; ++m) {
        v[m] = conj_if(v[m], pd.conj_out);
        if (pd.scale != 1.0) v[m] = {v[m].x * scale, v[m].y * scale};
    }
    if constexpr (MODE == kLineStaged) {
        if constexpr (PL::NS > 1) __syncthreads();
        if (active) {
#pragma unroll
            for (int m = 0; m < PL::E; ++m) lds[lidx<MODE>(j + m * PL::TPL, w, pitch)] = v[m];
        }
        __syncthreads();
        const int64_t tbase = (t << pd.logW) << LOGL;
        const int lb = pd.logB, bm = (1 << lb) - 1;
        if (active) {
#pragma unroll
            for (int c = 0; c < PL::E; ++c) {
                const int e = tid + c * pd.threads;
                put<CO>(&out[tbase + e], lds[lidx<MODE>((e >> lb) & (PL::L - 1), ((e >> (lb + LOGL)) << lb) | (e & bm), pitch)]);
            }
        }
    } else if (active) {
#pragma unroll
        for (int m = 0; m < PL::E; ++m) put<CO>(&out[base + int64_t(j + m * PL::TPL) * xstride], v[m]);
    }
}

// omega_L^e for e in [L] into LDS (every thread of the block takes part).
template <typename T, int LOGL>
__device__ __forceinline__ void line_twiddles(cx<T> *tw, const cx<T> *__restrict__ table, int lognmax, int tid)
{
    for (int e = tid; e < (1 << LOGL); e += blockDim.x) tw[e] = table[e << (lognmax - LOGL)];
}

}  // namespace fftu
