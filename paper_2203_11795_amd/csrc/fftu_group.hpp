// k_group2 device code (one tile of whole planes at a time), shared by the
// k_group2 kernels and the persistent batch kernel. See fftu_group.hip for the
// description of the pass.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fftu_device.hpp"
#include "fftu_internal.hpp"

namespace fftu {

constexpr int kGroupUnroll = 8;

// Stage S's outputs written back to their Stockham positions in the line.
template <typename T, int LOGL, int S>
__device__ __forceinline__ void group_scatter(const cx<T> (&v)[LinePlan<LOGL>::E], cx<T> *tile, int base, int stride,
                                              int j)
{
    using PL = LinePlan<LOGL>;
    constexpr int LR = PL::lr(S), R = 1 << LR, LNS = PL::lns(S), NB = PL::E / R;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        const int jj = j + c * PL::TPL;
        const int ob = ((jj >> LNS) << (LNS + LR)) + (jj & ((1 << LNS) - 1));
#pragma unroll
        for (int r = 0; r < R; ++r) tile[base + (ob + (r << LNS)) * stride] = v[c + r * NB];
    }
}

// All lines of one dimension of the tile: line of thread `u` (if active) starts
// at tile index `base` and has positions `stride` apart. Every thread executes
// every barrier.
template <typename T, int LOGL>
__device__ __forceinline__ void group_axis(cx<T> *tile, int base, int stride, int j, bool active,
                                           const cx<T> *tw)
{
    using PL = LinePlan<LOGL>;
    cx<T> v[PL::E];
    if (active) {
#pragma unroll
        for (int m = 0; m < PL::E; ++m) v[m] = tile[base + (j + m * PL::TPL) * stride];
    }
    __syncthreads();
    if (active) line_compute<T, LOGL, 0>(v, j, tw);
    if constexpr (PL::NS > 1) {
        if (active) group_scatter<T, LOGL, 0>(v, tile, base, stride, j);
        __syncthreads();
        if (active) {
#pragma unroll
            for (int m = 0; m < PL::E; ++m) v[m] = tile[base + (j + m * PL::TPL) * stride];
            line_compute<T, LOGL, 1>(v, j, tw);
        }
    }
    if constexpr (PL::NS > 2) {
        __syncthreads();
        if (active) group_scatter<T, LOGL, 1>(v, tile, base, stride, j);
        __syncthreads();
        if (active) {
#pragma unroll
            for (int m = 0; m < PL::E; ++m) v[m] = tile[base + (j + m * PL::TPL) * stride];
            line_compute<T, LOGL, 2>(v, j, tw);
        }
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int m = 0; m < PL::E; ++m) tile[base + (j + m * PL::TPL) * stride] = v[m];
    }
    __syncthreads();
}

// One tile of a k_group2 pass: W = 2^pd.logW whole planes of L1 x L2 elements,
// from in to out (in place allowed). tw1 / tw2 hold omega_L1 / omega_L2; tile is
// the LDS tile. Threads beyond the pass's own (a larger workgroup) only join the
// barriers. nt = the workgroup's size, wave-uniform. CO: the results are stored
// device-coherently (see put()).
template <typename T, int LOGL1, int LOGL2, bool CO = false>
__device__ __forceinline__ void group2_tile(const cx<T> *in, cx<T> *out, const PassDesc &pd, const cx<T> *tw1,
                                            const cx<T> *tw2, cx<T> *tile, int64_t t, int tid, int nt)
{
    using P1 = LinePlan<LOGL1>;
    using P2L = LinePlan<LOGL2>;
    constexpr int L1 = 1 << LOGL1, L2 = 1 << LOGL2, LOGG = LOGL1 + LOGL2;
    constexpr int P2 = L2 + 1, PG = L1 * P2;
    const int W = 1 << pd.logW;
    // inner-dimension lines (w, x1): thread -> (line, j), j fastest
    const int u2 = tid >> P2L::LOGTPL, j2 = tid & (P2L::TPL - 1);
    const bool act2 = u2 < (W << LOGL1);
    const int base2 = (u2 >> LOGL1) * PG + (u2 & (L1 - 1)) * P2;
    // outer-dimension lines (w, x2)
    const int u1 = tid >> P1::LOGTPL, j1 = tid & (P1::TPL - 1);
    const bool act1 = u1 < (W << LOGL2);
    const int base1 = (u1 >> LOGL2) * PG + (u1 & (L2 - 1));
    const T scale = static_cast<T>(pd.scale);
    const int n = W << LOGG;
    const int64_t gbase = (t << pd.logW) << LOGG;
    // loads in groups of kGroupUnroll per thread, all issued before the LDS writes
    for (int e0 = tid; e0 < n; e0 += kGroupUnroll * nt) {
        cx<T> r[kGroupUnroll];
#pragma unroll
        for (int u = 0; u < kGroupUnroll; ++u)
            if (e0 + u * nt < n) r[u] = get<CO>(&in[gbase + e0 + u * nt]);
#pragma unroll
        for (int u = 0; u < kGroupUnroll; ++u) {
            const int e = e0 + u * nt;
            if (e < n) {
                const int w = e >> LOGG, x1 = (e >> LOGL2) & (L1 - 1), x2 = e & (L2 - 1);
                tile[w * PG + x1 * P2 + x2] = conj_if(r[u], pd.conj_in);
            }
        }
    }
    __syncthreads();   // the whole tile is in LDS before any line is read
    group_axis<T, LOGL2>(tile, base2, 1, j2, act2, tw2);
    group_axis<T, LOGL1>(tile, base1, P2, j1, act1, tw1);
    // stores in groups of kGroupUnroll per thread: the LDS reads first, then the stores
    for (int e0 = tid; e0 < n; e0 += kGroupUnroll * nt) {
        cx<T> r[kGroupUnroll];
#pragma unroll
        for (int u = 0; u < kGroupUnroll; ++u) {
            const int e = e0 + u * nt;
            if (e < n) {
                const int w = e >> LOGG, x1 = (e >> LOGL2) & (L1 - 1), x2 = e & (L2 - 1);
                r[u] = conj_if(tile[w * PG + x1 * P2 + x2], pd.conj_out);
            }
        }
#pragma unroll
        for (int u = 0; u < kGroupUnroll; ++u) {
            const int e = e0 + u * nt;
            if (e < n) {
                cx<T> v = r[u];
                if (pd.scale != 1.0) v = {v.x * scale, v.y * scale};
                put<CO>(&out[gbase + e], v);
            }
        }
    }
}

}  // namespace fftu
