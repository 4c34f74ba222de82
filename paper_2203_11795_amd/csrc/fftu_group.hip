// k_group2: the local FFT of Superstep 0 (Algorithm 2.3, arXiv 2203.11795) over
// the two innermost local dimensions at once, for small contiguous planes
// (L1 x L2 elements, both sides 4..64).
//
// A workgroup moves W whole planes (W L1 L2 contiguous elements) from HBM into an
// LDS tile with linear, fully coalesced loads; transforms every line along the
// inner dimension, then every line along the outer one, each with the register
// radix stages of k_line (line exchanges happen in place in the tile); and writes
// the tile back linearly. One pass over HBM instead of two.
//
// Tile layout: plane w, row x1, column x2 at w*PG + x1*P2 + x2 with P2 = L2 + 1,
// so that lines along x1 (stride P2, odd) spread over the LDS banks.
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

template <typename T, int LOGL1, int LOGL2>
__global__ __launch_bounds__(kLineMaxThreads) void k_group2(const cx<T> *in, cx<T> *out, const PassDesc pd,
                                                            const cx<T> *__restrict__ table)
{
    using P1 = LinePlan<LOGL1>;
    using P2L = LinePlan<LOGL2>;
    constexpr int L1 = 1 << LOGL1, L2 = 1 << LOGL2, LOGG = LOGL1 + LOGL2;
    constexpr int P2 = L2 + 1, PG = L1 * P2;
    extern __shared__ unsigned char smem_raw[];
    cx<T> *tw1 = reinterpret_cast<cx<T> *>(smem_raw);
    cx<T> *tw2 = tw1 + L1;
    cx<T> *tile = tw2 + L2;
    const int W = 1 << pd.logW;
    const int tid = threadIdx.x;
    // launch sizes in scalar registers, read before any divergent code, so that the
    // tile loop (which holds barriers) is wave-uniform
    const int nt = __builtin_amdgcn_readfirstlane(int(blockDim.x));
    const int64_t nblocks = __builtin_amdgcn_readfirstlane(int(gridDim.x));
    for (int e = tid; e < L1; e += nt) tw1[e] = table[e << (pd.lognmax - LOGL1)];
    for (int e = tid; e < L2; e += nt) tw2[e] = table[e << (pd.lognmax - LOGL2)];

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
    for (int64_t t = blockIdx.x; t < pd.tiles; t += nblocks) {
        __syncthreads();
        const int64_t gbase = (t << pd.logW) << LOGG;
        // loads in groups of kGroupUnroll per thread, all issued before the LDS writes
        for (int e0 = tid; e0 < n; e0 += kGroupUnroll * nt) {
            cx<T> r[kGroupUnroll];
#pragma unroll
            for (int u = 0; u < kGroupUnroll; ++u)
                if (e0 + u * nt < n) r[u] = in[gbase + e0 + u * nt];
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
        for (int e = tid; e < n; e += nt) {
            const int w = e >> LOGG, x1 = (e >> LOGL2) & (L1 - 1), x2 = e & (L2 - 1);
            cx<T> v = conj_if(tile[w * PG + x1 * P2 + x2], pd.conj_out);
            if (pd.scale != 1.0) v = {v.x * scale, v.y * scale};
            out[gbase + e] = v;
        }
    }
}

namespace {
constexpr int64_t kMaxGroupBlocks = int64_t(1) << 21;

template <typename T, int A, int B>
hipError_t launch_g(const void *in, void *out, const PassDesc &pd, const void *table, hipStream_t stream)
{
    const uint32_t blocks = uint32_t(pd.tiles < kMaxGroupBlocks ? pd.tiles : kMaxGroupBlocks);
    hipLaunchKernelGGL((k_group2<T, A, B>), dim3(blocks), dim3(uint32_t(pd.threads)), pd.lds_bytes, stream,
                       static_cast<const cx<T> *>(in), static_cast<cx<T> *>(out), pd,
                       static_cast<const cx<T> *>(table));
    return hipGetLastError();
}

template <typename T, int A>
hipError_t launch_gb(const void *in, void *out, const PassDesc &pd, const void *table, hipStream_t stream)
{
    switch (pd.loglen[1]) {
    case 2: return launch_g<T, A, 2>(in, out, pd, table, stream);
    case 3: return launch_g<T, A, 3>(in, out, pd, table, stream);
    case 4: return launch_g<T, A, 4>(in, out, pd, table, stream);
    case 5: return launch_g<T, A, 5>(in, out, pd, table, stream);
    case 6: return launch_g<T, A, 6>(in, out, pd, table, stream);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_ga(const void *in, void *out, const PassDesc &pd, const void *table, hipStream_t stream)
{
    switch (pd.loglen[0]) {
    case 2: return launch_gb<T, 2>(in, out, pd, table, stream);
    case 3: return launch_gb<T, 3>(in, out, pd, table, stream);
    case 4: return launch_gb<T, 4>(in, out, pd, table, stream);
    case 5: return launch_gb<T, 5>(in, out, pd, table, stream);
    case 6: return launch_gb<T, 6>(in, out, pd, table, stream);
    default: return hipErrorInvalidValue;
    }
}
}  // namespace

hipError_t launch_group2(Precision prec, const void *in, void *out, const PassDesc &pd, const void *table,
                         hipStream_t stream)
{
    return prec == Precision::F64 ? launch_ga<double>(in, out, pd, table, stream)
                                  : launch_ga<float>(in, out, pd, table, stream);
}

}  // namespace fftu
