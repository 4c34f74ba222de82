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

#include "fftu_group.hpp"

namespace fftu {

template <typename T, int LOGL1, int LOGL2>
__global__ __launch_bounds__(kLineMaxThreads) void k_group2(const cx<T> *in, cx<T> *out, const PassDesc pd,
                                                            const cx<T> *__restrict__ table)
{
    constexpr int L1 = 1 << LOGL1, L2 = 1 << LOGL2;
    extern __shared__ unsigned char smem_raw[];
    cx<T> *tw1 = reinterpret_cast<cx<T> *>(smem_raw);
    cx<T> *tw2 = tw1 + L1;
    cx<T> *tile = tw2 + L2;
    const int tid = threadIdx.x;
    // launch sizes in scalar registers, read before any divergent code, so that the
    // tile loop (which holds barriers) is wave-uniform
    const int nt = __builtin_amdgcn_readfirstlane(int(blockDim.x));
    const int64_t nblocks = __builtin_amdgcn_readfirstlane(int(gridDim.x));
    for (int e = tid; e < L1; e += nt) tw1[e] = table[e << (pd.lognmax - LOGL1)];
    for (int e = tid; e < L2; e += nt) tw2[e] = table[e << (pd.lognmax - LOGL2)];
    for (int64_t t = blockIdx.x; t < pd.tiles; t += nblocks) {
        __syncthreads();   // twiddle copy done / previous tile's LDS reads done
        group2_tile<T, LOGL1, LOGL2>(in, out, pd, tw1, tw2, tile, t, tid, nt);
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
