// k_exchange: Superstep 0's twiddle, Superstep 1 (the one all-to-all) and
// Superstep 2 (the length-p FFTs) of Algorithm 2.3 (arXiv 2203.11795) in one
// pass over HBM.
//
// For a local index k = r + t p (elementwise, r in [p], t in [q]) the values
// Z^(s')[k] of all P source processors s' are the inputs of one
// F_{p_1} x ... x F_{p_d} (Theorem 2.1: W^(r)[s' q + t] = Z^(s')[r + t p]), whose
// output k' lands in V^(r)[t + k' q]. So the exchange needs no separate
// permutation buffer: a group of 64 consecutive k (one per lane) is gathered from
// every source block (each load instruction reads 64 consecutive elements of one
// block), twiddled by prod_l omega_{n_l}^{k_l s'_l} (one table entry per element,
// exponent reduced exactly in integers), transformed, and scattered (each store
// instruction writes runs of 64/p_d consecutive elements).
//
// The grid dimensions with p_l > 1 split into NH leading "wave" dimensions of
// 2^LPH each and NR trailing "register" dimensions of 2^LPR each. A thread holds
// the 2^(NR LPR) sources of one wave index, applies the register dimensions'
// DFTs with compile-time constant roots, the waves swap values through LDS so
// that each thread holds every wave index for 1/2^(NH LPH) of the register
// outputs, and the wave dimensions' DFTs follow the same way.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fftu_exchange.hpp"

namespace fftu {

// Without a pointwise product (ex.mul null): the product's code would hold 32 more
// VGPRs (158 against 126 for complex128 <2, 2, 1, 2>), one wave per SIMD less.
template <typename T, int NR, int LPR, int NH, int LPH>
__global__ __launch_bounds__(kExchangeThreads) void k_exchange(const cx<T> *__restrict__ Z, cx<T> *__restrict__ V,
                                                               const ExchangeDesc ex, const cx<T> *__restrict__ table)
{
    constexpr int KG = (kExchangeThreads / 64) >> (NH * LPH);
    extern __shared__ unsigned char smem_raw[];
    const int64_t ngroups = (ex.g.M + 63) >> 6;
    const int64_t nblocks = __builtin_amdgcn_readfirstlane(int(gridDim.x));   // uniform loop (barriers inside)
    for (int64_t gb = int64_t(blockIdx.x) * KG; gb < ngroups; gb += nblocks * KG)
        exchange_group<T, NR, LPR, NH, LPH, false, 1>(Z, V, ex, table, smem_raw, gb, threadIdx.x);
}

// With the pointwise product by ex.mul (a convolution's filter spectrum).
template <typename T, int NR, int LPR, int NH, int LPH>
__global__ __launch_bounds__(kExchangeThreads) void k_exchange_mul(const cx<T> *__restrict__ Z,
                                                                   cx<T> *__restrict__ V, const ExchangeDesc ex,
                                                                   const cx<T> *__restrict__ table)
{
    constexpr int KG = (kExchangeThreads / 64) >> (NH * LPH);
    extern __shared__ unsigned char smem_raw[];
    const int64_t ngroups = (ex.g.M + 63) >> 6;
    const int64_t nblocks = __builtin_amdgcn_readfirstlane(int(gridDim.x));   // uniform loop (barriers inside)
    for (int64_t gb = int64_t(blockIdx.x) * KG; gb < ngroups; gb += nblocks * KG)
        exchange_group<T, NR, LPR, NH, LPH, false, 0>(Z, V, ex, table, smem_raw, gb, threadIdx.x);
}

// k_exchange with every output negated by the parity of its buffer index under
// ex.sign_mask (no pointwise product): the last kernel of a transform whose result
// is wanted with signs (the inverse DST-II's signal).
template <typename T, int NR, int LPR, int NH, int LPH>
__global__ __launch_bounds__(kExchangeThreads) void k_exchange_sign(const cx<T> *__restrict__ Z,
                                                                    cx<T> *__restrict__ V, const ExchangeDesc ex,
                                                                    const cx<T> *__restrict__ table)
{
    constexpr int KG = (kExchangeThreads / 64) >> (NH * LPH);
    extern __shared__ unsigned char smem_raw[];
    const int64_t ngroups = (ex.g.M + 63) >> 6;
    const int64_t nblocks = __builtin_amdgcn_readfirstlane(int(gridDim.x));   // uniform loop (barriers inside)
    for (int64_t gb = int64_t(blockIdx.x) * KG; gb < ngroups; gb += nblocks * KG)
        exchange_group<T, NR, LPR, NH, LPH, false, 3>(Z, V, ex, table, smem_raw, gb, threadIdx.x);
}

namespace {
constexpr int64_t kMaxExchangeBlocks = int64_t(1) << 20;

template <typename T, int NR, int LPR, int NH, int LPH>
hipError_t launch_t(const void *in, void *out, const ExchangeDesc &ex, const void *table, hipStream_t stream)
{
    constexpr int KG = (kExchangeThreads / 64) >> (NH * LPH);
    const int64_t ngroups = (ex.g.M + 63) >> 6;
    const int64_t want = (ngroups + KG - 1) / KG;
    const uint32_t blocks = uint32_t(want < kMaxExchangeBlocks ? want : kMaxExchangeBlocks);
    if (ex.sign_mask != 0) {
        if (ex.mul) return hipErrorInvalidValue;   // signs and a product are not combined
        hipLaunchKernelGGL((k_exchange_sign<T, NR, LPR, NH, LPH>), dim3(blocks), dim3(kExchangeThreads), ex.lds_bytes,
                           stream, static_cast<const cx<T> *>(in), static_cast<cx<T> *>(out), ex,
                           static_cast<const cx<T> *>(table));
        return hipGetLastError();
    }
    if (ex.mul)
        hipLaunchKernelGGL((k_exchange_mul<T, NR, LPR, NH, LPH>), dim3(blocks), dim3(kExchangeThreads), ex.lds_bytes,
                           stream, static_cast<const cx<T> *>(in), static_cast<cx<T> *>(out), ex,
                           static_cast<const cx<T> *>(table));
    else
        hipLaunchKernelGGL((k_exchange<T, NR, LPR, NH, LPH>), dim3(blocks), dim3(kExchangeThreads), ex.lds_bytes,
                           stream, static_cast<const cx<T> *>(in), static_cast<cx<T> *>(out), ex,
                           static_cast<const cx<T> *>(table));
    return hipGetLastError();
}

// Wave part: none, one dimension of 2 or 4, or two dimensions of 2.
template <typename T, int NR, int LPR>
hipError_t launch_h(const void *in, void *out, const ExchangeDesc &ex, const void *table, hipStream_t stream)
{
    constexpr int LOGR = NR * LPR;
    if (ex.nh == 0) return launch_t<T, NR, LPR, 0, 0>(in, out, ex, table, stream);
    if constexpr (LOGR >= 1)
        if (ex.nh == 1 && ex.lph == 1) return launch_t<T, NR, LPR, 1, 1>(in, out, ex, table, stream);
    if constexpr (LOGR >= 2) {
        if (ex.nh == 1 && ex.lph == 2) return launch_t<T, NR, LPR, 1, 2>(in, out, ex, table, stream);
        if (ex.nh == 2 && ex.lph == 1) return launch_t<T, NR, LPR, 2, 1>(in, out, ex, table, stream);
    }
    return hipErrorInvalidValue;
}

// Register part: NR dimensions of 2^LPR with NR * LPR <= MAXR.
template <typename T, int MAXR>
hipError_t launch_r(const void *in, void *out, const ExchangeDesc &ex, const void *table, hipStream_t stream)
{
    const int key = ex.nr * 8 + ex.lpr;
    switch (key) {
    case 0 * 8 + 0: return launch_h<T, 0, 0>(in, out, ex, table, stream);
    case 1 * 8 + 1: return launch_h<T, 1, 1>(in, out, ex, table, stream);
    case 2 * 8 + 1: return launch_h<T, 2, 1>(in, out, ex, table, stream);
    case 3 * 8 + 1: return launch_h<T, 3, 1>(in, out, ex, table, stream);
    case 4 * 8 + 1: return launch_h<T, 4, 1>(in, out, ex, table, stream);
    case 1 * 8 + 2: return launch_h<T, 1, 2>(in, out, ex, table, stream);
    case 2 * 8 + 2: return launch_h<T, 2, 2>(in, out, ex, table, stream);
    case 1 * 8 + 3: return launch_h<T, 1, 3>(in, out, ex, table, stream);
    case 1 * 8 + 4: return launch_h<T, 1, 4>(in, out, ex, table, stream);
    case 5 * 8 + 1:
        if constexpr (MAXR >= 5) return launch_h<T, 5, 1>(in, out, ex, table, stream);
        return hipErrorInvalidValue;
    case 1 * 8 + 5:
        if constexpr (MAXR >= 5) return launch_h<T, 1, 5>(in, out, ex, table, stream);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}
}  // namespace

hipError_t launch_exchange(Precision prec, const void *in, void *out, const ExchangeDesc &ex, const void *table,
                           hipStream_t stream)
{
    return prec == Precision::F64 ? launch_r<double, kExchangeRegBitsF64>(in, out, ex, table, stream)
                                  : launch_r<float, kExchangeRegBitsF32>(in, out, ex, table, stream);
}

}  // namespace fftu
