// k_line: batched 1-D FFTs of length L = 2^LOGL along one axis, register-direct.
//
// Superstep 0 of Algorithm 2.3 (arXiv 2203.11795) transforms every local array
// along each dimension; for a single dimension per pass this kernel replaces the
// generic LDS-tile pass. A line is split over TPL = L / E threads, each holding E
// elements in registers: thread j owns positions j + TPL*m, m in [E], of its line
// both before the first and after the last radix stage, so it loads them from HBM
// and stores them back without passing through LDS. Between radix stages the
// line goes through LDS once (Stockham autosort: stage s with radix R after
// Ns = R_0...R_{s-1} reads jj + r L/R and writes (jj div Ns) Ns R + jj mod Ns + r Ns,
// with the twiddle omega_{Ns R}^{r (jj mod Ns)} read from an LDS copy of omega_L).
//
// Layouts:
//   kLineStrided    lines are columns of an (A, L, B) array: W consecutive lines
//                   of the A*B (a, b) lines per workgroup (W > B spans several
//                   outer blocks); lanes run over b first, so each load or store
//                   instruction covers runs of min(W, B) consecutive elements.
//   kLineContig     contiguous lines (B = 1), W consecutive lines per workgroup;
//                   lanes run along the line, runs of TPL elements.
//   kLineStaged     a tile of W >= B lines that is one contiguous run of W*L
//                   elements (contiguous lines whose thread runs would be short,
//                   or columns of short rows): it goes through LDS with linear
//                   coalesced loads and stores.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fftu_line.hpp"

namespace fftu {

template <typename T, int LOGL, int MODE>
__global__ __launch_bounds__(kLineMaxThreads) void k_line(const cx<T> *in, cx<T> *out, const PassDesc pd,
                                                          const cx<T> *__restrict__ table)
{
    using PL = LinePlan<LOGL>;
    extern __shared__ unsigned char smem_raw[];
    cx<T> *tw = reinterpret_cast<cx<T> *>(smem_raw);   // omega_L^e, e in [L]
    cx<T> *lds = tw + PL::L;                            // the tile
    // grid size in a scalar register, read before any divergent code: the tile loop
    // holds barriers and must be wave-uniform
    const int64_t nblocks = __builtin_amdgcn_readfirstlane(int(gridDim.x));
    line_twiddles<T, LOGL>(tw, table, pd.lognmax, threadIdx.x);
    for (int64_t t = blockIdx.x; t < pd.tiles; t += nblocks) {
        __syncthreads();   // twiddle copy done / previous tile's LDS reads done
        line_tile<T, LOGL, MODE>(in, out, pd, tw, lds, t, threadIdx.x);
    }
}

// k_line with the loaded elements negated by the parity of their index bits under
// pd.sign_mask: the first pass of a transform whose input is a signed copy of the
// buffer (the DST-II's signal), without a pass of its own for the signs.
template <typename T, int LOGL, int MODE>
__global__ __launch_bounds__(kLineMaxThreads) void k_line_sign(const cx<T> *in, cx<T> *out, const PassDesc pd,
                                                               const cx<T> *__restrict__ table)
{
    using PL = LinePlan<LOGL>;
    extern __shared__ unsigned char smem_raw[];
    cx<T> *tw = reinterpret_cast<cx<T> *>(smem_raw);
    cx<T> *lds = tw + PL::L;
    const int64_t nblocks = __builtin_amdgcn_readfirstlane(int(gridDim.x));
    line_twiddles<T, LOGL>(tw, table, pd.lognmax, threadIdx.x);
    for (int64_t t = blockIdx.x; t < pd.tiles; t += nblocks) {
        __syncthreads();
        line_tile<T, LOGL, MODE, false, true>(in, out, pd, tw, lds, t, threadIdx.x);
    }
}

namespace {
constexpr int64_t kMaxLineBlocks = int64_t(1) << 21;

template <typename T, int LOGL, int MODE>
hipError_t launch_line_t(const void *in, void *out, const PassDesc &pd, const void *table, hipStream_t stream)
{
    const uint32_t blocks = uint32_t(pd.tiles < kMaxLineBlocks ? pd.tiles : kMaxLineBlocks);
    if (pd.sign_mask != 0)
        hipLaunchKernelGGL((k_line_sign<T, LOGL, MODE>), dim3(blocks), dim3(uint32_t(pd.threads)), pd.lds_bytes, stream,
                           static_cast<const cx<T> *>(in), static_cast<cx<T> *>(out), pd,
                           static_cast<const cx<T> *>(table));
    else
        hipLaunchKernelGGL((k_line<T, LOGL, MODE>), dim3(blocks), dim3(uint32_t(pd.threads)), pd.lds_bytes, stream,
                           static_cast<const cx<T> *>(in), static_cast<cx<T> *>(out), pd,
                           static_cast<const cx<T> *>(table));
    return hipGetLastError();
}

template <typename T, int MODE>
hipError_t launch_line_mode(const void *in, void *out, const PassDesc &pd, const void *table, hipStream_t stream)
{
    switch (pd.loglen[0]) {
    case 1: return launch_line_t<T, 1, MODE>(in, out, pd, table, stream);
    case 2: return launch_line_t<T, 2, MODE>(in, out, pd, table, stream);
    case 3: return launch_line_t<T, 3, MODE>(in, out, pd, table, stream);
    case 4: return launch_line_t<T, 4, MODE>(in, out, pd, table, stream);
    case 5: return launch_line_t<T, 5, MODE>(in, out, pd, table, stream);
    case 6: return launch_line_t<T, 6, MODE>(in, out, pd, table, stream);
    case 7: return launch_line_t<T, 7, MODE>(in, out, pd, table, stream);
    case 8: return launch_line_t<T, 8, MODE>(in, out, pd, table, stream);
    case 9: return launch_line_t<T, 9, MODE>(in, out, pd, table, stream);
    case 10: return launch_line_t<T, 10, MODE>(in, out, pd, table, stream);
    case 11: return launch_line_t<T, 11, MODE>(in, out, pd, table, stream);
    case 12: return launch_line_t<T, 12, MODE>(in, out, pd, table, stream);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_line_prec(const void *in, void *out, const PassDesc &pd, const void *table, hipStream_t stream)
{
    switch (pd.kind) {
    case kLineStrided: return launch_line_mode<T, kLineStrided>(in, out, pd, table, stream);
    case kLineContig: return launch_line_mode<T, kLineContig>(in, out, pd, table, stream);
    case kLineStaged: return launch_line_mode<T, kLineStaged>(in, out, pd, table, stream);
    default: return hipErrorInvalidValue;
    }
}
}  // namespace

hipError_t launch_line(Precision prec, const void *in, void *out, const PassDesc &pd, const void *table,
                       hipStream_t stream)
{
    return prec == Precision::F64 ? launch_line_prec<double>(in, out, pd, table, stream)
                                  : launch_line_prec<float>(in, out, pd, table, stream);
}

}  // namespace fftu
