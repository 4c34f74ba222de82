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
//   kLineStrided    lines are columns of an (A, L, B) array with B >= W; W lines
//                   of consecutive b per workgroup; lanes run over b first, so each
//                   load or store instruction covers W consecutive elements.
//   kLineContig     contiguous lines (B = 1), W consecutive lines per workgroup;
//                   lanes run along the line, runs of TPL elements.
//   kLineStaged     contiguous lines whose thread runs would be short: the W*L
//                   contiguous elements go through LDS with linear coalesced
//                   loads and stores.
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
template <typename T, int LOGL, int S, int MODE, typename V, typename GET>
__device__ __forceinline__ void line_scatter(const cx<T> (&v)[LinePlan<LOGL>::E], int j, int w, int pitch, V *lds,
                                             GET get)
{
    using PL = LinePlan<LOGL>;
    constexpr int LR = PL::lr(S), R = 1 << LR, LNS = PL::lns(S), NB = PL::E / R;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        const int jj = j + c * PL::TPL;
        const int ob = ((jj >> LNS) << (LNS + LR)) + (jj & ((1 << LNS) - 1));
#pragma unroll
        for (int r = 0; r < R; ++r) lds[lidx<MODE>(ob + (r << LNS), w, pitch)] = get(v[c + r * NB]);
    }
}

template <typename T, int LOGL, int MODE, typename V, typename PUT>
__device__ __forceinline__ void line_gather(cx<T> (&v)[LinePlan<LOGL>::E], int j, int w, int pitch, const V *lds,
                                            PUT put)
{
    using PL = LinePlan<LOGL>;
#pragma unroll
    for (int m = 0; m < PL::E; ++m) put(v[m], lds[lidx<MODE>(j + m * PL::TPL, w, pitch)]);
}

template <typename T, int LOGL, int S, int MODE>
__device__ __forceinline__ void line_exchange(cx<T> (&v)[LinePlan<LOGL>::E], int j, int w, int pitch, void *smem)
{
    if constexpr (sizeof(T) == 8) {
        T *lds = static_cast<T *>(smem);
        line_scatter<T, LOGL, S, MODE>(v, j, w, pitch, lds, [](const cx<T> &a) { return a.x; });
        __syncthreads();
        line_gather<T, LOGL, MODE>(v, j, w, pitch, lds, [](cx<T> &a, T b) { a.x = b; });
        __syncthreads();
        line_scatter<T, LOGL, S, MODE>(v, j, w, pitch, lds, [](const cx<T> &a) { return a.y; });
        __syncthreads();
        line_gather<T, LOGL, MODE>(v, j, w, pitch, lds, [](cx<T> &a, T b) { a.y = b; });
    } else {
        cx<T> *lds = static_cast<cx<T> *>(smem);
        line_scatter<T, LOGL, S, MODE>(v, j, w, pitch, lds, [](const cx<T> &a) { return a; });
        __syncthreads();
        line_gather<T, LOGL, MODE>(v, j, w, pitch, lds, [](cx<T> &a, cx<T> b) { a = b; });
    }
}

template <typename T, int LOGL, int MODE>
__device__ __forceinline__ void line_stages(cx<T> (&v)[LinePlan<LOGL>::E], int j, int w, int pitch, void *smem,
                                            const cx<T> *tw)
{
    using PL = LinePlan<LOGL>;
    line_compute<T, LOGL, 0>(v, j, tw);
    if constexpr (PL::NS > 1) {
        line_exchange<T, LOGL, 0, MODE>(v, j, w, pitch, smem);
        line_compute<T, LOGL, 1>(v, j, tw);
    }
    if constexpr (PL::NS > 2) {
        __syncthreads();
        line_exchange<T, LOGL, 1, MODE>(v, j, w, pitch, smem);
        line_compute<T, LOGL, 2>(v, j, tw);
    }
}

template <typename T, int LOGL, int MODE>
__global__ __launch_bounds__(kLineMaxThreads) void k_line(const cx<T> *in, cx<T> *out, const PassDesc pd,
                                               const cx<T> *__restrict__ table)
{
    using PL = LinePlan<LOGL>;
    extern __shared__ unsigned char smem_raw[];
    cx<T> *tw = reinterpret_cast<cx<T> *>(smem_raw);          // omega_L^e, e in [L]
    cx<T> *lds = tw + PL::L;                                   // W lines
    const int W = 1 << pd.logW;
    const int pitch = pd.lw;
    for (int e = threadIdx.x; e < PL::L; e += blockDim.x) tw[e] = table[e << (pd.lognmax - LOGL)];

    int j, w;
    if constexpr (MODE == kLineStrided) {
        w = threadIdx.x & (W - 1);
        j = threadIdx.x >> pd.logW;
    } else {
        j = threadIdx.x & (PL::TPL - 1);
        w = threadIdx.x >> PL::LOGTPL;
    }
    const T scale = static_cast<T>(pd.scale);

    for (int64_t t = blockIdx.x; t < pd.tiles; t += gridDim.x) {
        __syncthreads();   // twiddle copy done / previous tile's LDS reads done
        cx<T> v[PL::E];
        int64_t base;      // global offset of element 0 of this thread's line
        int64_t xstride;   // global distance between consecutive line elements
        if constexpr (MODE == kLineStrided) {
            const int64_t a = t >> pd.logTPA;
            const int64_t b0 = (t & ((int64_t(1) << pd.logTPA) - 1)) << pd.logW;
            base = a * pd.GB + b0 + w;
            xstride = int64_t(1) << pd.logB;
        } else {
            base = ((t << pd.logW) + w) << LOGL;
            xstride = 1;
        }

        if constexpr (MODE == kLineStaged) {
            const int64_t tbase = (t << pd.logW) << LOGL;
            const int n = W << LOGL;
            for (int e = threadIdx.x; e < n; e += blockDim.x)
                lds[lidx<MODE>(e & (PL::L - 1), e >> LOGL, pitch)] = conj_if(in[tbase + e], pd.conj_in);
            __syncthreads();
            line_gather<T, LOGL, MODE>(v, j, w, pitch, lds, [](cx<T> &a, cx<T> b) { a = b; });
            __syncthreads();
        } else {
#pragma unroll
            for (int m = 0; m < PL::E; ++m) v[m] = conj_if(in[base + int64_t(j + m * PL::TPL) * xstride], pd.conj_in);
        }

        line_stages<T, LOGL, MODE>(v, j, w, pitch, static_cast<void *>(lds), tw);

#pragma unroll
        for (int m = 0; m < PL::E; ++m) {
            v[m] = conj_if(v[m], pd.conj_out);
            if (pd.scale != 1.0) v[m] = {v[m].x * scale, v[m].y * scale};
        }
        if constexpr (MODE == kLineStaged) {
            if constexpr (PL::NS > 1) __syncthreads();
#pragma unroll
            for (int m = 0; m < PL::E; ++m) lds[lidx<MODE>(j + m * PL::TPL, w, pitch)] = v[m];
            __syncthreads();
            const int64_t tbase = (t << pd.logW) << LOGL;
            const int n = W << LOGL;
            for (int e = threadIdx.x; e < n; e += blockDim.x)
                out[tbase + e] = lds[lidx<MODE>(e & (PL::L - 1), e >> LOGL, pitch)];
        } else {
#pragma unroll
            for (int m = 0; m < PL::E; ++m) out[base + int64_t(j + m * PL::TPL) * xstride] = v[m];
        }
    }
}

namespace {
constexpr int64_t kMaxLineBlocks = int64_t(1) << 21;

template <typename T, int LOGL, int MODE>
hipError_t launch_line_t(const void *in, void *out, const PassDesc &pd, const void *table, hipStream_t stream)
{
    const uint32_t blocks = uint32_t(pd.tiles < kMaxLineBlocks ? pd.tiles : kMaxLineBlocks);
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
