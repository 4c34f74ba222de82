// k_pair: Superstep 0 of Algorithm 2.3 (arXiv 2203.11795) along two adjacent
// dimensions in one pass over HBM, for lines of 8, 16 or 32 points. The local
// d-D FFT factorises over dimensions (eq. (1.3)), so two of its 1-D passes can
// share one read and one write of the array.
//
// The array is viewed as (A, LA, LB, B) row-major: lines of LA points along the
// outer dimension of the pair (stride LB B) and of LB points along the inner one
// (stride B). A workgroup of NT threads takes one tile: one outer index a and
// W = NT / max(LA, LB) consecutive columns c of B, i.e. LA LB W elements. NT is
// 256 for complex128 and 512 for complex64, or 1024 where a line of 32 has rows
// 64 KiB or more apart: the tile's 1024 rows then span many pages, and twice
// the columns per tile halve the pages and DRAM rows opened per byte (one
// workgroup per CU then, so nearby rows keep 512 threads and two per CU).
//   1. Thread (x, w), x < LA, loads the whole inner line (a, x, :, c0 + w) into
//      registers (lanes run over w, so every load instruction covers runs of W
//      consecutive elements) and transforms it with the in-register DFT, whose
//      roots are exact compile-time constants: no table is read.
//   2. An LDS transpose (real parts, then imaginary parts, so a tile needs one
//      word per element) hands thread (y, w), y < LB, the outer line (a, :, y, w).
//   3. That line is transformed in registers and stored, again in runs of W.
// Each element is read from and written to HBM once, and goes through LDS once.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fftu_device.hpp"
#include "fftu_internal.hpp"

namespace fftu {

template <typename T, int LOGLA, int LOGLB, int LOGNT>
__global__ __launch_bounds__(1 << LOGNT) void k_pair(const cx<T> *in, cx<T> *out, const PassDesc pd)
{
    constexpr int LA = 1 << LOGLA, LB = 1 << LOGLB;
    constexpr int LMAX = LA > LB ? LA : LB;
    constexpr int LOGW = pair_logw(LOGLA, LOGLB, LOGNT);
    constexpr int W = 1 << LOGW;
    constexpr int PITCH = pair_pitch(LOGLA, LOGLB, LOGNT);   // words per inner position
    static_assert(LMAX * W == (1 << LOGNT), "one line per thread in the larger phase");
    extern __shared__ unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);

    const int tid = threadIdx.x;
    const int w = tid & (W - 1), x = tid >> LOGW;
    const int64_t t = blockIdx.x;
    const int64_t B = int64_t(1) << pd.logB;
    // element (a, 0, 0, c0 + w) of this tile
    const int64_t base = (t >> pd.logTPA) * pd.GB + ((t & ((int64_t(1) << pd.logTPA) - 1)) << LOGW) + w;

    cx<T> v[LMAX];
    // 1. inner lines: thread (x, w) holds positions b of line (a, x, :, c0 + w)
    if (x < LA) {
        const cx<T> *src = in + base + int64_t(x) * (B << LOGLB);
#pragma unroll
        for (int b = 0; b < LB; ++b) v[b] = conj_if(get(src + int64_t(b) * B), pd.conj_in);
        Dft<T, LB>::run(v);
    }
    // 2. transpose through LDS: word (b, x, w) at b PITCH + x W + w
    cx<T> u[LMAX];
    if (x < LA) {
#pragma unroll
        for (int b = 0; b < LB; ++b) lds[b * PITCH + x * W + w] = v[b].x;
    }
    __syncthreads();
    if (x < LB) {
#pragma unroll
        for (int a = 0; a < LA; ++a) u[a].x = lds[x * PITCH + a * W + w];
    }
    __syncthreads();
    if (x < LA) {
#pragma unroll
        for (int b = 0; b < LB; ++b) lds[b * PITCH + x * W + w] = v[b].y;
    }
    __syncthreads();
    // 3. outer lines: thread (y = x, w) holds positions a of line (a, :, y, c0 + w)
    if (x < LB) {
#pragma unroll
        for (int a = 0; a < LA; ++a) u[a].y = lds[x * PITCH + a * W + w];
        Dft<T, LA>::run(u);
        const T scale = static_cast<T>(pd.scale);
        cx<T> *dst = out + base + int64_t(x) * B;
#pragma unroll
        for (int a = 0; a < LA; ++a) {
            cx<T> r = conj_if(u[a], pd.conj_out);
            if (pd.scale != 1.0) r = {r.x * scale, r.y * scale};
            put<false>(dst + int64_t(a) * (B << LOGLB), r);
        }
    }
}

namespace {

template <typename T, int LOGLA, int LOGLB, int LOGNT>
hipError_t launch_pair_t(const void *in, void *out, const PassDesc &pd, hipStream_t stream)
{
    const int esize = int(sizeof(T) * 2);
    if (pd.logW != pair_logw(LOGLA, LOGLB, LOGNT) || pd.tiles < 1 || pd.tiles > pair_max_tiles(LOGNT) ||
        pd.logB < pd.logW || pd.logTPA != pd.logB - pd.logW || pd.GB != (int64_t(1) << (LOGLA + LOGLB + pd.logB)) ||
        pd.lds_bytes != pair_lds_bytes(LOGLA, LOGLB, LOGNT, esize))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_pair<T, LOGLA, LOGLB, LOGNT>), dim3(uint32_t(pd.tiles)), dim3(uint32_t(pd.threads)),
                       pd.lds_bytes, stream, static_cast<const cx<T> *>(in), static_cast<cx<T> *>(out), pd);
    return hipGetLastError();
}

// the thread count is the planner's (pair_lognt); only its instantiations exist
template <typename T, int LOGLA, int LOGLB>
hipError_t launch_pair_nt(const void *in, void *out, const PassDesc &pd, hipStream_t stream)
{
    if constexpr (sizeof(T) == 8) {
        if (pd.threads == 256) return launch_pair_t<T, LOGLA, LOGLB, 8>(in, out, pd, stream);
    } else {
        if (pd.threads == 512) return launch_pair_t<T, LOGLA, LOGLB, 9>(in, out, pd, stream);
        if constexpr (LOGLA == 5 || LOGLB == 5)
            if (pd.threads == 1024) return launch_pair_t<T, LOGLA, LOGLB, 10>(in, out, pd, stream);
    }
    return hipErrorInvalidValue;
}

template <typename T, int LOGLA>
hipError_t launch_pair_b(const void *in, void *out, const PassDesc &pd, hipStream_t stream)
{
    switch (pd.loglen[1]) {
    case 3: return launch_pair_nt<T, LOGLA, 3>(in, out, pd, stream);
    case 4: return launch_pair_nt<T, LOGLA, 4>(in, out, pd, stream);
    case 5: return launch_pair_nt<T, LOGLA, 5>(in, out, pd, stream);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_pair_prec(const void *in, void *out, const PassDesc &pd, hipStream_t stream)
{
    switch (pd.loglen[0]) {
    case 3: return launch_pair_b<T, 3>(in, out, pd, stream);
    case 4: return launch_pair_b<T, 4>(in, out, pd, stream);
    case 5: return launch_pair_b<T, 5>(in, out, pd, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_pair(Precision prec, const void *in, void *out, const PassDesc &pd, hipStream_t stream)
{
    if (pd.kind != kPair || pd.naxes != 2) return hipErrorInvalidValue;
    return prec == Precision::F64 ? launch_pair_prec<double>(in, out, pd, stream)
                                  : launch_pair_prec<float>(in, out, pd, stream);
}

}  // namespace fftu
