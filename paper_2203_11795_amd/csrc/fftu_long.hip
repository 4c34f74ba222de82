// k_long: batched 1-D FFTs of long lines (2^11 or 2^12 points) along a dimension
// whose rows are short (B elements after it), for Superstep 0 (and the unfused
// Superstep 2) of Algorithm 2.3 (arXiv 2203.11795) where no per-thread split of
// k_line fits: a line of 4096 complex64 spans 32 KiB, of 4096 complex128 64 KiB
// (W = 1 line per workgroup, up to B = 8 columns: eight tiles share each line).
//
// A workgroup of 512 threads takes W whole lines (E = 16 complex64 or 8 complex128
// elements per thread, within 128 VGPRs, so two workgroups share a CU and one loads
// or stores while the other computes): W / B whole outer blocks of L rows of B
// columns when B <= W (one contiguous run), or W of the G W columns (G = 2, 4) of one
// outer block. It
//   1. loads the tile linearly (consecutive lanes on consecutive addresses);
//   2. regroups it through LDS so that thread j of line w holds positions
//      j + TPL m, m in [E];
//   3. runs radix-E stages (the last one may be smaller; Stockham autosort,
//      in-register DFTs with exact roots), exchanging through LDS between stages;
//   4. regroups through LDS once more and stores the tile linearly.
// With G tiles per outer block they share every 128-byte line: they run on the same
// XCD at the same time (workgroups go to the 8 XCDs round-robin) and load and store
// with plain (not non-temporal) accesses, so that all but the first read the lines
// from that XCD's L2 and L2 merges the pieces of each line they write.
// LDS holds one word per element (real parts, then imaginary parts), rows of
// L + L/16 + 64/W words per line: one pad word per 16 positions spreads the radix
// scatters over the banks, and the row length spreads the linear accesses. The
// stage twiddles omega_L^e are products of two small LDS tables,
// omega_L^(e mod 64) and omega_L^(64 (e div 64)), 1 KiB per tile: a copy of the
// full table of L entries (32 KiB for 4096 complex64) per tile cost more than the
// extra multiply.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fftu_device.hpp"
#include "fftu_internal.hpp"

namespace fftu {

// E = 2^LOGE elements per thread, stages of radix 2^LOGR (the last one smaller):
// a thread runs E / R butterflies per stage
template <int LOGL, int LOGE, int LOGR>
struct LongPlan {
    static constexpr int L = 1 << LOGL;
    static constexpr int E = 1 << LOGE;
    static constexpr int LOGTPL = LOGL - LOGE;
    static constexpr int TPL = 1 << LOGTPL;
    static constexpr int NS = (LOGL + LOGR - 1) / LOGR;
    static constexpr int lr(int s) { return s < NS - 1 ? LOGR : LOGL - (NS - 1) * LOGR; }
    static constexpr int lns(int s) { return s * LOGR; }
};

// LDS word of position x of tile line w
template <int LOGL, int ESIZE>
__device__ __forceinline__ int long_word(int x, int w)
{
    return w * long_pitch(LOGL, ESIZE) + x + (x >> 4);
}

template <typename T, int LOGL>
__device__ __forceinline__ cx<T> long_root(int e, const cx<T> *lo, const cx<T> *hi)
{
    return cmul(hi[e >> 6], lo[e & 63]);
}

// radix stage S on registers v (register m <-> position j + TPL m)
template <typename T, typename PL, int LOGL, int S>
__device__ __forceinline__ void long_compute(cx<T> (&v)[PL::E], int j, const cx<T> *lo, const cx<T> *hi)
{
    constexpr int LR = PL::lr(S), R = 1 << LR, LNS = PL::lns(S), NB = PL::E / R;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        cx<T> x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = v[c + r * NB];
        if constexpr (S > 0) {
            const int jm = (j + c * PL::TPL) & ((1 << LNS) - 1);
#pragma unroll
            for (int r = 1; r < R; ++r) x[r] = cmul(x[r], long_root<T, LOGL>((r * jm) << (LOGL - LNS - LR), lo, hi));
        }
        Dft<T, R>::run(x);
#pragma unroll
        for (int r = 0; r < R; ++r) v[c + r * NB] = x[r];
    }
}

// stage S's outputs to their Stockham positions, one part (real or imaginary) per round
template <typename T, typename PL, int LOGL, int S, typename GET>
__device__ __forceinline__ void long_scatter(const cx<T> (&v)[PL::E], int j, int w, T *ld, GET part)
{
    constexpr int LR = PL::lr(S), R = 1 << LR, LNS = PL::lns(S), NB = PL::E / R;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        const int jj = j + c * PL::TPL;
        const int ob = ((jj >> LNS) << (LNS + LR)) + (jj & ((1 << LNS) - 1));
#pragma unroll
        for (int r = 0; r < R; ++r) ld[long_word<LOGL, int(sizeof(T) * 2)>(ob + (r << LNS), w)] = part(v[c + r * NB]);
    }
}

template <typename T, typename PL, int LOGL, int S>
__device__ __forceinline__ void long_exchange(cx<T> (&v)[PL::E], int j, int w, T *ld)
{
    long_scatter<T, PL, LOGL, S>(v, j, w, ld, [](const cx<T> &a) { return a.x; });
    __syncthreads();
#pragma unroll
    for (int m = 0; m < PL::E; ++m) v[m].x = ld[long_word<LOGL, int(sizeof(T) * 2)>(j + m * PL::TPL, w)];
    __syncthreads();
    long_scatter<T, PL, LOGL, S>(v, j, w, ld, [](const cx<T> &a) { return a.y; });
    __syncthreads();
#pragma unroll
    for (int m = 0; m < PL::E; ++m) v[m].y = ld[long_word<LOGL, int(sizeof(T) * 2)>(j + m * PL::TPL, w)];
    __syncthreads();
}

template <typename T, int LOGL, int LOGB>
__global__ __launch_bounds__(kLongThreads) void k_long(const cx<T> *in, cx<T> *out, const PassDesc pd,
                                                       const cx<T> *__restrict__ table)
{
    constexpr int NT = kLongThreads;
    constexpr int LOGW = long_logw(LOGL, int(sizeof(T) * 2));
    constexpr int LOGTPL = kLongLogThreads - LOGW;
    static_assert(LOGB <= LOGW + (LOGW == 0 ? 3 : 2), "rows of at most 4 W columns (8 when W = 1)");
    using PL = LongPlan<LOGL, LOGL - LOGTPL, LOGL - LOGTPL>;
    constexpr int E = PL::E, L = PL::L, TPL = PL::TPL;
    static_assert(E * NT == (L << LOGW), "the tile is W whole lines");
    extern __shared__ unsigned char smem_raw[];
    cx<T> *lo = reinterpret_cast<cx<T> *>(smem_raw);   // omega_L^e, e in [64]
    cx<T> *hi = lo + 64;                               // omega_L^(64 i), i in [L / 64]
    T *ld = reinterpret_cast<T *>(hi + L / 64);        // the tile, one part at a time
    const int tid = threadIdx.x;
    for (int e = tid; e < 64 + L / 64; e += NT) {
        const int ex = e < 64 ? e : (e - 64) << 6;
        lo[e] = table[int64_t(ex) << (pd.lognmax - LOGL)];
    }
    const int j = tid & (TPL - 1), w = tid >> LOGTPL;
    constexpr int lb = LOGB;   // compile-time, so that the staged LDS addresses fold into offsets
    // tile index: with B = G W (G = 2, 4, or 8 when W = 1) the G tiles of a block are workgroups
    // v, v + 8, ..., which run on one XCD at the same time (a bijection on each
    // aligned run of 8 G)
    constexpr int LOGG = LOGB > LOGW ? LOGB - LOGW : 0;
    int64_t t = blockIdx.x;
    if constexpr (LOGB > LOGW) {
        const int64_t nb = gridDim.x;
        if ((nb & ((8 << LOGG) - 1)) == 0)
            t = ((((t >> 3) >> LOGG) << 3 | (t & 7)) << LOGG) | ((t >> 3) & ((1 << LOGG) - 1));
    }
    // element e of the tile -> (global offset, LDS word). B <= W: outer block e / (L B),
    // row x, column c, line (block, c). B = G W: row e / W, column (t mod G) W + e mod W
    // of block t / G.
    auto goff = [&](int e) -> int64_t {
        if constexpr (LOGB <= LOGW) {
            return (t << (LOGW + LOGL)) + e;
        } else {
            return ((t >> LOGG) << (LOGL + LOGB)) + (int64_t(e >> LOGW) << LOGB) + ((t & ((1 << LOGG) - 1)) << LOGW) + (e & ((1 << LOGW) - 1));
        }
    };
    auto at = [&](int e) {
        if constexpr (LOGB <= LOGW) {
            const int x = (e >> lb) & (L - 1);
            const int ln = ((e >> (lb + LOGL)) << lb) | (e & ((1 << lb) - 1));
            return long_word<LOGL, int(sizeof(T) * 2)>(x, ln);
        } else {
            return long_word<LOGL, int(sizeof(T) * 2)>(e >> LOGW, e & ((1 << LOGW) - 1));
        }
    };

    cx<T> r[E];
#pragma unroll
    for (int c = 0; c < E; ++c) {
        // G tiles share each line when B = G W: plain loads keep the lines in L2 for the
        // others (non-temporal ones fetched 2.06 times the bytes from HBM with G = 4)
        if constexpr (LOGB > LOGW) {
            r[c] = conj_if(in[goff(tid + c * NT)], pd.conj_in);
        } else {
            r[c] = conj_if(get(&in[goff(tid + c * NT)]), pd.conj_in);
        }
    }
    cx<T> v[E];
#pragma unroll
    for (int c = 0; c < E; ++c) ld[at(tid + c * NT)] = r[c].x;
    __syncthreads();   // also: the twiddle tables are in LDS
#pragma unroll
    for (int m = 0; m < E; ++m) v[m].x = ld[long_word<LOGL, int(sizeof(T) * 2)>(j + m * TPL, w)];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < E; ++c) ld[at(tid + c * NT)] = r[c].y;
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) v[m].y = ld[long_word<LOGL, int(sizeof(T) * 2)>(j + m * TPL, w)];
    __syncthreads();

    long_compute<T, PL, LOGL, 0>(v, j, lo, hi);
    if constexpr (PL::NS > 1) {
        long_exchange<T, PL, LOGL, 0>(v, j, w, ld);
        long_compute<T, PL, LOGL, 1>(v, j, lo, hi);
    }
    if constexpr (PL::NS > 2) {
        long_exchange<T, PL, LOGL, 1>(v, j, w, ld);
        long_compute<T, PL, LOGL, 2>(v, j, lo, hi);
    }
    if constexpr (PL::NS > 3) {
        long_exchange<T, PL, LOGL, 2>(v, j, w, ld);
        long_compute<T, PL, LOGL, 3>(v, j, lo, hi);
    }
    static_assert(PL::NS <= 4, "at most four radix stages");

    // after the last stage register m holds position j + TPL m again
    const T scale = static_cast<T>(pd.scale);
#pragma unroll
    for (int m = 0; m < E; ++m) {
        v[m] = conj_if(v[m], pd.conj_out);
        if (pd.scale != 1.0) v[m] = {v[m].x * scale, v[m].y * scale};
    }
#pragma unroll
    for (int m = 0; m < E; ++m) ld[long_word<LOGL, int(sizeof(T) * 2)>(j + m * TPL, w)] = v[m].x;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < E; ++c) r[c].x = ld[at(tid + c * NT)];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) ld[long_word<LOGL, int(sizeof(T) * 2)>(j + m * TPL, w)] = v[m].y;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < E; ++c) {
        r[c].y = ld[at(tid + c * NT)];
        // G tiles share each line when B = G W: plain stores let L2 merge the pieces
        // (non-temporal ones wrote 1.35 times the bytes to HBM with G = 2)
        if constexpr (LOGB > LOGW) {
            out[goff(tid + c * NT)] = r[c];
        } else {
            put<false>(&out[goff(tid + c * NT)], r[c]);
        }
    }
}

namespace {

template <typename T, int LOGL, int LOGB>
hipError_t launch_long_t(const void *in, void *out, const PassDesc &pd, const void *table, hipStream_t stream)
{
    if (pd.logW != long_logw(LOGL, int(sizeof(T) * 2)) || pd.logB != LOGB || pd.threads != kLongThreads || pd.tiles < 1 ||
        pd.tiles > kLongMaxTiles || pd.lds_bytes != long_lds_bytes(LOGL, int(sizeof(T) * 2)) || pd.lognmax < LOGL)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_long<T, LOGL, LOGB>), dim3(uint32_t(pd.tiles)), dim3(kLongThreads), pd.lds_bytes, stream,
                       static_cast<const cx<T> *>(in), static_cast<cx<T> *>(out), pd,
                       static_cast<const cx<T> *>(table));
    return hipGetLastError();
}

template <typename T, int LOGL, int LOGB = 0>
hipError_t launch_long_b(const void *in, void *out, const PassDesc &pd, const void *table, hipStream_t stream)
{
    if (pd.logB == LOGB) return launch_long_t<T, LOGL, LOGB>(in, out, pd, table, stream);
    constexpr int logw = long_logw(LOGL, int(sizeof(T) * 2));
    if constexpr (LOGB < logw + (logw == 0 ? 3 : 2))
        return launch_long_b<T, LOGL, LOGB + 1>(in, out, pd, table, stream);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_long(Precision prec, const void *in, void *out, const PassDesc &pd, const void *table,
                       hipStream_t stream)
{
    if (pd.kind != kLong || pd.naxes != 1) return hipErrorInvalidValue;
    const int logL = pd.loglen[0];
    if (prec == Precision::F64) {
        if (logL == 12) return launch_long_b<double, 12>(in, out, pd, table, stream);
        if (logL == 11) return launch_long_b<double, 11>(in, out, pd, table, stream);
    } else {
        if (logL == 12) return launch_long_b<float, 12>(in, out, pd, table, stream);
        if (logL == 11) return launch_long_b<float, 11>(in, out, pd, table, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace fftu
