// Persistent batch kernel: many independent transforms of uneven shapes (each
// Algorithm 2.3 of arXiv 2203.11795 on its own grid) in one launch.
//
// The batch is a list of stage descriptors, one per (stage, transform), in
// stage-major order: every transform's first Superstep-0 pass, then every
// second pass, ..., then every exchange. Each descriptor owns a contiguous range
// of work items (tiles of a k_line or k_group2 pass, or groups of the fused
// exchange).
// Workgroups take items (runs of about 2^17 elements' worth of tiles) from one
// global counter in that order. Before an item of a descriptor with a dependency
// (the previous stage of the same transform) runs, its workgroup waits until
// every item of that dependency has finished; because items are handed out in
// stage-major order, every dependency is already held by a running workgroup,
// so the wait always ends. The wait is bounded all the same (wait_limit ticks of
// the real-time clock, or at once when another wait has given up): then the
// workgroup records an error flag and skips the item, so every workgroup
// reaches the end.
//
// Completion protocol: a stage's results are stored device-coherently (relaxed
// device-scope atomic stores, written through to the level all XCDs read from);
// each thread waits for its stores to complete, then (after a barrier) thread 0
// increments the descriptor's counter before it takes the next item. A waiting
// workgroup polls the counter with relaxed device-scope loads (no cache
// invalidation per poll) and, once it is complete, every thread issues one
// device-scope acquire fence (which drops stale lines from its L2) before
// reading the data.
// Counters are cleared by k_batch_reset (a kernel, so the pair can be captured
// in a graph and replayed). The caller's buffers are read from a device array
// that k_batch_bind writes on the same stream before the batch, so a change of
// buffers never waits for the host and a graph replays with its own.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fftu_exchange.hpp"
#include "fftu_group.hpp"
#include "fftu_line.hpp"

namespace fftu {

__global__ void k_batch_reset(BatchDesc bd)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < bd.nstages; i += gridDim.x * blockDim.x) bd.done[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *bd.next = 0;
        *bd.error = 0;
    }
}

__global__ void k_batch_bind(BatchBind *bind, const BindChunk c)
{
    const int i = threadIdx.x;
    if (i < c.count) bind[c.first + i] = c.b[i];
}

// Values every lane of a wave holds alike, moved to scalar registers. The
// persistent loop below decides its branches and loop bounds only on such values:
// the compiler then keeps its control flow wave-uniform, so every thread of the
// workgroup executes the same sequence of barriers. (Decided on per-lane copies
// read from LDS, the loop was restructured so that thread 0 left it after each
// item while the other lanes went straight back to the first barrier, and the
// workgroup repeated one item forever.)
__device__ __forceinline__ int uniform32(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v))));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(uint64_t(v) >> 32))));
    return int64_t((uint64_t(hi) << 32) | lo);
}

// Tiles [first, last) of a k_line pass; the block's twiddles are loaded once.
// key = log2(line length) * 8 + pass kind, uniform.
template <typename T>
__device__ __forceinline__ void run_line(const BatchStage &st, const void *src, void *dst, int key,
                                         const cx<T> *__restrict__ table, cx<T> *tw, cx<T> *tile, int64_t first,
                                         int64_t last, int tid)
{
    const cx<T> *in = static_cast<const cx<T> *>(src);
    cx<T> *out = static_cast<cx<T> *>(dst);
    const PassDesc &pd = st.pd;
#define FFTU_LINE_CASE(LG, MD)                                                    \
    case (LG) * 8 + (MD):                                                         \
        line_twiddles<T, LG>(tw, table, pd.lognmax, tid);                         \
        for (int64_t t = first; t < last; ++t) {                                  \
            __syncthreads(); /* twiddles in; previous tile's LDS reads done */    \
            line_tile<T, LG, MD, true>(in, out, pd, tw, tile, t, tid);            \
        }                                                                         \
        break;
#define FFTU_LINE_MODES(LG) FFTU_LINE_CASE(LG, kLineStrided) FFTU_LINE_CASE(LG, kLineContig) FFTU_LINE_CASE(LG, kLineStaged)
    switch (key) {
        FFTU_LINE_MODES(1)
        FFTU_LINE_MODES(2)
        FFTU_LINE_MODES(3)
        FFTU_LINE_MODES(4)
        FFTU_LINE_MODES(5)
        FFTU_LINE_MODES(6)
        FFTU_LINE_MODES(7)
        FFTU_LINE_MODES(8)
    default: break;
    }
#undef FFTU_LINE_MODES
#undef FFTU_LINE_CASE
}

// Tiles [first, last) of a k_group2 pass (both innermost dimensions, whole planes)
// with L1 = 2^A, L2 = 2^B; tw takes omega_L1 then omega_L2. A function of its own
// (not inlined) for each plane shape: inlined, the 25 shapes raised the register
// use of the whole persistent kernel.
template <typename T, int A, int B>
__device__ __noinline__ void group2_item(const BatchStage &st, const void *src, void *dst,
                                         const cx<T> *__restrict__ table, cx<T> *tw, cx<T> *tile, int64_t first,
                                         int64_t last, int tid)
{
    const cx<T> *in = static_cast<const cx<T> *>(src);
    cx<T> *out = static_cast<cx<T> *>(dst);
    const PassDesc &pd = st.pd;
    // arguments arrive in vector registers: the tile loop (which holds barriers)
    // runs on scalar copies
    const int64_t t0 = uniform64(first), t1 = uniform64(last);
    for (int e = tid; e < (1 << A); e += kBatchThreads) tw[e] = table[e << (pd.lognmax - A)];
    for (int e = tid; e < (1 << B); e += kBatchThreads) tw[(1 << A) + e] = table[e << (pd.lognmax - B)];
    for (int64_t t = t0; t < t1; ++t) {
        __syncthreads();
        group2_tile<T, A, B, true>(in, out, pd, tw, tw + (1 << A), tile, t, tid, kBatchThreads);
    }
}

// key = log2(L1) * 8 + log2(L2), uniform.
template <typename T>
__device__ __forceinline__ void run_group2(const BatchStage &st, const void *src, void *dst, int key,
                                           const cx<T> *__restrict__ table, cx<T> *tw, cx<T> *tile, int64_t first,
                                           int64_t last, int tid)
{
#define FFTU_G2_CASE(A, B) \
    case (A) * 8 + (B): group2_item<T, A, B>(st, src, dst, table, tw, tile, first, last, tid); break;
#define FFTU_G2_ROW(A) FFTU_G2_CASE(A, 2) FFTU_G2_CASE(A, 3) FFTU_G2_CASE(A, 4) FFTU_G2_CASE(A, 5) FFTU_G2_CASE(A, 6)
    switch (key) {
        FFTU_G2_ROW(2)
        FFTU_G2_ROW(3)
        FFTU_G2_ROW(4)
        FFTU_G2_ROW(5)
        FFTU_G2_ROW(6)
    default: break;
    }
#undef FFTU_G2_ROW
#undef FFTU_G2_CASE
}

// Tiles [first, last) of the fused exchange; a tile is 4 groups of 64 local
// indices (no wave dimensions in a batch, so no LDS is shared between tiles).
// key = register dimensions * 8 + log2(their radix), uniform.
template <typename T>
__device__ __forceinline__ void run_exchange(const BatchStage &st, const void *src, void *dst, int key,
                                             const cx<T> *__restrict__ table, unsigned char *smem, int64_t first,
                                             int64_t last, int tid)
{
    const cx<T> *Z = static_cast<const cx<T> *>(src);
    cx<T> *V = static_cast<cx<T> *>(dst);
    const ExchangeDesc &ex = st.ex;
#define FFTU_EX_CASE(NR, LPR)                                                     \
    case (NR) * 8 + (LPR):                                                        \
        for (int64_t t = first; t < last; ++t)                                    \
            exchange_group<T, NR, LPR, 0, 0, true>(Z, V, ex, table, smem, t * (kExchangeThreads / 64), tid); \
        break;
    switch (key) {
        FFTU_EX_CASE(0, 0)
        FFTU_EX_CASE(1, 1)
        FFTU_EX_CASE(2, 1)
        FFTU_EX_CASE(3, 1)
        FFTU_EX_CASE(4, 1)
        FFTU_EX_CASE(1, 2)
        FFTU_EX_CASE(2, 2)
        FFTU_EX_CASE(1, 3)
        FFTU_EX_CASE(1, 4)
    default: break;
    }
#undef FFTU_EX_CASE
}

template <typename T>
// complex64: at least 4 waves per SIMD (128 VGPRs: 8 spill to scratch, measured 3.93 -> 3.65 ms on
// the 256-transform batch; 139 VGPRs unconstrained give 3 waves); complex128 unconstrained
__global__ __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) void k_batch(
    const BatchDesc bd, const cx<T> *__restrict__ table)
{
    extern __shared__ unsigned char smem_raw[];
    __shared__ int64_t s_item;
    __shared__ int s_k;
    __shared__ int s_skip;
    cx<T> *tw = reinterpret_cast<cx<T> *>(smem_raw);       // omega_L, L <= kBatchMaxLine
    cx<T> *tile = tw + kBatchMaxLine;
    const int tid = threadIdx.x;
    int prev = -1;   // descriptor of the item this workgroup finished last (uniform)
    for (;;) {
        // The previous item's results were stored device-coherently (written through
        // to the level every XCD reads from): each thread waits until its stores have
        // completed, and after the barrier thread 0 counts the item. This orders the
        // data before the count without a write-back of the L2 (a device-scope
        // release fence), which cost about a third of the batch time.
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (tid == 0) {
            if (prev >= 0) __hip_atomic_fetch_add(&bd.done[prev], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int64_t item = int64_t(atomicAdd(bd.next, 1ull));
            int k = -1, skip = 0;
            if (item < bd.nitems) {
                // descriptor k owns items [starts[k], starts[k + 1])
                int lo = 0, hi = bd.nstages - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (bd.starts[mid] <= item) lo = mid;
                    else hi = mid - 1;
                }
                k = lo;
                const int dep = bd.dep[k];
                if (dep >= 0) {
                    const int need = int(bd.starts[dep + 1] - bd.starts[dep]);
                    const uint64_t t0 = wall_clock64();
                    while (__hip_atomic_load(&bd.done[dep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                        // give up past the time limit, or at once when another wait has given up
                        if (int64_t(wall_clock64() - t0) > bd.wait_limit ||
                            __hip_atomic_load(bd.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                            atomicExch(bd.error, 1);
                            skip = 1;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(8);
                    }
                }
            }
            s_item = item;
            s_k = k;
            s_skip = skip;
        }
        __syncthreads();
        const int64_t item = uniform64(s_item);
        if (item >= bd.nitems) break;
        const int k = uniform32(s_k);
        const int skip = uniform32(s_skip);
        prev = k;
        if (uniform32(bd.dep[k]) >= 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (skip) continue;
        const BatchStage &st = bd.stages[k];
        const int kind = uniform32(st.kind);
        const int64_t per = uniform32(st.per_item);
        const int64_t tiles = uniform64(st.tiles);
        const int64_t first = (item - uniform64(bd.starts[k])) * per;
        const int64_t last = first + per < tiles ? first + per : tiles;
        const int io = uniform32(st.io);
        const int mem = uniform32(st.member);
        const void *src = reinterpret_cast<const void *>(
            uniform64(int64_t(reinterpret_cast<uintptr_t>((io & 1) ? bd.bind[mem].in : st.src))));
        void *dst = reinterpret_cast<void *>(
            uniform64(int64_t(reinterpret_cast<uintptr_t>((io & 2) ? bd.bind[mem].out : st.dst))));
        if (kind == kExchangeStage)
            run_exchange<T>(st, src, dst, uniform32(st.ex.nr * 8 + st.ex.lpr), table,
                            smem_raw + kBatchMaxLine * sizeof(cx<T>), first, last, tid);
        else if (kind == kGroup2)
            run_group2<T>(st, src, dst, uniform32(st.pd.loglen[0] * 8 + st.pd.loglen[1]), table, tw, tile, first,
                          last, tid);
        else
            run_line<T>(st, src, dst, uniform32(st.pd.loglen[0] * 8 + kind), table, tw, tile, first, last, tid);
    }
}

int batch_blocks_per_cu(Precision prec, uint32_t lds_bytes)
{
    int nb = 0;
    hipError_t e = prec == Precision::F64
                       ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<double>, kBatchThreads, lds_bytes)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<float>, kBatchThreads, lds_bytes);
    return e == hipSuccess && nb > 0 ? nb : 1;
}

hipError_t launch_batch_reset(const BatchDesc &bd, hipStream_t stream)
{
    hipLaunchKernelGGL(k_batch_reset, dim3(uint32_t((bd.nstages + 255) / 256 + 1)), dim3(256), 0, stream, bd);
    return hipGetLastError();
}

hipError_t launch_batch_bind(BatchBind *bind, const BindChunk &c, hipStream_t stream)
{
    hipLaunchKernelGGL(k_batch_bind, dim3(1), dim3(kBindChunk), 0, stream, bind, c);
    return hipGetLastError();
}

hipError_t launch_batch(Precision prec, const BatchDesc &bd, const void *table, uint32_t blocks, uint32_t lds_bytes,
                        hipStream_t stream)
{
    if (prec == Precision::F64)
        hipLaunchKernelGGL(k_batch<double>, dim3(blocks), dim3(kBatchThreads), lds_bytes, stream, bd,
                           static_cast<const cx<double> *>(table));
    else
        hipLaunchKernelGGL(k_batch<float>, dim3(blocks), dim3(kBatchThreads), lds_bytes, stream, bd,
                           static_cast<const cx<float> *>(table));
    return hipGetLastError();
}

}  // namespace fftu
