// Internal descriptors shared by the planner (fftu_api.cpp) and the kernels
// (fftu_kernels.hip). Every size in this build is a power of two, so sizes are
// carried as base-2 logarithms and indices are formed with shifts and masks.
#pragma once

#include <cstdint>
#include <vector>

#include "../../include/fftu.h"

namespace fftu {

constexpr int kMaxDims = FFTU_MAX_DIMS;
constexpr int kMaxGroup = 4;     // dimensions transformed by one pass kernel
constexpr int kMaxStages = 12;   // radix stages per dimension inside a pass
constexpr int kMaxLogP = 6;      // largest grid (P = 64) whose length-p FFTs run in registers
constexpr int kPassThreads = 256;
constexpr int kExchangeThreads = 256;
constexpr int kPointwiseThreads = 256;
// Elements per LDS tile of k_pass (the register budget of a stage is sized from it):
// 2^11 complex128 or 2^12 complex64, 32 KiB either way before row padding.
constexpr int kLogTileF64 = 11;
constexpr int kLogTileF32 = 12;

// One pass kernel: 1-D FFTs along a group of consecutive dimensions of an array
// viewed as (A, G, B) row-major, where G is the product of the group's lengths
// and B the product of the lengths after it. A tile holds W = 2^logW columns:
// W consecutive inner indices (B >= W) or W/B consecutive outer blocks (B < W).
struct PassDesc {
    int64_t tiles;         // workgroups launched
    int64_t GB;            // elements per outer block, G * B
    int32_t logB;
    int32_t logG;
    int32_t logW;
    int32_t logBt;         // log2 min(B, W)
    int32_t logTPA;        // log2(B / W) when B >= W (tiles per outer block), else 0
    int32_t lw;            // LDS row pitch in elements (W plus padding)
    int32_t naxes;         // dimensions in the group, outermost first
    int32_t loglen[kMaxGroup];
    int32_t logstride[kMaxGroup];  // stride of each group dimension inside the group (in group positions)
    int32_t nstages[kMaxGroup];
    int32_t lograd[kMaxGroup][kMaxStages];
    int32_t lognmax;       // twiddle table holds omega_{2^lognmax}^j
    int32_t conj_in;       // conjugate on load
    int32_t conj_out;      // conjugate on store
    double scale;          // multiply on store (1.0: none)
    uint32_t lds_bytes;    // dynamic LDS per workgroup
};

// Geometry of the cyclic buffer: d dimensions, n = m * p, m = q * p.
struct GridDesc {
    int64_t M;             // elements per virtual processor
    int64_t N;
    int32_t d;
    int32_t lognmax;
    int32_t logn[kMaxDims];
    int32_t logm[kMaxDims];
    int32_t logp[kMaxDims];
    int32_t logmstride[kMaxDims];  // log2 prod_{j>l} m_j
    int32_t logpstride[kMaxDims];  // log2 prod_{j>l} p_j
    int32_t conj_in;
    int32_t conj_out;
    double scale;
};

// The fused Superstep-1/2 kernel: twiddle, permutation, F_{p_1} x ... x F_{p_d}
// in registers, conjugation and scaling. Bit b of the flat processor index s'
// (row-major over the grid) belongs to dimension bit_dim[b] at bit bit_h[b]
// of s'_l. Register i ends up holding output k' whose offset inside the
// destination block is okp[i] = sum_l bitrev(k'_l) q_l prod_{j>l} m_j.
struct ExchangeDesc {
    GridDesc g;
    int32_t logP;
    int32_t bit_dim[kMaxLogP];
    int32_t bit_h[kMaxLogP];
    int64_t okp[1 << kMaxLogP];
};

enum class Precision { F32, F64 };

// Launchers (fftu_kernels.hip). All return hipSuccess or the launch error.
hipError_t launch_pass(Precision prec, const void *in, void *out, const PassDesc &pd, const void *table,
                       hipStream_t stream);
hipError_t launch_twiddle(Precision prec, const void *in, void *out, const GridDesc &g, const void *table,
                          hipStream_t stream);
hipError_t launch_permute(Precision prec, const void *in, void *out, const GridDesc &g, hipStream_t stream);
hipError_t launch_exchange(Precision prec, const void *in, void *out, const ExchangeDesc &ex, const void *table,
                           hipStream_t stream);

}  // namespace fftu
