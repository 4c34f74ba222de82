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
constexpr int kMaxLogP = 7;      // largest grid (P = 128) of the fused exchange kernel
constexpr int kExchangeRegBitsF64 = 4;   // complex128 values per thread in the exchange: 16
constexpr int kExchangeRegBitsF32 = 5;   // complex64: 32
constexpr int kExchangeMaxWaveBits = 2;  // at most 4 waves share one group of 64 local indices
constexpr int kPassThreads = 256;
constexpr int kExchangeThreads = 256;
constexpr int kPointwiseThreads = 256;
// Elements per LDS tile of k_pass (the register budget of a stage is sized from it):
// 2^11 complex128 or 2^12 complex64, 32 KiB either way before row padding.
constexpr int kLogTileF64 = 11;
constexpr int kLogTileF32 = 12;

// Pass kernels. kTilePass: generic LDS tile over a group of dimensions (k_pass).
// The others are k_line layouts for a single dimension (see fftu_line.hip).
constexpr int kTilePass = 0;
constexpr int kLineStrided = 1;
constexpr int kLineContig = 2;
constexpr int kLineStaged = 3;
constexpr int kGroup2 = 4;             // k_group2: two innermost dimensions of small contiguous planes
constexpr int kPair = 5;               // k_pair: two adjacent strided dimensions of short lines (fftu_pair.hip)
constexpr int kLong = 6;               // k_long: lines of 2^11 / 2^12 over short rows (fftu_long.hip)
constexpr int kLineMaxThreads = 256;   // k_line workgroup bound (register budget per thread)

// Radix split of k_line for a line of 2^logl: 1, 2 or 3 stages of 2^line_loge
// elements per thread (the last stage may be smaller). Shared by host and device.
constexpr int line_stages_of(int logl) { return logl <= 4 ? 1 : (logl <= 8 ? 2 : 3); }
constexpr int line_loge(int logl) { return (logl + line_stages_of(logl) - 1) / line_stages_of(logl); }

// One pass kernel: 1-D FFTs along a group of consecutive dimensions of an array
// viewed as (A, G, B) row-major, where G is the product of the group's lengths
// and B the product of the lengths after it. A tile holds W = 2^logW columns:
// W consecutive inner indices (B >= W) or W/B consecutive outer blocks (B < W).
struct PassDesc {
    int32_t kind;          // kTilePass or a k_line layout
    int32_t threads;       // workgroup size
    int64_t tiles;         // tiles (workgroups, or grid-stride iterations)
    int64_t GB;            // elements per outer block, G * B
    int32_t logB;
    int32_t logG;
    int32_t logW;
    int32_t logBt;         // log2 min(B, W)
    int32_t logTPA;        // log2(B / W) when B >= W (tiles per outer block), else 0 (generic tile pass only)
    int32_t lw;            // LDS pitch in elements (tile: row of W plus padding; k_line: see fftu_line.hip)
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
    // k_line_sign: the element at buffer index i is negated on load when i & sign_mask
    // has an odd number of bits (0: no signs; only that kernel reads it)
    uint64_t sign_mask = 0;
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

// The fused kernel for Superstep 0's twiddle, Superstep 1 and Superstep 2. The grid
// dimensions with p_l > 1 split into nh leading "wave" dimensions of 2^lph each
// (joined through LDS across waves) and nr trailing "register" dimensions of
// 2^lpr each (held by one thread): hdim[] and rdim[] list their indices.
// oshift[l] = log2(q_l prod_{j>l} m_j), the move of output digit k'_l.
struct ExchangeDesc {
    GridDesc g;
    int32_t nr, lpr, nh, lph;
    int32_t rdim[kMaxDims];
    int32_t hdim[kMaxDims];
    int32_t oshift[kMaxDims];
    uint32_t lds_bytes;
    const void *mul;       // null, or N elements in the output layout that every output is multiplied by
    // k_exchange_sign: the output at buffer index i is negated when i & sign_mask has an
    // odd number of bits (0: no signs; only that kernel reads it)
    uint64_t sign_mask = 0;
};

// k_pair (fftu_pair.hip): lines of 2^3..2^5 points along two adjacent dimensions,
// one whole line per thread. 2^lognt threads: 256 (complex128) or 512 (complex64),
// or 1024 for complex64 lines of 32 whose rows lie 64 KiB or more apart (then the
// tile's W = 32 columns halve the pages and DRAM rows opened per byte). A tile is
// W = threads / max(LA, LB) columns, W * esize = 128 bytes or more.
constexpr int kPairMinLogL = 3;
constexpr int kPairMaxLogL = 5;
constexpr int pair_lognt(int logla, int loglb, int logb, int esize)
{
    return esize == 16 ? 8 : ((logla == 5 || loglb == 5) && logb + 3 >= 16 ? 10 : 9);
}
constexpr int pair_logw(int logla, int loglb, int lognt) { return lognt - (logla > loglb ? logla : loglb); }
// words (one real part) per inner position of the LDS transpose: LA W plus W of
// padding, so that the column reads of a wave fall in distinct banks
constexpr int pair_pitch(int logla, int loglb, int lognt) { return ((1 << logla) + 1) << pair_logw(logla, loglb, lognt); }
constexpr uint32_t pair_lds_bytes(int logla, int loglb, int lognt, int esize)
{
    return uint32_t((1 << loglb) * pair_pitch(logla, loglb, lognt) * (esize / 2));
}
constexpr int64_t pair_max_tiles(int lognt) { return int64_t(1) << (31 - lognt); }

// k_long (fftu_long.hip): 512 threads hold W whole lines of L = 2^11 or 2^12 points,
// E elements per thread: 16 complex64 (W = 2 for L = 4096, 4 for L = 2048) or 8
// complex128 (W = 2 for L = 2048, 1 for L = 4096), within 128 VGPRs so that two
// workgroups share a CU.
// A tile is W / B whole outer blocks when rows have B <= W columns, or W of the
// B = 2W or 4W columns of one outer block. LDS: two twiddle tables of 64 and L / 64
// entries, then W rows of long_pitch words of one real part.
constexpr int kLongLogThreads = 9;
constexpr int kLongThreads = 1 << kLongLogThreads;
constexpr int kLongMinLogL = 11;
constexpr int kLongMaxLogL = 12;
constexpr int64_t kLongMaxTiles = int64_t(1) << (31 - kLongLogThreads);
constexpr int long_loge(int esize) { return esize == 16 ? 3 : 4; }
constexpr int long_logw(int logl, int esize) { return kLongLogThreads - (logl - long_loge(esize)); }
// L + L/16 words per line, plus 64 / W so that a wave's linear accesses (W lines x
// 64 / W positions) fall in distinct banks
constexpr int long_pitch(int logl, int esize)
{
    return (1 << logl) + (1 << (logl - 4)) + (64 >> long_logw(logl, esize));
}
constexpr uint32_t long_lds_bytes(int logl, int esize)
{
    return uint32_t((64 + (1 << (logl - 6))) * esize +
                    (1 << long_logw(logl, esize)) * long_pitch(logl, esize) * (esize / 2));
}

// k_lastx (fftu_lastx.hpp): the innermost dimension's Superstep-0 lines fused with
// the exchange. A workgroup of 2^lognt threads holds RW rows of all P blocks; its
// threads hold E = 2^logr elements in both the line plan (a line of 2^logl,
// lastx_loge(logl, logr) == logr) and the exchange (logr register bits, logh wave bits).
// lognt is 9, or 10 where 512 threads cannot hold one row of every block (a line
// of 256 over 64 blocks).
constexpr int kLastxLogThreads = 9;
constexpr int kLastxMaxLogThreads = 10;
constexpr int kLastxMinLogL = 5;
constexpr int kLastxMaxLogL = 8;
// one workgroup per tile, at most 2^31 threads per grid
constexpr int64_t lastx_max_tiles(int lognt) { return int64_t(1) << (31 - lognt); }

// Compiled register/wave splits: 2^3 = (2,2,2) or 2^4 = (2,2,2,2) / (4,4) in registers,
// and none, one 2, two 2s or one 4 across waves.
// k_lastx's line elements per thread (2^loge, which must be the split's 2^logr
// register sources): k_line's, except that lines of 32 and 64 meet a split of 16
// register sources as 16 elements per thread (stages of 16 and 2, or 16 and 4)
// instead of 8.
constexpr int lastx_loge(int logl, int logr)
{
    return (logl == 5 || logl == 6) && logr == 4 ? 4 : line_loge(logl);
}

constexpr bool lastx_split_ok(int logl, int nr, int lpr, int nh, int lph, int lognt = kLastxLogThreads)
{
    const int loge = lastx_loge(logl, nr * lpr);
    const bool reg = (loge == 3 && nr == 3 && lpr == 1) || (loge == 4 && ((nr == 4 && lpr == 1) || (nr == 2 && lpr == 2)));
    const bool wave = (nh == 0) || (nh == 1 && (lph == 1 || lph == 2)) || (nh == 2 && lph == 1);
    const int logh = nh * lph, logp = nr * lpr + logh;
    const int logtpl = logl - loge;
    const int logrw = lognt - logtpl - logp;
    return logl >= kLastxMinLogL && logl <= kLastxMaxLogL && reg && wave && logh <= 2 && logrw >= 0 &&
           logrw + logl >= 6 && (lognt == kLastxLogThreads || lognt == kLastxMaxLogThreads);
}

// The 1024-thread kernel exists only for the splits that 512 threads cannot hold.
constexpr bool lastx_split_needs_1024(int logl, int nr, int lpr, int nh, int lph)
{
    return !lastx_split_ok(logl, nr, lpr, nh, lph, kLastxLogThreads) &&
           lastx_split_ok(logl, nr, lpr, nh, lph, kLastxMaxLogThreads);
}

// k_lastx reads its tile linearly and regroups it through LDS when one thread's run
// of a line (TPL = L / E elements) is shorter than 128 bytes.
constexpr bool lastx_staged_load(int logl, int loge, int esize)
{
    return (int64_t(1) << (logl - loge)) * esize < 128;
}

// LDS bytes of k_lastx: omega_L table, then max(transpose, line stages) rows of 8-byte words.
constexpr uint32_t lastx_lds_bytes(int logl, int loge, int esize, int lognt = kLastxLogThreads)
{
    const int L = 1 << logl;
    const int tpl = 1 << (logl - loge);
    const int lp = L + tpl, pitch = L + L / 16 + 1;
    const int lines = 1 << (lognt - (logl - loge));
    return uint32_t(L * esize + lines * (lp > pitch ? lp : pitch) * 8);
}

// k_lastx copies the omega table into LDS when two 512-thread workgroups per CU still fit.
constexpr uint32_t kLastxTableLdsMax = 80 * 1024;
constexpr bool lastx_table_in_lds(int logl, int loge, int lognmax, int esize, int lognt = kLastxLogThreads)
{
    return lognt == kLastxLogThreads &&
           uint64_t(lastx_lds_bytes(logl, loge, esize, lognt)) + (uint64_t(esize) << lognmax) <= kLastxTableLdsMax;
}

struct LastxDesc {
    ExchangeDesc ex;       // its conj_in must be 0: the lines take the input conjugation
    int64_t tiles;         // M / (RW m_d)
    int32_t logl;
    int32_t lognt;         // log2 threads per workgroup (9 or 10)
    int32_t conj_in;       // conjugate on load (the first kernel of a plan)
    int32_t table_lds;     // the omega table in LDS (plain plans; convolution keeps it in HBM)
    uint32_t lds_bytes;    // with table_lds: lastx_lds_bytes + the table
};

// Mixed-radix path (fftu_mixed.hip): sides with factors 2, 3, 5 and 7.
constexpr int kMixedThreads = 256;
constexpr int kMixedPreF64 = 4;        // k_mline: tile elements per thread (the next tile, prefetched)
constexpr int kMixedPreF32 = 8;
constexpr int kMixedMaxW = 256;        // lines per k_mline tile at most
constexpr int kMixedMaxStages = 24;

// A pass of 1-D FFTs of length L over an array viewed as (A, L, B), B the
// stride of a line. A tile holds W (a power of two) consecutive lines of the A B
// lines, line u = a B + b.
struct MixedPassDesc {
    int64_t A, B;
    int64_t tiles;         // ceil(A B / W)
    int64_t pitch;         // LDS elements per tile line: L, or L + 1 when L is even (odd: no bank conflicts
                           // between consecutive lines)
    int32_t L;
    int32_t W, logW;
    int32_t nstages;
    int32_t radix[kMixedMaxStages];
    int64_t tstep;         // T / L: omega_L^j = table[j tstep], table = omega_T
    int32_t conj_in, conj_out;
    double scale;
    uint32_t lds_bytes;
};

// Geometry for the twiddle and the permutation of the mixed-radix path.
struct MixedGridDesc {
    int32_t d;
    int64_t N, M, P;
    int32_t n[kMaxDims], p[kMaxDims], m[kMaxDims], q[kMaxDims];
    int64_t tstep[kMaxDims];   // T / n_l
    int64_t T;
    int32_t conj_in, conj_out;
    int32_t twiddle;           // k_mpermute / k_mexchange: apply Superstep 0's twiddle on the way
    double scale;
    const void *mul;           // k_mexchange: null, or N elements in the output layout to multiply by
};

// Grids beyond p_max (some p_l^2 not dividing n_l): the group-cyclic levels of
// each dimension and the Put of one communication superstep (fftu_gcyclic.hip).
// Level i of dimension l works on sub-transforms of n_i points, each held by a
// group of p_i processors (p_0 = p_l, n_0 = n_l, n_{i+1} = p_i, p_{i+1} = p_i / m_l);
// the last level h has p_h^2 | n_h.
constexpr int kGcMaxLevels = 32;
struct GroupPutDim {
    int32_t mode;          // 0: nothing moves along this dimension; 1: Put of a level below h; 2: Put of level h
    int32_t m, p;          // local side m_l and grid side p_l
    int32_t pi;            // group size p_i of the level
    int32_t pn;            // mode 1: p_{i+1} = p_i / m
    int32_t q;             // mode 2: m / p_h
    int32_t mh;            // mode 2: m^h, groups of the last level
    int32_t h;             // mode 2: base-m digits of a group number
    int32_t ni;            // n_i: the twiddle is omega_{n_i}^{u k}
    int32_t reserved;
    int64_t tstep;         // T / n_i
};
// k_gplast (fftu_gcyclic.hip): the last Put of a power-of-two plan with its length-p_h
// FFTs, G = prod p_h <= 2^kGplastMaxLogG elements per thread.
constexpr int kGplastMaxLogG = 4;
struct GroupPutDesc {
    int32_t d;
    int32_t twiddle;       // multiply by the level's twiddle of the source element
    int32_t permute;       // move the element (0: the twiddle alone, in place of the source)
    int32_t conj_in, conj_out;
    int64_t N, M, T;
    double scale;
    GroupPutDim dim[kMaxDims];
};
// The real-input transform (fftu_real.hip): the packed complex array of shape
// n' = (n_1, ..., n_{d-1}, n_d/2), cyclic over p, and the Nyquist plane of shape
// (n_1, ..., n_{d-1}), cyclic over (p_1, ..., p_{d-1}), stored after it.
struct RealDesc {
    int32_t d;
    int32_t h;              // n_d / 2
    int64_t Nh;             // elements of the packed array (N / 2)
    int64_t Mh;             // of them per processor (Nh / P)
    int64_t Mp;             // elements of the Nyquist plane per processor of dimensions 1..d-1
    int32_t n[kMaxDims];    // n'
    int32_t p[kMaxDims];
    int32_t m[kMaxDims];    // n'_l / p_l
};

// The DCT-II / DST-II and their inverses (fftu_r2r.hip) on top of the real transform:
// the signal v (the zig-zag order of x) in the real-side layout of RealDesc, the
// coefficients y (N reals) cyclic over p. A thread takes one group of indices that
// are mirror images k_l <-> n_l - k_l in any subset of the dimensions.
constexpr int kR2RMaxDims = 4;
struct R2RDesc {
    int32_t d;
    int32_t dst;            // 1: DST (coefficients stored at n_l - 1 - k_l, the DCT of the signed signal)
    int32_t n[kMaxDims];    // full sides n_l
    int32_t p[kMaxDims];
    int32_t m[kMaxDims];    // n_l / p_l
    int32_t tstep[kMaxDims];  // T4 / (4 n_l): omega_{4 n_l}^k is table entry k tstep_l
    int64_t M;              // coefficients per processor (N / P)
    int64_t groups;         // prod_l (n_l / 2 + 1)
    RealDesc rd;            // the half spectrum of the signal (packed shape, Nyquist plane)
};

// k_r2rpost_rows (whole coefficient rows staged in LDS) where every wave's lanes start
// on a multiple of 64 along the last dimension (n_d / 2 a multiple of 64), the
// 2^(d-1) rows of a workgroup fit 32 KiB and there are enough rows to fill the device;
// returns its LDS bytes, or 0 for the one-group-per-thread k_r2rpost.
inline uint32_t r2rpost_rows_lds(const R2RDesc &g, size_t esize)
{
    if (g.d < 2 || g.d > kR2RMaxDims) return 0;
    const int64_t nd = g.n[g.d - 1], h = nd / 2;
    if (h % 64 != 0 || nd >= (int64_t(1) << 22)) return 0;
    const int64_t bytes = (int64_t(1) << (g.d - 1)) * int64_t(g.p[g.d - 1]) * (int64_t(g.m[g.d - 1]) + 1) * int64_t(esize);
    if (bytes > 32768 || g.groups / (h + 1) < 1024) return 0;
    return uint32_t(bytes);
}

// k_r2rpre with one workgroup per row of representatives (n_d / 2 a multiple of 64,
// at least 1024 rows), or one group per thread.
inline bool r2rpre_rows(const R2RDesc &g)
{
    if (g.d < 2 || g.d > kR2RMaxDims) return false;
    const int64_t h = g.n[g.d - 1] / 2;
    return h % 64 == 0 && g.groups / (h + 1) >= 1024;
}

// k_r2rpre_merge (the inverse's spectrum and the real transform's merge in one pass)
// where k_r2rpre takes rows and the row's 2^(d-1) (n_d / 2 + 1) spectrum values fit
// 32 KiB of LDS; returns its LDS bytes, or 0.
inline uint32_t r2rpre_merge_lds(const R2RDesc &g, size_t esize)
{
    if (!r2rpre_rows(g)) return 0;
    const int64_t bytes = (int64_t(1) << (g.d - 1)) * (g.n[g.d - 1] / 2 + 1) * int64_t(esize);
    return bytes <= 32768 ? uint32_t(bytes) : 0;
}

// k_mxexchange (fftu_mixed.hip): the mixed-radix exchange for grids whose sides are
// powers of two (any local sides): the register and wave split of k_exchange (NR
// register dimensions of 2^LPR, NH wave dimensions of 2^LPH) with general index
// arithmetic for the local sides.
struct MxSplit {
    int32_t nr, lpr, nh, lph;
    int32_t rdim[kMaxDims];
    int32_t hdim[kMaxDims];
    uint32_t lds_bytes;
};
// k_mxexchange work items: W = rows x nchunk, bit consecutive items per workgroup.
struct MxRows {
    uint32_t nchunk, W, bit;
};

// k_mxexchange with whole rows staged in LDS (kMxRowsThreads threads take one row of the
// last dimension and write each output row contiguously): where the output segments of
// q_{d-1} elements are not whole 128-byte lines, the last dimension is a register
// dimension of the split, there are wave dimensions (their LDS is reused) and a row
// fits the workgroup (m_{d-1} <= kMxRowsThreads / 2^(NH LPH)).
constexpr int kMxRowsThreads = 512;
inline bool mx_rows_staged(const MixedGridDesc &g, const MxSplit &sp, size_t esize)
{
    if (sp.nh < 1 || sp.nr < 1 || sp.nr * sp.lpr > 4 || g.d < 1) return false;
    const int last = g.d - 1;
    if (sp.rdim[sp.nr - 1] != last || (1 << sp.lpr) != g.p[last]) return false;
    const int H = 1 << (sp.nh * sp.lph);
    if (int64_t(g.m[last]) > int64_t(kMxRowsThreads / H)) return false;
    return (int64_t(g.q[last]) * int64_t(esize)) % 128 != 0;
}

// k_mexchange: P sources of 64 local indices in LDS, grid sides of one radix stage.
constexpr int64_t kMexMaxP = 64;
constexpr int kMexThreads = 512;
constexpr int kMexBatch = 8;           // source loads per lane in flight
constexpr size_t kMexTableLdsMax = 80 * 1024;   // LDS for tile + digit tables + the omega_T copy
// k_mexchange keeps its twiddle table in LDS when two workgroups per CU still fit.
constexpr bool mexchange_table_in_lds(int64_t P, int64_t T, int esize)
{
    return size_t(P) * (64 * size_t(esize) + 8) + size_t(T) * size_t(esize) <= kMexTableLdsMax;
}
constexpr bool mexchange_radix_ok(int p)
{
    return p == 1 || p == 2 || p == 3 || p == 4 || p == 5 || p == 7 || p == 8;
}

// Persistent batch (fftu_batch.hip). One descriptor per (stage, transform).
constexpr int kBatchThreads = 256;
constexpr int kBatchMaxLogLine = 8;     // longest Superstep-0 line of a batched transform: 2^8
constexpr int kBatchMaxLine = 1 << kBatchMaxLogLine;
constexpr int kExchangeStage = 8;       // BatchStage::kind of the fused exchange
constexpr int kBatchItemLog = 17;       // about 2^17 elements per work item

struct BatchStage {
    int32_t kind;          // kLineStrided / kLineContig / kLineStaged, or kExchangeStage
    int32_t per_item;      // tiles (line tiles, or exchange groups of 4 x 64 indices) per work item
    int64_t tiles;
    int32_t member;        // transform this stage belongs to
    int32_t io;            // bit 0: reads the transform's input, bit 1: writes its output (BatchDesc::bind)
    const void *src;       // the transform's workspace, unless io bit 0
    void *dst;             // the transform's workspace, unless io bit 1
    PassDesc pd;           // line passes
    ExchangeDesc ex;       // the exchange (no wave dimensions)
};

// The caller's buffers of one transform. They live in a device array of their
// own, written by k_batch_bind on the execution stream, so that new buffers are
// bound in stream order (no host wait) and a captured graph carries its own.
struct BatchBind {
    const void *in;
    void *out;
};
constexpr int kBindChunk = 96;         // buffer pairs per k_batch_bind launch (passed by value)
struct BindChunk {
    int32_t first;                     // first transform of this chunk
    int32_t count;                     // pairs used, <= kBindChunk
    BatchBind b[kBindChunk];
};

struct BatchDesc {
    int32_t nstages;             // descriptors
    int32_t reserved;
    int64_t wait_limit;          // real-time-clock ticks a dependency wait may last (then: error flag)
    int64_t nitems;              // work items in total
    const BatchStage *stages;    // [nstages], stage-major
    const int64_t *starts;       // [nstages + 1] first item of each descriptor
    const int32_t *dep;          // [nstages] descriptor that must finish first, or -1
    int32_t *done;               // [nstages] finished items
    unsigned long long *next;    // next item to hand out
    int32_t *error;              // set when a wait gave up
    const BatchBind *bind;       // [transforms] the caller's buffers
};

// Host-side work list of a batch plan (built by build_batch_worklist in fftu_api.cpp).
struct BatchWorklist {
    std::vector<BatchStage> stages;   // stage-major
    std::vector<int64_t> starts;      // stages.size() + 1
    std::vector<int32_t> dep;         // descriptor each one waits for, or -1
    std::vector<int> member;          // transform of each descriptor
    std::vector<int> first;           // 1: reads the transform's input
    std::vector<int> last;            // 1: writes the transform's output
    std::vector<int64_t> N;           // elements of each transform
    std::vector<uint64_t> ws;         // workspace offset of each transform (elements)
    uint64_t ws_total = 0;
    int lognmax = 0;
    int64_t items = 0;
    uint32_t lds = 0;                 // dynamic LDS of the persistent kernel
};
fftu_status build_batch_worklist(int count, const int d[], const int64_t *const n[], const int64_t *const p[],
                                 fftu_dtype dtype, fftu_direction direction, BatchWorklist &wl);

enum class Precision { F32, F64 };

// Launchers (fftu_kernels.hip). All return hipSuccess or the launch error.
hipError_t launch_pass(Precision prec, const void *in, void *out, const PassDesc &pd, const void *table,
                       hipStream_t stream);
hipError_t launch_line(Precision prec, const void *in, void *out, const PassDesc &pd, const void *table,
                       hipStream_t stream);
hipError_t launch_group2(Precision prec, const void *in, void *out, const PassDesc &pd, const void *table,
                         hipStream_t stream);
hipError_t launch_batch_reset(const BatchDesc &bd, hipStream_t stream);   // counters to zero (a kernel)
hipError_t launch_batch_bind(BatchBind *bind, const BindChunk &c, hipStream_t stream);   // bind[first + i] = b[i]
hipError_t launch_mline(Precision prec, const void *in, void *out, const MixedPassDesc &pd, const void *table,
                        hipStream_t stream);
hipError_t launch_mtwiddle(Precision prec, const void *in, void *out, const MixedGridDesc &g, const void *table,
                           hipStream_t stream);
hipError_t launch_mpermute(Precision prec, const void *in, void *out, const MixedGridDesc &g, const void *table,
                           hipStream_t stream);
hipError_t launch_mexchange(Precision prec, const void *in, void *out, const MixedGridDesc &g, const void *table,
                            hipStream_t stream);
hipError_t launch_pointwise(Precision prec, const void *a, const void *b, void *out, int64_t count, double scale,
                            hipStream_t stream);
hipError_t launch_fill_uniform(Precision prec, void *out, int64_t count, uint32_t k0, uint32_t k1, uint64_t base,
                               hipStream_t stream);
hipError_t launch_batch(Precision prec, const BatchDesc &bd, const void *table, uint32_t blocks, uint32_t lds_bytes,
                        hipStream_t stream);
int batch_blocks_per_cu(Precision prec, uint32_t lds_bytes);
hipError_t launch_twiddle(Precision prec, const void *in, void *out, const GridDesc &g, const void *table,
                          hipStream_t stream);
hipError_t launch_permute(Precision prec, const void *in, void *out, const GridDesc &g, hipStream_t stream);
hipError_t launch_exchange(Precision prec, const void *in, void *out, const ExchangeDesc &ex, const void *table,
                           hipStream_t stream);
hipError_t launch_pair(Precision prec, const void *in, void *out, const PassDesc &pd, hipStream_t stream);
// Superstep 0's twiddle and Superstep 1 as one tiled transpose, for grids with every
// q_l = 1 (m = p) and M >= 64; in and out must differ. ld > 0: also the innermost
// dimension's length-2^ld FFTs of Superstep 0 (before the twiddle) and of Superstep 2
// (after the transpose); g.conj_out and g.scale apply on the store.
hipError_t launch_ttranspose(Precision prec, const void *in, void *out, const GridDesc &g, int ld, const void *table,
                             hipStream_t stream);
hipError_t launch_long(Precision prec, const void *in, void *out, const PassDesc &pd, const void *table,
                       hipStream_t stream);
hipError_t launch_lastx(Precision prec, const void *in, void *out, const LastxDesc &lx, const void *table,
                        hipStream_t stream);
// The real-input transform's steps around the complex transform of the packed
// array (fftu_real.hip); `table` holds omega_{n_d}^j, j in [n_d]. rsplit: in place
// on buf (forward; writes the Nyquist plane after the Nh packed elements). rmerge:
// from in (half spectrum and plane) to out (Nh elements; in == out allowed).
hipError_t launch_mxexchange(Precision prec, const void *in, void *out, const MixedGridDesc &g, const MxSplit &sp,
                             const void *table, hipStream_t stream);
hipError_t launch_rsplit(Precision prec, void *buf, const RealDesc &rd, const void *table, hipStream_t stream);
// Coefficients from the half spectrum (forward), the half spectrum from the
// coefficients (inverse), and the sign pattern of the DST's signal (in place allowed).
hipError_t launch_r2r_post(Precision prec, const void *spec, void *y, const R2RDesc &g, const void *table4,
                           hipStream_t stream);
hipError_t launch_r2r_pre(Precision prec, const void *y, void *spec, const R2RDesc &g, const void *table4,
                          hipStream_t stream);
// The inverse's spectrum merged into the packed spectrum z (N / 2 complex) in one pass
// (r2rpre_merge_lds(g, ...) > 0); z is the real transform's complex input.
hipError_t launch_r2r_pre_merge(Precision prec, const void *y, void *z, const R2RDesc &g, const void *table4,
                                hipStream_t stream);
hipError_t launch_r2r_sign(Precision prec, const void *in, void *out, const R2RDesc &g, hipStream_t stream);
hipError_t launch_rmerge(Precision prec, const void *in, void *out, const RealDesc &rd, const void *table,
                         hipStream_t stream);
// One communication superstep of a group-cyclic plan (fftu_gcyclic.hip); in != out when g.permute.
hipError_t launch_gplast(Precision prec, const void *in, void *out, const GroupPutDesc &g, const void *table,
                         hipStream_t stream);
// k_gputt (fftu_gcyclic.hip): a power-of-two Put as a bit permutation in tiles of
// 2^K <= 2^kGputTileLog elements (see gput_tiling).
constexpr int kGputTileLog = 10;
struct GputTileDesc {
    int32_t K;              // log2 elements per tile
    int32_t ntb;            // bits that enumerate the tiles
    int32_t pad_shift;      // LDS slot s at s + (s >> pad_shift)
    int32_t lsrc[kGputTileLog], dslot[kGputTileLog], xdst[kGputTileLog];
    int32_t ysrc[31], ydst[31];
    int64_t ntiles;
};
bool gput_tiling(const GroupPutDesc &g, int esize, GputTileDesc &tl);
hipError_t launch_gput(Precision prec, const void *in, void *out, const GroupPutDesc &g, const void *table,
                       hipStream_t stream);

// Plan facts for entry points outside fftu_api.cpp.
bool plan_is_batch(const fftu_plan_s *plan);
int plan_device(const fftu_plan_s *plan);                 // device the plan was made on
size_t plan_workspace_bytes(const fftu_plan_s *plan);     // N b: the workspace one execution needs
fftu_status record_status(fftu_status s);                 // sets fftu_last_error() of this thread

}  // namespace fftu
