// Host side of libfftu: argument checks, the planner, twiddle-table generation
// and the C ABI declared in include/fftu.h.
//
// The planner maps Algorithm 2.3 (arXiv 2203.11795) onto kernel launches:
//   Superstep 0, local FFTs   -> one k_pass launch per group of consecutive local
//                                dimensions whose tile fits in LDS (innermost first)
//   Superstep 0, twiddle      \
//   Superstep 1, the Put       > one k_exchange launch when the grid splits (see exchange_split);
//   Superstep 2, F_p          /  k_twiddle, k_permute and one k_pass per grid dimension
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "fftu_internal.hpp"

using fftu::ExchangeDesc;
using fftu::GridDesc;
using fftu::PassDesc;
using fftu::Precision;

struct fftu_plan_s {
    int d = 0;
    int64_t n[fftu::kMaxDims] = {};
    int64_t p[fftu::kMaxDims] = {};
    fftu_dtype dtype = FFTU_C128;
    fftu_direction dir = FFTU_FORWARD;
    Precision prec = Precision::F64;
    size_t esize = 16;
    int device = 0;
    void *table = nullptr;
    void *ws = nullptr;
    bool external = false;           // fftu_plan_external: shared table, workspace given per call
    fftu_plan_s *conv_inv = nullptr; // fftu_plan_convolution: the inverse plan (external, uses this plan's workspace)
    // mixed-radix plans (some side not a power of two)
    bool mixed = false;
    bool mfused = false;             // mixed radix with k_mexchange (or k_mxexchange)
    bool mx = false;                 // the fused exchange on k_mxexchange
    fftu::MxSplit mxs{};
    std::vector<fftu::MixedPassDesc> ms0, ms2;
    fftu::MixedGridDesc mg{};
    int64_t table_T = 0;             // entries of the twiddle table omega_T
    uint64_t table_bytes = 0;
    uint64_t ws_bytes = 0;
    GridDesc grid{};                 // geometry, no conjugation or scaling
    std::vector<PassDesc> s0;        // Superstep 0 local FFT passes
    std::vector<PassDesc> s2;        // Superstep 2 passes (unfused form)
    bool fused = false;
    bool ttrans = false;             // unfused, every q_l = 1: twiddle and permutation as one k_ttranspose
    int ttrans_ld = 0;               // > 0: k_ttranspose also runs the innermost dimension's FFTs of Supersteps 0, 2
    std::vector<PassDesc> s0t, s2t;  // with ttrans_ld: Superstep 0 and 2 passes without the innermost dimension
    ExchangeDesc ex{};
    bool lastx = false;              // k_lastx: the innermost dimension's lines fused with the exchange
    std::vector<PassDesc> s0x;       // the other Superstep 0 passes, run before k_lastx
    fftu::LastxDesc lx{};
    // real-input transforms (fftu_plan_real): the complex plan of the packed array, the
    // split / merge step and its omega_{n_d} table
    bool real = false;
    fftu_plan_s *rc = nullptr;
    fftu::RealDesc rd{};
    void *rtable = nullptr;
    int64_t real_in_elems = 0, real_out_elems = 0;   // complex elements of each side's buffer
    // DCT / DST (fftu_plan_r2r): the real plan of the zig-zag signal (rc), the
    // coefficient step and its omega_{T4} table (rtable), the spectrum in ws
    bool r2r = false;
    fftu_r2r_kind r2r_kind = FFTU_DCT;
    bool r2r_sign_fused = false;   // DST forward: the signs in the complex transform's first pass
    bool r2r_pre_merge = false;    // inverse: k_r2rpre_merge in place of k_r2rpre and k_rmerge
    fftu::R2RDesc r2d{};
    // grids beyond p_max (some p_l^2 not dividing n_l): group-cyclic levels, several supersteps
    bool gc = false;
    int gc_H = 0;                                       // communication supersteps
    bool gc_pow2 = false;                                   // phases on the power-of-two pass kernels
    int gc_last_logg = 0;                                   // > 0: k_gplast fuses the last Put and phase H
    std::vector<std::vector<fftu::MixedPassDesc>> gphase;   // computation phases 0..H: local FFT passes
    std::vector<std::vector<PassDesc>> gphase2;             // the same with every side a power of two
    std::vector<fftu::GroupPutDesc> gput;                   // communication supersteps 0..H-1 (twiddle + Put)
    // per-kernel timing (fftu_timing_begin / fftu_timing_end)
    std::vector<std::string> launch_names;   // kernel of each launch of fftu_execute
    // batch plans (fftu_plan_batch)
    bool is_batch = false;
    int count = 0;
    std::vector<int64_t> member_N;             // elements of each transform
    std::vector<uint64_t> member_ws;           // workspace offset (elements) of each transform
    std::vector<fftu::BatchStage> hstages;     // host copy of the work list
    std::vector<int> stage_member;             // transform of each descriptor
    std::vector<int> stage_first;              // 1 if the descriptor reads the transform's input
    std::vector<int> stage_last;               // 1 if it writes the transform's output
    int64_t batch_items = 0;
    uint32_t batch_blocks = 0;
    uint32_t batch_lds = 0;
    int64_t batch_wait_ticks = 0;          // bound of one dependency wait (about 2 s)
    void *dstages = nullptr;
    void *dstarts = nullptr;
    void *ddep = nullptr;
    void *ddone = nullptr;
    void *dnext = nullptr;
    void *derror = nullptr;
    void *dbind = nullptr;                     // [count] BatchBind: the buffers the device list holds
    std::vector<int64_t> hstarts;              // external batches: the work list's item ranges and
    std::vector<int32_t> hdep;                 // dependencies, copied with the list on every call
    void *last_ws = nullptr;                   // external batches: workspace of the last call (error flag)
    std::vector<const void *> bound_in;        // what dbind holds once the enqueued work has run
    std::vector<void *> bound_out;
    std::vector<hipEvent_t> events;  // timing_max x (launches + 1)
    int timing_max = 0;
    int timing_used = 0;
    int launches = 0;
};

namespace {

thread_local fftu_status g_last = FFTU_SUCCESS;

// Planner tuning knobs (fftu_set_tuning); -1 = default.
// Planner knobs (fftu_set_tuning): process-wide, read when a plan is made.
std::atomic<int> g_tune[FFTU_TUNE_COUNT] = {{-1}, {-1}, {-1}, {-1}, {-1}, {-1}, {-1}, {-1}};
int knob(int i) { return g_tune[i].load(std::memory_order_relaxed); }
const int g_tune_min[FFTU_TUNE_COUNT] = {2, 0, 0, 16, 0, 0, 2, 9};
const int g_tune_max[FFTU_TUNE_COUNT] = {6, 8, 4, 160, 1, 1, 8, 12};

int64_t lds_cap()
{
    const int v = knob(FFTU_TUNE_MAX_LDS_KB);
    return int64_t(v >= 0 ? v : 64) * 1024;
}

fftu_status record(fftu_status s)
{
    g_last = s;
    return s;
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// Only the prime factors 2, 3, 5 and 7 (the mixed-radix stages).
bool is_smooth(int64_t v)
{
    if (v < 1) return false;
    for (int f : {2, 3, 5, 7})
        while (v % f == 0) v /= f;
    return v == 1;
}

int64_t gcd64(int64_t a, int64_t b)
{
    while (b) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

int64_t lcm64(int64_t a, int64_t b) { return a / gcd64(a, b) * b; }

// Longest line of the mixed-radix pass: two LDS buffers of a line plus its roots in 64 KiB.
int64_t max_mixed_len(fftu_dtype dt) { return dt == FFTU_C128 ? 1024 : 2048; }

int ilog2(int64_t v)
{
    int r = 0;
    while ((int64_t(1) << r) < v) ++r;
    return r;
}

// Largest local length (n_l / p_l) and grid side p_l that one LDS tile can hold.
int log_tile(fftu_dtype dt) { return dt == FFTU_C128 ? fftu::kLogTileF64 : fftu::kLogTileF32; }
int64_t max_len(fftu_dtype dt) { return int64_t(1) << log_tile(dt); }
int log_wmax(fftu_dtype dt) { return dt == FFTU_C128 ? 5 : 6; }       // 512-byte column runs

// The group-cyclic levels of one dimension (Section 2.3, the paragraph after
// eq. (2.13)): level i transforms sub-transforms of n_i points on groups of p_i
// processors; n_0 = n, p_0 = p, and while p_i^2 does not divide n_i the level's
// m = n / p sub-transforms of each group go to groups of p_{i+1} = p_i / m
// (which needs m | p_i) as sub-transforms of n_{i+1} = p_i points. Level h, the
// first with p_h^2 | n_h, ends with Algorithm 2.2's own Put.
struct GcLevels {
    int h = 0;
    int64_t m = 1;
    int64_t n[fftu::kGcMaxLevels] = {};
    int64_t p[fftu::kGcMaxLevels] = {};
};

bool gc_levels(int64_t n, int64_t p, GcLevels &lv)
{
    lv = GcLevels{};
    if (p < 1 || n % p) return false;
    lv.m = n / p;
    int64_t ni = n, pi = p;
    for (int i = 0; i < fftu::kGcMaxLevels; ++i) {
        lv.n[i] = ni;
        lv.p[i] = pi;
        lv.h = i;
        if ((ni / pi) % pi == 0) return true;
        if (lv.m == 1 || pi % lv.m) return false;
        ni = pi;
        pi /= lv.m;
    }
    return false;
}

// Some dimension has p_l | n_l but not p_l^2 | n_l.
bool plan_is_group_cyclic(int d, const int64_t n[], const int64_t p[])
{
    for (int l = 0; l < d; ++l)
        if (p[l] >= 1 && n[l] % p[l] == 0 && (n[l] / p[l]) % p[l] != 0) return true;
    return false;
}

fftu_status validate(int d, const int64_t n[], const int64_t p[], fftu_dtype dtype, fftu_direction direction)
{
    if (d < 1 || !n || !p) return FFTU_ERROR_INVALID_VALUE;
    if (dtype != FFTU_C64 && dtype != FFTU_C128) return FFTU_ERROR_INVALID_VALUE;
    if (direction != FFTU_FORWARD && direction != FFTU_INVERSE) return FFTU_ERROR_INVALID_VALUE;
    if (d > FFTU_MAX_DIMS) return FFTU_ERROR_UNSUPPORTED;
    for (int l = 0; l < d; ++l)
        if (n[l] < 1 || p[l] < 1) return FFTU_ERROR_INVALID_VALUE;
    // Algorithm 2.3, Input: p_l^2 | n_l. Otherwise (p_l | n_l only) the grid needs the
    // group-cyclic levels of Section 2.3 (gc_levels).
    for (int l = 0; l < d; ++l)
        if (n[l] % p[l] != 0) return FFTU_ERROR_NOT_DIVISIBLE;
    if (plan_is_group_cyclic(d, n, p)) {
        int64_t N = 1, T = 1;
        for (int l = 0; l < d; ++l) {
            GcLevels lv;
            if (!gc_levels(n[l], p[l], lv)) return FFTU_ERROR_NOT_DIVISIBLE;
            if (!is_smooth(n[l])) return FFTU_ERROR_UNSUPPORTED;
            if (n[l] / p[l] > max_mixed_len(dtype) || lv.p[lv.h] > max_mixed_len(dtype)) return FFTU_ERROR_UNSUPPORTED;
            if (N > (int64_t(1) << 31) / n[l]) return FFTU_ERROR_UNSUPPORTED;
            N *= n[l];
            T = lcm64(T, n[l]);
            if (T > (int64_t(1) << 24)) return FFTU_ERROR_UNSUPPORTED;
        }
        if (N >= (int64_t(1) << 31)) return FFTU_ERROR_UNSUPPORTED;
        return FFTU_SUCCESS;
    }
    bool all_pow2 = true;
    for (int l = 0; l < d; ++l) all_pow2 = all_pow2 && is_pow2(n[l]) && is_pow2(p[l]);
    if (all_pow2) {
        int logN = 0;
        for (int l = 0; l < d; ++l) {
            logN += ilog2(n[l]);
            if (n[l] / p[l] > max_len(dtype) || p[l] > max_len(dtype)) {
                // complex128 lines of 4096 points exist only in k_long, for rows of at most 8
                // columns after the dimension (Superstep 0: the local sides after l;
                // Superstep 2: q_l times them)
                if (dtype != FFTU_C128 || n[l] / p[l] > 4096 || p[l] > 4096) return FFTU_ERROR_UNSUPPORTED;
                int64_t after = 1;
                for (int j = l + 1; j < d; ++j) after *= n[j] / p[j];
                if (n[l] / p[l] == 4096 && after > 8) return FFTU_ERROR_UNSUPPORTED;
                if (p[l] == 4096 && (n[l] / p[l] / p[l]) * after > 8) return FFTU_ERROR_UNSUPPORTED;
            }
        }
        if (logN >= 40) return FFTU_ERROR_UNSUPPORTED;
        return FFTU_SUCCESS;
    }
    // Mixed-radix path: prime factors 2, 3, 5, 7 only; lines up to the LDS tile;
    // N < 2^31 (32-bit index arithmetic); table omega_T with T = lcm(n_l) <= 2^24.
    int64_t N = 1, T = 1;
    for (int l = 0; l < d; ++l) {
        if (!is_smooth(n[l])) return FFTU_ERROR_UNSUPPORTED;
        if (n[l] / p[l] > max_mixed_len(dtype) || p[l] > max_mixed_len(dtype)) return FFTU_ERROR_UNSUPPORTED;
        if (N > (int64_t(1) << 31) / n[l]) return FFTU_ERROR_UNSUPPORTED;
        N *= n[l];
        T = lcm64(T, n[l]);
        if (T > (int64_t(1) << 24)) return FFTU_ERROR_UNSUPPORTED;
    }
    if (N >= (int64_t(1) << 31)) return FFTU_ERROR_UNSUPPORTED;
    return FFTU_SUCCESS;
}

bool plan_is_mixed(int d, const int64_t n[], const int64_t p[])
{
    for (int l = 0; l < d; ++l)
        if (!is_pow2(n[l]) || !is_pow2(p[l])) return true;
    return false;
}

// Radix split of a length 2^logL into stages of at most 16, as even as possible.
void split_radix(int logL, int32_t *out, int32_t *count)
{
    const int nst = (logL + 3) / 4;
    for (int s = 0; s < nst; ++s) out[s] = logL / nst + (s < logL % nst ? 1 : 0);
    *count = nst;
}

// k_line for a single dimension of length 2^logL when a good layout exists;
// returns false to fall back to the generic tile pass.
bool make_line_pass(int logA, int logL, int logB, fftu_dtype dt, int lognmax, PassDesc &pd, int min_log_threads = 0)
{
    if (logL < 1 || logL > 12) return false;
    const int esize = dt == FFTU_C128 ? 16 : 8;
    const int xbytes = 8;   // LDS bytes per element in a stage exchange: one double (re/im rounds) or one complex64
    const int logTPL = logL - fftu::line_loge(logL);
    const int64_t L = int64_t(1) << logL;
    const int64_t cap = lds_cap();
    pd = PassDesc{};
    pd.loglen[0] = logL;
    pd.naxes = 1;
    pd.logB = logB;
    pd.logG = logL;
    pd.GB = int64_t(1) << (logL + logB);
    pd.lognmax = lognmax;
    pd.scale = 1.0;
    if (logB >= 2) {
        // columns: W consecutive lines of the (A, B) lines per workgroup, i.e. runs of
        // min(W, B) elements per row; W > B spans several outer blocks
        const int kw = knob(FFTU_TUNE_LINE_STRIDED_LOGW);
        int logW = kw >= 0 ? kw : log_wmax(dt);
        logW = std::max(logW, min_log_threads - logTPL);
        logW = std::min(logW, logA + logB);
        const int kp = knob(FFTU_TUNE_LINE_PAD);
        const int pad = kp >= 0 ? kp : 1;
        while (logW > 0 && (((int64_t(1) << logW) + pad) * L * xbytes + L * esize) > cap) --logW;
        while (logW > 0 && (logW + logTPL) > 8) --logW;
        if (logW < 2) return false;
        if (logW >= logB && (int64_t(esize) << logB) < 256) {
            // rows of the tile are shorter than 256 bytes, but the tile spans whole outer
            // blocks and so is contiguous: load and store it linearly through LDS
            const int32_t lw = int32_t(L + (L >> 4) + 1);
            const int64_t bytes = L * esize + (int64_t(1) << logW) * lw * esize;
            if (bytes <= cap) {
                pd.kind = fftu::kLineStaged;
                pd.logW = logW;
                pd.logBt = logB;
                pd.logTPA = 0;
                pd.lw = lw;
                pd.tiles = int64_t(1) << (logA + logB - logW);
                pd.threads = 1 << (logW + logTPL);
                pd.lds_bytes = uint32_t(bytes);
                return true;
            }
        }
        pd.kind = fftu::kLineStrided;
        pd.logW = logW;
        pd.logBt = std::min(logW, logB);
        pd.logTPA = logB >= logW ? logB - logW : 0;
        pd.lw = (1 << logW) + pad;
        pd.tiles = int64_t(1) << (logA + logB - logW);
        pd.threads = 1 << (logW + logTPL);
        pd.lds_bytes = uint32_t(L * esize + L * pd.lw * xbytes);
        return true;
    }
    if (logB == 0) {
        // contiguous lines: about 2^9 (complex128) or 2^10 (complex64) elements per workgroup
        const int log_target = dt == FFTU_C128 ? 9 : 10;
        const int kc = knob(FFTU_TUNE_LINE_CONTIG_LOGW);
        int logW = kc >= 0 ? kc : std::max(0, log_target - logL);
        logW = std::max(logW, min_log_threads - logTPL);
        logW = std::min(logW, logA);
        while (logW > 0 && (logW + logTPL) > 8) --logW;
        if (logW + logTPL > 8) return false;
        pd.kind = ((int64_t(1) << logTPL) * esize >= 128) ? fftu::kLineContig : fftu::kLineStaged;
        pd.lw = int32_t(L + (L >> 4) + 1);
        const int per = pd.kind == fftu::kLineStaged ? esize : xbytes;
        while (logW > 0 && L * esize + (int64_t(1) << logW) * pd.lw * per > cap) --logW;
        pd.logW = logW;
        pd.logBt = 0;
        pd.logTPA = 0;
        pd.tiles = int64_t(1) << (logA - logW);
        pd.threads = 1 << (logW + logTPL);
        pd.lds_bytes = uint32_t(L * esize + (int64_t(1) << logW) * pd.lw * per);
        return pd.lds_bytes <= cap;
    }
    return false;
}

// A pass over an array viewed as (A, group..., B).
// k_long: lines of 2^11 / 2^12 points over rows of B <= 4W columns (W whole lines per
// tile), where k_line has no per-thread split.
bool make_long_pass(int logA, int logL, int logB, fftu_dtype dt, int lognmax, PassDesc &pd)
{
    const int esize = dt == FFTU_C128 ? 16 : 8;
    if (logL < fftu::kLongMinLogL || logL > fftu::kLongMaxLogL) return false;
    const int logW = fftu::long_logw(logL, esize);
    if (logB > logW + (logW == 0 ? 3 : 2) || logA + logB < logW) return false;
    const int64_t tiles = int64_t(1) << (logA + logB - logW);
    if (tiles > fftu::kLongMaxTiles) return false;
    pd = PassDesc{};
    pd.kind = fftu::kLong;
    pd.threads = fftu::kLongThreads;
    pd.naxes = 1;
    pd.loglen[0] = logL;
    pd.logG = logL;
    pd.logB = logB;
    pd.GB = int64_t(1) << (logL + logB);
    pd.logW = logW;
    pd.logBt = logB;
    pd.logTPA = 0;
    pd.lw = fftu::long_pitch(logL, esize);
    pd.tiles = tiles;
    pd.lognmax = lognmax;
    pd.scale = 1.0;
    pd.lds_bytes = fftu::long_lds_bytes(logL, esize);
    return true;
}

PassDesc make_pass(int logA, const std::vector<int> &loglens, int logB, fftu_dtype dt, int lognmax)
{
    PassDesc pd{};
    if (loglens.size() == 1 && make_line_pass(logA, loglens[0], logB, dt, lognmax, pd)) return pd;
    if (loglens.size() == 1 && make_long_pass(logA, loglens[0], logB, dt, lognmax, pd)) return pd;
    pd.kind = fftu::kTilePass;
    pd.threads = fftu::kPassThreads;
    int logG = 0;
    for (int v : loglens) logG += v;
    const int esize = dt == FFTU_C128 ? 16 : 8;
    int logW = std::min(log_tile(dt) - logG, logB + logA);
    if (logB >= log_wmax(dt)) logW = std::min(logW, log_wmax(dt));
    if (logW < 0) logW = 0;
    pd.logB = logB;
    pd.logG = logG;
    pd.logW = logW;
    pd.logBt = std::min(logB, logW);
    pd.logTPA = logB >= logW ? logB - logW : 0;
    pd.GB = int64_t(1) << (logG + logB);
    pd.tiles = int64_t(1) << (logA + logB - logW);
    pd.lw = (1 << logW) + (logW >= 2 ? 1 : 0);
    pd.naxes = int32_t(loglens.size());
    int stride = 0;
    for (int i = pd.naxes - 1; i >= 0; --i) {
        pd.loglen[i] = loglens[i];
        pd.logstride[i] = stride;
        stride += loglens[i];
        split_radix(loglens[i], pd.lograd[i], &pd.nstages[i]);
    }
    pd.lognmax = lognmax;
    pd.conj_in = 0;
    pd.conj_out = 0;
    pd.scale = 1.0;
    pd.lds_bytes = uint32_t(uint32_t(pd.lw) * (1u << logG) * uint32_t(esize));
    return pd;
}

struct Geometry {
    int d;
    int logn[fftu::kMaxDims], logp[fftu::kMaxDims], logm[fftu::kMaxDims], logq[fftu::kMaxDims];
    int logP, logM, logN, lognmax;
};

Geometry geometry(int d, const int64_t n[], const int64_t p[])
{
    Geometry G{};
    G.d = d;
    for (int l = 0; l < d; ++l) {
        G.logn[l] = ilog2(n[l]);
        G.logp[l] = ilog2(p[l]);
        G.logm[l] = G.logn[l] - G.logp[l];
        G.logq[l] = G.logm[l] - G.logp[l];
        G.logP += G.logp[l];
        G.logM += G.logm[l];
        G.lognmax = std::max(G.lognmax, G.logn[l]);
    }
    G.logN = G.logP + G.logM;
    return G;
}

// k_group2 for the two innermost dimensions 2^logL1 (outer) x 2^logL2 (inner) of
// contiguous planes (B = 1), when both sides are 4..64 and a plane fits in 16 KiB.
bool make_group2_pass(int logA, int logL1, int logL2, fftu_dtype dt, int lognmax, PassDesc &pd)
{
    if (logL1 < 2 || logL1 > 6 || logL2 < 2 || logL2 > 6) return false;
    const int esize = dt == FFTU_C128 ? 16 : 8;
    const int logG = logL1 + logL2;
    if ((int64_t(1) << logG) * esize > 16 * 1024) return false;
    // threads per plane along each dimension: (lines) x (threads per line)
    const int t1 = logL2 + (logL1 - fftu::line_loge(logL1));
    const int t2 = logL1 + (logL2 - fftu::line_loge(logL2));
    const int tmax = std::max(t1, t2);
    if (tmax > 8) return false;
    int logW = std::min(8 - tmax, logA);
    const int64_t L1 = int64_t(1) << logL1, L2 = int64_t(1) << logL2;
    const int64_t PG = L1 * (L2 + 1);
    while (logW > 0 && (L1 + L2 + (int64_t(1) << logW) * PG) * esize > lds_cap()) --logW;
    pd = PassDesc{};
    pd.kind = fftu::kGroup2;
    pd.naxes = 2;
    pd.loglen[0] = logL1;
    pd.loglen[1] = logL2;
    pd.logG = logG;
    pd.logB = 0;
    pd.GB = int64_t(1) << logG;
    pd.logW = logW;
    pd.tiles = int64_t(1) << (logA - logW);
    pd.threads = 1 << (logW + tmax);
    pd.lognmax = lognmax;
    pd.scale = 1.0;
    pd.lds_bytes = uint32_t((L1 + L2 + (int64_t(1) << logW) * PG) * esize);
    return pd.lds_bytes <= lds_cap();
}

// k_pair: two adjacent dimensions (outer lines of 2^logLA, inner lines of 2^logLB,
// B = 2^logB elements after them, A = 2^logA outer blocks) in one strided pass.
// Needs lines of 8..32 points and whole tiles of W columns inside B.
bool make_pair_pass(int logA, int logLA, int logLB, int logB, fftu_dtype dt, int lognmax, PassDesc &pd)
{
    if (knob(FFTU_TUNE_PAIR) == 0) return false;
    if (logLA < fftu::kPairMinLogL || logLA > fftu::kPairMaxLogL || logLB < fftu::kPairMinLogL ||
        logLB > fftu::kPairMaxLogL)
        return false;
    const int esize = dt == FFTU_C128 ? 16 : 8;
    const int lognt = fftu::pair_lognt(logLA, logLB, logB, esize);
    const int logW = fftu::pair_logw(logLA, logLB, lognt);
    if (logB < logW) return false;
    const int64_t tiles = int64_t(1) << (logA + logB - logW);
    if (tiles > fftu::pair_max_tiles(lognt)) return false;
    pd = PassDesc{};
    pd.kind = fftu::kPair;
    pd.threads = 1 << lognt;
    pd.tiles = tiles;
    pd.naxes = 2;
    pd.loglen[0] = logLA;
    pd.loglen[1] = logLB;
    pd.logG = logLA + logLB;
    pd.logB = logB;
    pd.GB = int64_t(1) << (pd.logG + logB);
    pd.logW = logW;
    pd.logBt = logW;
    pd.logTPA = logB - logW;
    pd.lw = fftu::pair_pitch(logLA, logLB, lognt);
    pd.lognmax = lognmax;
    pd.scale = 1.0;
    pd.lds_bytes = fftu::pair_lds_bytes(logLA, logLB, lognt, esize);
    return true;
}

// Passes over the block array (P, m_1, ..., m_d) (2^logP blocks, sides 2^logm[l]) that
// transform lines of 2^len[l] points along each dimension with len[l] > 0, the
// points 2^sub[l] elements apart inside that dimension's own extent (len + sub =
// logm: sub = 0 is the whole side). Innermost dimension first (the order is free:
// the DFT factorises over dimensions, eq. (1.3)). The two innermost dimensions
// share one k_group2 pass when they are whole, contiguous (B = 1) and their planes
// small (allow_group2); further whole dimensions with nothing between them share
// k_pair passes two by two where their lines are short; the rest get one pass each.
std::vector<PassDesc> plan_local(int d, int logP, const int logm[], const int len[], const int sub[], fftu_dtype dt,
                                 int lognmax, bool allow_group2)
{
    std::vector<PassDesc> passes;
    std::vector<int> dims;   // dimensions with lines to transform, innermost first
    for (int l = d - 1; l >= 0; --l)
        if (len[l] > 0) dims.push_back(l);
    auto outer_of = [&](int l) {
        int logA = logP;
        for (int j = 0; j < l; ++j) logA += logm[j];
        return logA;
    };
    auto inner_of = [&](int l) {
        int logB = 0;
        for (int j = l + 1; j < d; ++j) logB += logm[j];
        return logB;
    };
    // whole sides li (inner) and lo (outer) with no elements between them
    auto adjacent = [&](int lo, int li) {
        return sub[lo] == 0 && sub[li] == 0 && inner_of(lo) == logm[li] + inner_of(li);
    };
    size_t first = 0;
    if (dims.size() >= 2 && allow_group2) {
        PassDesc pd;
        const int li = dims[0], lo = dims[1];
        if (inner_of(li) == 0 && adjacent(lo, li) &&
            make_group2_pass(outer_of(lo), len[lo], len[li], dt, lognmax, pd)) {
            passes.push_back(pd);
            first = 2;
        }
    }
    for (size_t i = first; i < dims.size(); ++i) {
        const int l = dims[i];
        PassDesc pd;
        if (i + 1 < dims.size() && adjacent(dims[i + 1], l) &&
            make_pair_pass(outer_of(dims[i + 1]), len[dims[i + 1]], len[l], inner_of(l), dt, lognmax, pd)) {
            passes.push_back(pd);
            ++i;
            continue;
        }
        passes.push_back(make_pass(outer_of(l), {len[l]}, inner_of(l) + sub[l], dt, lognmax));
    }
    return passes;
}

// Superstep 0: the local d-D FFT (every side whole).
// skip_last: leave the innermost dimension out (k_ttranspose runs it).
std::vector<PassDesc> plan_s0(const Geometry &G, fftu_dtype dt, bool skip_last = false)
{
    int len[fftu::kMaxDims], sub[fftu::kMaxDims];
    for (int l = 0; l < G.d; ++l) {
        len[l] = G.logm[l];
        sub[l] = 0;
    }
    if (skip_last) len[G.d - 1] = 0;
    return plan_local(G.d, G.logP, G.logm, len, sub, dt, G.lognmax, !skip_last);
}

// Superstep 2 in unfused form: one pass per grid dimension with p_l > 1; inside a
// destination block the local index splits as (s'_1, t_1, ..., s'_d, t_d).
std::vector<PassDesc> plan_s2(const Geometry &G, fftu_dtype dt, bool skip_last = false)
{
    std::vector<PassDesc> passes;
    for (int l = G.d - 1 - (skip_last ? 1 : 0); l >= 0; --l) {
        if (G.logp[l] == 0) continue;
        int logA = G.logP, logB = G.logq[l];
        for (int j = 0; j < l; ++j) logA += G.logm[j];
        for (int j = l + 1; j < G.d; ++j) logB += G.logm[j];
        passes.push_back(make_pass(logA, {G.logp[l]}, logB, dt, G.lognmax));
    }
    return passes;
}

GridDesc make_grid(const Geometry &G)
{
    GridDesc g{};
    g.d = G.d;
    g.M = int64_t(1) << G.logM;
    g.N = int64_t(1) << G.logN;
    g.lognmax = G.lognmax;
    int ms = 0, ps = 0;
    for (int l = G.d - 1; l >= 0; --l) {
        g.logn[l] = G.logn[l];
        g.logm[l] = G.logm[l];
        g.logp[l] = G.logp[l];
        g.logmstride[l] = ms;
        g.logpstride[l] = ps;
        ms += G.logm[l];
        ps += G.logp[l];
    }
    g.conj_in = g.conj_out = 0;
    g.scale = 1.0;
    return g;
}

// Split of the grid for k_exchange: the dimensions with p_l > 1, in order, become
// nh leading wave dimensions (all of one size 2^lph, at most 2 bits in total) and
// nr trailing register dimensions (all of one size 2^lpr, at most 16 complex128 or
// 32 complex64 values). Returns false when no split has a compiled kernel; the
// unfused path (twiddle, permutation, one pass per grid dimension) is used then.
struct ExchangeSplit {
    int nr = 0, lpr = 0, nh = 0, lph = 0;
    std::vector<int> rdims, hdims;
};

bool reg_part_ok(int nr, int lpr, int rmax)
{
    if (nr == 0) return true;
    if (nr * lpr > rmax) return false;
    return lpr == 1 || (lpr == 2 && nr <= 2) || nr == 1;
}

bool wave_part_ok(int nh, int lph)
{
    return nh == 0 || (nh == 1 && (lph == 1 || lph == 2)) || (nh == 2 && lph == 1);
}

// want_logr >= 0: only splits with exactly that many register bits that k_lastx
// has compiled for a line of 2^logl and 2^lognt threads (the first such split is taken).
bool exchange_split(const Geometry &G, fftu_dtype dt, ExchangeSplit *out, int want_logr = -1, int logl = 0,
                    int lognt = fftu::kLastxLogThreads)
{
    const int rmax = dt == FFTU_C128 ? fftu::kExchangeRegBitsF64 : fftu::kExchangeRegBitsF32;
    std::vector<int> dims;
    for (int l = 0; l < G.d; ++l)
        if (G.logp[l] > 0) dims.push_back(l);
    for (size_t c = 0; c <= dims.size(); ++c) {
        ExchangeSplit sp;
        bool uniform = true;
        for (size_t i = 0; i < dims.size(); ++i) {
            const int lp = G.logp[dims[i]];
            if (i < c) {
                if (sp.nh > 0 && lp != sp.lph) uniform = false;
                sp.lph = lp;
                ++sp.nh;
                sp.hdims.push_back(dims[i]);
            } else {
                if (sp.nr > 0 && lp != sp.lpr) uniform = false;
                sp.lpr = lp;
                ++sp.nr;
                sp.rdims.push_back(dims[i]);
            }
        }
        const int logH = sp.nh * sp.lph, logR = sp.nr * sp.lpr;
        if (!uniform || logH > fftu::kExchangeMaxWaveBits) continue;
        if (!wave_part_ok(sp.nh, sp.lph) || !reg_part_ok(sp.nr, sp.lpr, rmax)) continue;
        if (logH > 0 && logH > logR) continue;
        if (want_logr >= 0 && (logR != want_logr || !fftu::lastx_split_ok(logl, sp.nr, sp.lpr, sp.nh, sp.lph, lognt)))
            continue;
        *out = sp;
        return true;
    }
    return false;
}

ExchangeDesc make_exchange(const Geometry &G, const GridDesc &g, const ExchangeSplit &sp, fftu_dtype dt)
{
    ExchangeDesc ex{};
    ex.g = g;
    ex.nr = sp.nr;
    ex.lpr = sp.lpr;
    ex.nh = sp.nh;
    ex.lph = sp.lph;
    for (size_t i = 0; i < sp.rdims.size(); ++i) ex.rdim[i] = sp.rdims[i];
    for (size_t i = 0; i < sp.hdims.size(); ++i) ex.hdim[i] = sp.hdims[i];
    for (int l = 0; l < G.d; ++l) ex.oshift[l] = G.logq[l] + g.logmstride[l];
    (void)dt;
    const int logR = sp.nr * sp.lpr;   // the LDS swap moves one double (complex128: re, then im) or one complex64
    ex.lds_bytes = sp.nh > 0 ? uint32_t(fftu::kExchangeThreads / 64) * 64u * (1u << logR) * 8u : 0u;
    return ex;
}

// k_lastx: Superstep 0 of every dimension but the innermost as ordinary passes
// (k_pair for adjacent short lines), then the innermost dimension's lines, the
// twiddle, the exchange and the length-p FFTs in one kernel. Taken when k_lastx
// has a kernel for the line length and the grid and a tile's rows exist, and,
// where the innermost two dimensions would share a k_group2 pass, when it saves
// a pass over that plan.
bool plan_lastx(const Geometry &G, const GridDesc &g, fftu_dtype dt, std::vector<PassDesc> &s0x,
                fftu::LastxDesc &lx)
{
    if (knob(FFTU_TUNE_FUSE_LAST) == 0) return false;
    const int li = G.d - 1;
    const int logl = G.logm[li];
    if (logl < fftu::kLastxMinLogL || logl > fftu::kLastxMaxLogL) return false;
    // 512 threads per workgroup, or 1024 where 512 cannot hold a row of every block; the
    // line held as k_line holds it, or (lines of 64) as 16 elements per thread for a
    // split of 16 register sources
    ExchangeSplit sp;
    int lognt = fftu::kLastxLogThreads, loge = -1;
    std::vector<int> cands = {fftu::line_loge(logl)};
    if (fftu::lastx_loge(logl, 4) != cands[0]) cands.push_back(fftu::lastx_loge(logl, 4));
    for (const int cand : cands) {
        lognt = fftu::kLastxLogThreads;
        if (exchange_split(G, dt, &sp, cand, logl, lognt)) {
            loge = cand;
            break;
        }
        lognt = fftu::kLastxMaxLogThreads;
        if (exchange_split(G, dt, &sp, cand, logl, lognt) &&
            fftu::lastx_split_needs_1024(logl, sp.nr, sp.lpr, sp.nh, sp.lph)) {
            loge = cand;
            break;
        }
    }
    if (loge < 0) return false;
    const int logrw = lognt - (logl - loge) - G.logP;
    if (G.logM - logl < logrw) return false;
    const int esize = dt == FFTU_C128 ? 16 : 8;
    const uint32_t lds = fftu::lastx_lds_bytes(logl, loge, esize, lognt);
    if (lds > 160u * 1024u) return false;
    if ((int64_t(1) << (G.logM - logrw - logl)) > fftu::lastx_max_tiles(lognt)) return false;
    // the other dimensions outermost first (measured about 1% faster at 512^3 than
    // innermost first: the longest stride then reads the input buffer)
    std::vector<int> od;   // the other dimensions with m_l > 1, outermost first
    for (int l = 0; l <= G.d - 2; ++l)
        if (G.logm[l] > 0) od.push_back(l);
    auto outer_of = [&](int l) {
        int logA = G.logP;
        for (int j = 0; j < l; ++j) logA += G.logm[j];
        return logA;
    };
    auto inner_of = [&](int l) {
        int logB = 0;
        for (int j = l + 1; j < G.d; ++j) logB += G.logm[j];
        return logB;
    };
    std::vector<PassDesc> passes;
    for (size_t i = 0; i < od.size(); ++i) {
        const int l = od[i];
        PassDesc pd;
        if (i + 1 < od.size() &&
            make_pair_pass(outer_of(l), G.logm[l], G.logm[od[i + 1]], inner_of(od[i + 1]), dt, G.lognmax, pd)) {
            passes.push_back(pd);
            ++i;
            continue;
        }
        passes.push_back(make_pass(outer_of(l), {G.logm[l]}, inner_of(l), dt, G.lognmax));
    }
    const std::vector<PassDesc> full = plan_s0(G, dt);
    if (!full.empty() && full[0].kind == fftu::kGroup2 && passes.size() >= full.size()) return false;
    s0x = passes;
    lx = fftu::LastxDesc{};
    lx.ex = make_exchange(G, g, sp, dt);
    lx.logl = logl;
    lx.lognt = lognt;
    lx.tiles = int64_t(1) << (G.logM - logrw - logl);
    lx.table_lds = fftu::lastx_table_in_lds(logl, loge, G.lognmax, esize, lognt) ? 1 : 0;
    lx.lds_bytes = lds + (lx.table_lds ? uint32_t(esize) << G.lognmax : 0u);
    return true;
}

// MUL: the instantiation that multiplies by a spectrum on the store (convolution
// plans; their table stays in HBM).
std::string lastx_kernel_name(const fftu::LastxDesc &lx, fftu_dtype dt, bool mul = false)
{
    const std::string t = dt == FFTU_C128 ? "double" : "float";
    auto s = [](int v) { return std::to_string(v); };
    const ExchangeDesc &ex = lx.ex;
    const int lph = ex.nh ? ex.lph : 0, lpr = ex.nr ? ex.lpr : 0;
    return "fftu::k_lastx<" + t + ", " + s(lx.logl) + ", " + s(ex.nr) + ", " + s(lpr) + ", " + s(ex.nh) + ", " +
           s(lph) + (mul ? ", true, false, " : (lx.table_lds ? ", false, true, " : ", false, false, ")) + s(lx.lognt) +
           ">";
}

// omega_L^j = exp(-2 pi i j / L) for j in [L], L = 2^logL, in FP64. Each value is
// reduced to the first octant by exact symmetries before cosl/sinl, so the table is
// exactly symmetric and exact at the multiples of L/8's quarter turns.
void cos_sin(int64_t L, int64_t j, long double &c, long double &s)
{
    if (L >= 2 && j >= L / 2) {
        cos_sin(L, j - L / 2, c, s);
        c = -c;
        s = -s;
        return;
    }
    if (L >= 4 && j >= L / 4) {
        long double c2, s2;
        cos_sin(L, j - L / 4, c2, s2);
        c = -s2;
        s = c2;
        return;
    }
    if (L >= 8 && j > L / 8) {
        const long double th = 2.0L * 3.14159265358979323846264338327950288L * (long double)(L / 4 - j) / (long double)L;
        c = sinl(th);
        s = cosl(th);
        return;
    }
    if (j == 0) {
        c = 1.0L;
        s = 0.0L;
        return;
    }
    const long double th = 2.0L * 3.14159265358979323846264338327950288L * (long double)j / (long double)L;
    c = cosl(th);
    s = sinl(th);
}

std::vector<double> make_table_f64(int logL)
{
    const int64_t L = int64_t(1) << logL;
    std::vector<double> t(size_t(2 * L));
    for (int64_t j = 0; j < L; ++j) {
        long double c, s;
        cos_sin(L, j, c, s);
        t[size_t(2 * j)] = double(c);
        t[size_t(2 * j + 1)] = -double(s);
    }
    return t;
}

// cos and sin of 2 pi j / L for any L: the half-turn symmetry (j > L/2 gives the
// conjugate of L - j) is exact for every L, the quarter points are exact, and an
// L divisible by 8 takes the octant reduction of cos_sin, so powers of two get
// exactly the entries of make_table_f64.
void cos_sin_general(int64_t L, int64_t j, long double &c, long double &s)
{
    if (L % 8 == 0) {
        cos_sin(L, j, c, s);
        return;
    }
    if (2 * j > L) {
        cos_sin_general(L, L - j, c, s);
        s = -s;
        return;
    }
    if (j == 0) {
        c = 1.0L;
        s = 0.0L;
        return;
    }
    if (2 * j == L) {
        c = -1.0L;
        s = 0.0L;
        return;
    }
    if (4 * j == L) {
        c = 0.0L;
        s = 1.0L;
        return;
    }
    const long double th = 2.0L * 3.14159265358979323846264338327950288L * (long double)j / (long double)L;
    c = cosl(th);
    s = sinl(th);
}

// omega_T^j = exp(-2 pi i j / T), j in [T], interleaved FP64.
std::vector<double> make_table_general(int64_t T)
{
    std::vector<double> t(size_t(2 * T));
    for (int64_t j = 0; j < T; ++j) {
        long double c, s;
        cos_sin_general(T, j, c, s);
        t[size_t(2 * j)] = double(c);
        t[size_t(2 * j + 1)] = -double(s);
    }
    return t;
}

// Radix stages of a mixed-radix line: 8s, then a 4 or a 2, then 7s, 5s, 3s.
// The largest power-of-two radix comes from the knob FFTU_TUNE_MIXED_RADIX (2, 4 or
// 8; default 8): radix R stages first, then one 4 or 2 for what is left of the
// power of two, then 7s, 5s, 3s.
int mixed_radices(int64_t L, int32_t *out)
{
    const int kr = knob(FFTU_TUNE_MIXED_RADIX);
    const int R = kr >= 8 || kr < 2 ? 8 : (kr >= 4 ? 4 : 2);
    int n = 0;
    while (L % R == 0 && n < fftu::kMixedMaxStages) {
        out[n++] = R;
        L /= R;
    }
    if (R > 4 && L % 4 == 0 && n < fftu::kMixedMaxStages) {
        out[n++] = 4;
        L /= 4;
    }
    if (R > 2 && L % 2 == 0 && n < fftu::kMixedMaxStages) {
        out[n++] = 2;
        L /= 2;
    }
    for (int f : {7, 5, 3})
        while (L % f == 0 && n < fftu::kMixedMaxStages) {
            out[n++] = f;
            L /= f;
        }
    return L == 1 ? n : -1;
}

bool make_mixed_pass(int64_t A, int64_t L, int64_t B, fftu_dtype dt, int64_t T, fftu::MixedPassDesc &pd)
{
    pd = fftu::MixedPassDesc{};
    const int64_t esize = dt == FFTU_C128 ? 16 : 8;
    const int64_t cap = 64 * 1024;
    pd.nstages = mixed_radices(L, pd.radix);
    if (pd.nstages < 0) return false;
    const int kt = knob(FFTU_TUNE_MIXED_TILE_LOG);
    // elements per tile: at most what the threads hold while they prefetch the next tile
    const int64_t held = int64_t(dt == FFTU_C128 ? fftu::kMixedPreF64 : fftu::kMixedPreF32) * fftu::kMixedThreads;
    const int64_t target = std::min(kt >= 9 ? (int64_t(1) << kt) : held, held);
    if (L > held) return false;
    // strided lines: odd pitch in LDS, so that lanes over consecutive lines hit different banks;
    // contiguous lines are loaded along the line, pitch L
    const int64_t pitch = (B == 1 || L % 2) ? L : L + 1;
    int64_t W = 1;
    while (W * 2 * L <= target && W < fftu::kMixedMaxW) W *= 2;
    while (W > 1 && W / 2 >= A * B) W /= 2;                  // no tile much wider than the lines there are
    auto lds = [&](int64_t w) { return (2 * w * pitch + L) * esize; };
    while (W > 1 && lds(W) > cap) W /= 2;
    if (lds(W) > cap) return false;
    pd.A = A;
    pd.B = B;
    pd.L = int32_t(L);
    pd.W = int32_t(W);
    pd.logW = ilog2(W);
    pd.pitch = pitch;
    pd.tiles = (A * B + W - 1) / W;
    pd.tstep = T / L;
    pd.scale = 1.0;
    pd.lds_bytes = uint32_t(lds(W));
    return true;
}

struct MixedPlan {
    std::vector<fftu::MixedPassDesc> s0, s2;
    fftu::MixedGridDesc g{};
    int64_t T = 1;
    bool fused = false;   // k_mexchange: twiddle, Put and Superstep 2 in one kernel
    bool mx = false;      // the fused form on k_mxexchange (every grid side a power of two)
    fftu::MxSplit mxs{};
};

bool plan_mixed(int d, const int64_t n[], const int64_t p[], fftu_dtype dt, MixedPlan &mp)
{
    mp = MixedPlan{};
    fftu::MixedGridDesc &g = mp.g;
    g.d = d;
    g.N = 1;
    g.P = 1;
    for (int l = 0; l < d; ++l) {
        g.n[l] = int32_t(n[l]);
        g.p[l] = int32_t(p[l]);
        g.m[l] = int32_t(n[l] / p[l]);
        g.q[l] = int32_t(n[l] / p[l] / p[l]);
        g.N *= n[l];
        g.P *= p[l];
        mp.T = lcm64(mp.T, n[l]);
    }
    g.M = g.N / g.P;
    g.T = mp.T;
    for (int l = 0; l < d; ++l) g.tstep[l] = mp.T / n[l];
    g.scale = 1.0;
    // Superstep 0: one pass per local dimension, innermost first: (P prod_{j<l} m_j, m_l, prod_{j>l} m_j).
    for (int l = d - 1; l >= 0; --l) {
        if (g.m[l] == 1) continue;
        int64_t A = g.P, B = 1;
        for (int j = 0; j < l; ++j) A *= g.m[j];
        for (int j = l + 1; j < d; ++j) B *= g.m[j];
        fftu::MixedPassDesc pd;
        if (!make_mixed_pass(A, g.m[l], B, dt, mp.T, pd)) return false;
        mp.s0.push_back(pd);
    }
    // Superstep 2: local index k_l = t_l + k'_l q_l, lines along k'_l:
    // (P prod_{j<l} m_j, p_l, q_l prod_{j>l} m_j).
    for (int l = d - 1; l >= 0; --l) {
        if (g.p[l] == 1) continue;
        int64_t A = g.P, B = g.q[l];
        for (int j = 0; j < l; ++j) A *= g.m[j];
        for (int j = l + 1; j < d; ++j) B *= g.m[j];
        fftu::MixedPassDesc pd;
        if (!make_mixed_pass(A, g.p[l], B, dt, mp.T, pd)) return false;
        mp.s2.push_back(pd);
    }
    mp.fused = g.P <= fftu::kMexMaxP;
    for (int l = 0; l < d; ++l) mp.fused = mp.fused && fftu::mexchange_radix_ok(g.p[l]);
    // every grid side a power of two: the register split of the power-of-two exchange
    bool pow2_grid = g.P > 1;
    for (int l = 0; l < d; ++l) pow2_grid = pow2_grid && is_pow2(p[l]);
    if (pow2_grid && g.N < (int64_t(1) << 31)) {
        Geometry G{};
        G.d = d;
        for (int l = 0; l < d; ++l) G.logp[l] = ilog2(p[l]);
        ExchangeSplit sp;
        if (exchange_split(G, dt, &sp)) {
            mp.mx = true;
            mp.fused = true;
            mp.mxs = fftu::MxSplit{};
            mp.mxs.nr = sp.nr;
            mp.mxs.lpr = sp.lpr;
            mp.mxs.nh = sp.nh;
            mp.mxs.lph = sp.lph;
            for (size_t i = 0; i < sp.rdims.size(); ++i) mp.mxs.rdim[i] = sp.rdims[i];
            for (size_t i = 0; i < sp.hdims.size(); ++i) mp.mxs.hdim[i] = sp.hdims[i];
            const int logR = sp.nr * sp.lpr;
            mp.mxs.lds_bytes = sp.nh > 0 ? uint32_t(fftu::kExchangeThreads / 64) * 64u * (1u << logR) * 8u : 0u;
        }
    }
    return true;
}

void fill_info_mixed(const MixedPlan &mp, fftu_dtype dt, fftu_plan_info *info)
{
    const uint64_t esize = dt == FFTU_C128 ? 16 : 8;
    *info = fftu_plan_info{};
    info->d = mp.g.d;
    info->N = mp.g.N;
    info->P = mp.g.P;
    info->M = mp.g.M;
    info->s0_kernels = int32_t(mp.s0.size());
    info->exchange_fused = mp.fused ? 1 : 0;
    // fused: one k_mexchange; else twiddle + permutation in one kernel, then the passes
    info->s2_kernels = mp.fused ? 0 : int32_t(1 + mp.s2.size());
    info->launches = info->s0_kernels + (mp.fused ? 1 : info->s2_kernels);
    info->workspace_bytes = uint64_t(mp.g.N) * esize;
    info->table_bytes = uint64_t(mp.T) * esize;
    info->supersteps = 1;
}

// Grids beyond p_max: every dimension's levels run side by side (Algorithm 2.3's
// combination of Algorithm 2.2 per dimension), H = max_l (h_l + 1) communication
// supersteps. Computation phase c: the local F_{m_l} of every dimension with
// levels left (c <= h_l), and the length-p_h FFTs of every dimension whose last
// Put was superstep c - 1 (local index s' q + t, lines along s'). Superstep c:
// one k_gput with each dimension's Put of level c (none for finished dimensions).
//
// When every side is a power of two the phases run on the power-of-two pass kernels
// (k_line, k_long, k_group2, k_pair: the same passes as Superstep 0 of the cyclic
// path), else on k_mline.
struct GcPlan {
    int H = 0;
    int64_t T = 1, N = 1, P = 1, M = 1;
    bool pow2 = false;
    int last_logg = 0;   // > 0: k_gplast runs the last Put and phase H (2^last_logg elements per thread)
    std::vector<std::vector<fftu::MixedPassDesc>> phase;   // mixed radix
    std::vector<std::vector<PassDesc>> phase2;             // powers of two
    std::vector<fftu::GroupPutDesc> put;
    size_t phase_size(size_t c) const { return pow2 ? phase2[c].size() : phase[c].size(); }
    // launches of the whole transform
    int launches() const
    {
        int k = H;
        for (int c = 0; c <= H; ++c) k += int(phase_size(size_t(c)));
        return last_logg > 0 ? k - int(phase_size(size_t(H))) : k;
    }
};

// A pass that its kernel can run (the tile pass has no check of its own).
bool pass_fits(const PassDesc &pd) { return pd.kind != fftu::kTilePass || int64_t(pd.lds_bytes) <= lds_cap(); }

bool plan_gc(int d, const int64_t n[], const int64_t p[], fftu_dtype dt, GcPlan &gp)
{
    gp = GcPlan{};
    GcLevels lv[fftu::kMaxDims];
    int64_t m[fftu::kMaxDims];
    for (int l = 0; l < d; ++l) {
        if (!gc_levels(n[l], p[l], lv[l])) return false;
        m[l] = n[l] / p[l];
        gp.H = std::max(gp.H, lv[l].h + 1);
        gp.N *= n[l];
        gp.P *= p[l];
        gp.T = lcm64(gp.T, n[l]);
    }
    gp.M = gp.N / gp.P;
    bool all_pow2 = true;
    for (int l = 0; l < d; ++l) all_pow2 = all_pow2 && is_pow2(n[l]);
    if (all_pow2) {
        int logm[fftu::kMaxDims], logP = 0, lognmax = 0;
        for (int l = 0; l < d; ++l) {
            logm[l] = ilog2(m[l]);
            logP += ilog2(p[l]);
            lognmax = std::max(lognmax, ilog2(n[l]));
        }
        bool ok = true;
        for (int c = 0; c <= gp.H && ok; ++c) {
            int len[fftu::kMaxDims], sub[fftu::kMaxDims];
            for (int l = 0; l < d; ++l) {
                len[l] = sub[l] = 0;
                if (c <= lv[l].h) {
                    len[l] = logm[l];                                  // level c's local F_m
                } else if (c == lv[l].h + 1) {
                    len[l] = ilog2(lv[l].p[lv[l].h]);                  // level h's length-p_h FFTs
                    sub[l] = logm[l] - len[l];
                }
            }
            std::vector<PassDesc> ph = plan_local(d, logP, logm, len, sub, dt, lognmax, true);
            for (const PassDesc &pd : ph) ok = ok && pass_fits(pd);
            gp.phase2.push_back(ph);
        }
        if (ok) {
            gp.pow2 = true;
        } else {
            gp.phase2.clear();
        }
    }
    for (int c = 0; c <= gp.H && !gp.pow2; ++c) {
        std::vector<fftu::MixedPassDesc> ph;
        for (int l = d - 1; l >= 0; --l) {
            int64_t A = gp.P, B = 1;
            for (int j = 0; j < l; ++j) A *= m[j];
            for (int j = l + 1; j < d; ++j) B *= m[j];
            int64_t L = 1;
            if (c <= lv[l].h) {
                L = m[l];                              // level c's local F_m
            } else if (c == lv[l].h + 1) {
                L = lv[l].p[lv[l].h];                  // level h's length-p_h FFTs
                B *= m[l] / L;
            }
            if (L == 1) continue;
            fftu::MixedPassDesc pd;
            if (!make_mixed_pass(A, L, B, dt, gp.T, pd)) return false;
            ph.push_back(pd);
        }
        gp.phase.push_back(ph);
    }
    for (int c = 0; c < gp.H; ++c) {
        fftu::GroupPutDesc g{};
        g.d = d;
        g.N = gp.N;
        g.M = gp.M;
        g.T = gp.T;
        g.twiddle = 1;
        g.permute = 1;
        g.scale = 1.0;
        for (int l = 0; l < d; ++l) {
            fftu::GroupPutDim &D = g.dim[l];
            D.m = int32_t(m[l]);
            D.p = int32_t(p[l]);
            if (c > lv[l].h) continue;                 // mode 0: this dimension is done
            D.mode = c < lv[l].h ? 1 : 2;
            D.pi = int32_t(lv[l].p[c]);
            D.ni = int32_t(lv[l].n[c]);
            D.tstep = gp.T / lv[l].n[c];
            if (D.mode == 1) {
                D.pn = int32_t(lv[l].p[c] / m[l]);
            } else {
                D.q = int32_t(m[l] / lv[l].p[c]);
                int64_t mh = 1;
                for (int i = 0; i < lv[l].h; ++i) mh *= m[l];
                D.mh = int32_t(mh);
                D.h = lv[l].h;
            }
        }
        gp.put.push_back(g);
    }
    // The last Put (every dimension in mode 2 or 0) and phase H (the length-p_h FFTs of
    // the mode-2 dimensions) in one k_gplast pass when the FFTs of one thread fit in
    // its registers.
    if (gp.pow2) {
        int logg = 0;
        for (int l = 0; l < d; ++l)
            if (gp.put[size_t(gp.H - 1)].dim[l].mode == 2) logg += ilog2(gp.put[size_t(gp.H - 1)].dim[l].pi);
        if (logg >= 1 && logg <= fftu::kGplastMaxLogG && gp.N < (int64_t(1) << 31) && gp.T < (int64_t(1) << 26))
            gp.last_logg = logg;
    }
    return true;
}

void fill_info_gc(const GcPlan &gp, int d, fftu_dtype dt, fftu_plan_info *info)
{
    const uint64_t esize = dt == FFTU_C128 ? 16 : 8;
    *info = fftu_plan_info{};
    info->d = d;
    info->N = gp.N;
    info->P = gp.P;
    info->M = gp.M;
    info->s0_kernels = int32_t(gp.phase_size(0));
    info->exchange_fused = 0;
    info->launches = gp.launches();
    info->s2_kernels = info->launches - info->s0_kernels;
    info->supersteps = gp.H;
    info->workspace_bytes = uint64_t(gp.N) * esize;
    info->table_bytes = uint64_t(gp.T) * esize;
}

// The unfused exchange of a grid with every q_l = 1 (m = p, so M = P) is a transpose
// of the P x M matrix of blocks: k_ttranspose applies the twiddle and moves 64 x 64
// tiles in one pass, instead of k_twiddle and k_permute.
bool transpose_exchange(const Geometry &G)
{
    for (int l = 0; l < G.d; ++l)
        if (G.logq[l] != 0) return false;
    return G.logM >= 6 && 2 * G.logM - 12 <= 31 - 8;
}

// log2 of the innermost side when k_ttranspose also takes its FFTs (2..32 points), else 0
int transpose_fused_ld(const Geometry &G)
{
    if (!transpose_exchange(G)) return 0;
    const int ld = G.logm[G.d - 1];
    return ld >= 1 && ld <= 5 ? ld : 0;
}

void fill_info(const Geometry &G, const std::vector<PassDesc> &s0, bool fused, size_t nS2, fftu_dtype dt,
               fftu_plan_info *info, bool lastx = false)
{
    const uint64_t esize = dt == FFTU_C128 ? 16 : 8;
    info->d = G.d;
    info->N = int64_t(1) << G.logN;
    info->P = int64_t(1) << G.logP;
    info->M = int64_t(1) << G.logM;
    info->s0_kernels = int32_t(s0.size());
    info->exchange_fused = fused ? 1 : 0;
    info->s2_kernels = fused ? 0 : int32_t((transpose_exchange(G) ? 1 : 2) + nS2);
    if (!fused && transpose_fused_ld(G) > 0) {
        // k_ttranspose takes the innermost dimension's passes of Supersteps 0 and 2
        info->s0_kernels = int32_t(plan_s0(G, dt, true).size());
        info->s2_kernels = int32_t(1 + plan_s2(G, dt, true).size());
    }
    info->launches = info->s0_kernels + (fused ? 1 : info->s2_kernels);
    if (lastx) info->exchange_fused = 2;   // s0 holds the passes before k_lastx
    info->workspace_bytes = uint64_t(info->N) * esize;
    info->table_bytes = (uint64_t(1) << G.lognmax) * esize;
    info->supersteps = 1;
}

// Profiler name of the kernel that runs a pass (matches the template arguments).
std::string pass_kernel_name(const PassDesc &pd, fftu_dtype dt)
{
    const std::string t = dt == FFTU_C128 ? "double" : "float";
    if (pd.kind == fftu::kGroup2)
        return "fftu::k_group2<" + t + ", " + std::to_string(pd.loglen[0]) + ", " + std::to_string(pd.loglen[1]) + ">";
    if (pd.kind == fftu::kPair)
        return "fftu::k_pair<" + t + ", " + std::to_string(pd.loglen[0]) + ", " + std::to_string(pd.loglen[1]) + ", " +
               std::to_string(__builtin_ctz(unsigned(pd.threads))) + ">";
    if (pd.kind == fftu::kLong)
        return "fftu::k_long<" + t + ", " + std::to_string(pd.loglen[0]) + ", " + std::to_string(pd.logB) + ">";
    if (pd.kind == fftu::kTilePass) return "fftu::k_pass<" + t + ">";
    return "fftu::k_line<" + t + ", " + std::to_string(pd.loglen[0]) + ", " + std::to_string(pd.kind) + ">";
}

std::string exchange_kernel_name(const ExchangeDesc &ex, fftu_dtype dt)
{
    const std::string t = dt == FFTU_C128 ? "double" : "float";
    auto s = [](int v) { return std::to_string(v); };
    const int lph = ex.nh ? ex.lph : 0, lpr = ex.nr ? ex.lpr : 0;
    return "fftu::k_exchange<" + t + ", " + s(ex.nr) + ", " + s(lpr) + ", " + s(ex.nh) + ", " + s(lph) + ">";
}

fftu_status from_hip(hipError_t e)
{
    if (e == hipSuccess) return FFTU_SUCCESS;
    if (e == hipErrorOutOfMemory) return FFTU_ERROR_OUT_OF_MEMORY;
    return FFTU_ERROR_DEVICE;
}

// Records the next timing event of the current call, if timing is on.
struct Marker {
    fftu_plan_s *pl;
    hipStream_t stream;
    int slot = -1;
    int next = 0;
    Marker(fftu_plan_s *p, hipStream_t s) : pl(p), stream(s)
    {
        if (pl->timing_max > 0 && pl->timing_used < pl->timing_max) slot = pl->timing_used++;
    }
    void mark()
    {
        if (slot >= 0 && next <= pl->launches)
            (void)hipEventRecord(pl->events[size_t(slot) * size_t(pl->launches + 1) + size_t(next++)], stream);
    }
};

// Run the passes of one superstep from `in` into `out`: the first pass reads `in`,
// the rest work in place on `out`. conj_first / conj_last conjugate the chain's
// first load and last store; scale_last multiplies the last store.
fftu_status run_passes(const fftu_plan_s *pl, const std::vector<PassDesc> &passes, const void *in, void *out,
                       int conj_first, int conj_last, double scale_last, hipStream_t stream,
                       Marker *mk = nullptr)
{
    if (passes.empty()) {
        if (in != out)
            return from_hip(hipMemcpyAsync(out, in, pl->grid.N * pl->esize, hipMemcpyDeviceToDevice, stream));
        return FFTU_SUCCESS;
    }
    const void *src = in;
    for (size_t i = 0; i < passes.size(); ++i) {
        PassDesc pd = passes[i];
        pd.conj_in = (i == 0) ? conj_first : 0;
        pd.conj_out = (i + 1 == passes.size()) ? conj_last : 0;
        pd.scale = (i + 1 == passes.size()) ? scale_last : 1.0;
        hipError_t e = fftu::launch_pass(pl->prec, src, out, pd, pl->table, stream);
        if (e != hipSuccess) return from_hip(e);
        if (mk) mk->mark();
        src = out;
    }
    return FFTU_SUCCESS;
}

// Device buffers hold whole complex elements: 8- or 16-byte aligned.
bool aligned(const void *p, size_t esize) { return (reinterpret_cast<uintptr_t>(p) & (esize - 1)) == 0; }

fftu_status check_exec_args(const fftu_plan_s *plan, const void *in, const void *out)
{
    if (!plan || !in || !out || plan->is_batch || plan->real || plan->r2r) return FFTU_ERROR_INVALID_VALUE;
    if (!aligned(in, plan->esize) || !aligned(out, plan->esize)) return FFTU_ERROR_INVALID_VALUE;
    if (in != out) {
        const char *a = static_cast<const char *>(in);
        const char *b = static_cast<const char *>(out);
        const size_t bytes = size_t(plan->grid.N) * plan->esize;
        if (a < b + bytes && b < a + bytes) return FFTU_ERROR_INVALID_VALUE;   // partial overlap
    }
    return FFTU_SUCCESS;
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
bool batch_exchange_ok(const ExchangeSplit &sp)
{
    if (sp.nh != 0) return false;
    const int key = sp.nr * 8 + sp.lpr;
    return key == 0 || key == 9 || key == 17 || key == 25 || key == 33 || key == 10 || key == 18 || key == 11 ||
           key == 12;
}

void free_batch(fftu_plan_s *pl)
{
    for (void *ptr : {pl->dstages, pl->dstarts, pl->ddep, pl->ddone, pl->dnext, pl->derror, pl->dbind})
        if (ptr) (void)hipFree(ptr);
    pl->dstages = pl->dstarts = pl->ddep = pl->ddone = pl->dnext = pl->derror = pl->dbind = nullptr;
}

// The buffers of a batch call: none NULL, each aligned to the element size,
// in[f] and out[f] either equal or disjoint, and no output overlapping another
// transform's input or output. O(count log count).
fftu_status check_batch_args(const fftu_plan_s *pl, const void *const in[], void *const out[])
{
    if (!pl || !pl->is_batch || !in || !out) return FFTU_ERROR_INVALID_VALUE;
    struct Span {
        uintptr_t lo, hi;
        int f;
    };
    std::vector<Span> outs(size_t(pl->count));
    for (int f = 0; f < pl->count; ++f) {
        if (!in[f] || !out[f] || !aligned(in[f], pl->esize) || !aligned(out[f], pl->esize))
            return FFTU_ERROR_INVALID_VALUE;
        const uintptr_t o = reinterpret_cast<uintptr_t>(out[f]);
        outs[size_t(f)] = {o, o + uintptr_t(pl->member_N[size_t(f)]) * pl->esize, f};
    }
    std::sort(outs.begin(), outs.end(), [](const Span &a, const Span &b) { return a.lo < b.lo; });
    for (size_t i = 1; i < outs.size(); ++i)
        if (outs[i].lo < outs[i - 1].hi) return FFTU_ERROR_INVALID_VALUE;   // two outputs overlap
    // the outputs are disjoint and sorted, so their ends are sorted too
    for (int f = 0; f < pl->count; ++f) {
        const uintptr_t lo = reinterpret_cast<uintptr_t>(in[f]);
        const uintptr_t hi = lo + uintptr_t(pl->member_N[size_t(f)]) * pl->esize;
        auto it = std::upper_bound(outs.begin(), outs.end(), lo, [](uintptr_t v, const Span &s) { return v < s.hi; });
        for (; it != outs.end() && it->lo < hi; ++it)
            if (it->f != f || it->lo != lo) return FFTU_ERROR_INVALID_VALUE;   // only in[f] == out[f] may meet
    }
    return FFTU_SUCCESS;
}

// Workspace of an external batch (bytes, 256-aligned pieces): the members'
// workspaces, then the image the host stages (stages, starts, dep, bind: the
// staging buffer holds [stages, staged) of this layout), then the counters that
// k_batch_reset clears.
struct BatchWsLayout {
    size_t stages = 0, starts = 0, dep = 0, bind = 0, staged = 0, done = 0, next = 0, error = 0, total = 0;
};

BatchWsLayout batch_ws_layout(const fftu_plan_s *pl)
{
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t K = pl->hstages.size();
    int64_t Ntot = 0;
    for (int64_t v : pl->member_N) Ntot += v;
    BatchWsLayout L;
    L.stages = up(size_t(Ntot) * pl->esize);
    L.starts = up(L.stages + K * sizeof(fftu::BatchStage));
    L.dep = up(L.starts + (K + 1) * sizeof(int64_t));
    L.bind = up(L.dep + K * sizeof(int32_t));
    L.staged = L.bind + size_t(pl->count) * sizeof(fftu::BatchBind);
    L.done = up(L.staged);
    L.next = up(L.done + K * sizeof(int32_t));
    L.error = L.next + sizeof(unsigned long long);
    L.total = up(L.error + sizeof(int32_t));
    return L;
}

// Write the buffers into the device list on `stream` (k_batch_bind launches that
// carry the pointers as arguments): stream-ordered, no host wait.
fftu_status enqueue_bind(const fftu_plan_s *pl, const void *const in[], void *const out[], hipStream_t stream)
{
    for (int first = 0; first < pl->count; first += fftu::kBindChunk) {
        fftu::BindChunk c{};
        c.first = first;
        c.count = std::min(fftu::kBindChunk, pl->count - first);
        for (int i = 0; i < c.count; ++i) c.b[i] = {in[first + i], out[first + i]};
        hipError_t e = fftu::launch_batch_bind(static_cast<fftu::BatchBind *>(pl->dbind), c, stream);
        if (e != hipSuccess) return from_hip(e);
    }
    return FFTU_SUCCESS;
}

bool same_binding(const fftu_plan_s *pl, const void *const in[], void *const out[])
{
    if (pl->bound_in.size() != size_t(pl->count)) return false;
    for (int f = 0; f < pl->count; ++f)
        if (pl->bound_in[size_t(f)] != in[f] || pl->bound_out[size_t(f)] != out[f]) return false;
    return true;
}

// The reset kernel, then the persistent kernel; with a marker, timing events
// bracket each of the two launches.
fftu_status enqueue_batch(fftu_plan_s *pl, hipStream_t stream, Marker *mk = nullptr)
{
    fftu::BatchDesc bd{};
    bd.nstages = int32_t(pl->hstages.size());
    bd.wait_limit = pl->batch_wait_ticks;
    bd.nitems = pl->batch_items;
    bd.stages = static_cast<const fftu::BatchStage *>(pl->dstages);
    bd.starts = static_cast<const int64_t *>(pl->dstarts);
    bd.dep = static_cast<const int32_t *>(pl->ddep);
    bd.done = static_cast<int32_t *>(pl->ddone);
    bd.next = static_cast<unsigned long long *>(pl->dnext);
    bd.error = static_cast<int32_t *>(pl->derror);
    bd.bind = static_cast<const fftu::BatchBind *>(pl->dbind);
    if (mk) mk->mark();
    hipError_t e = fftu::launch_batch_reset(bd, stream);
    if (e != hipSuccess) return from_hip(e);
    if (mk) mk->mark();
    e = fftu::launch_batch(pl->prec, bd, pl->table, pl->batch_blocks, pl->batch_lds, stream);
    if (e != hipSuccess) return from_hip(e);
    if (mk) mk->mark();
    return FFTU_SUCCESS;
}

fftu_status execute_with(fftu_plan_s *plan, const void *in, void *out, void *ws, hipStream_t stream,
                         const void *mul = nullptr, Marker *outer = nullptr);

}  // namespace

struct fftu_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    fftu_plan_s *batch = nullptr;            // batch graphs: the plan, whose device list each replay rebinds
    std::vector<const void *> in;            // the buffers captured (batch graphs)
    std::vector<void *> out;
};

namespace {

// Twiddle tables shared by external plans: one per (device, precision), the
// table omega_{2^K}^j, j in [2^K], for the largest K asked for so far (at least
// 2^12). A plan indexes it with its own lognmax = K; omega_n^j = omega_{2^K}^{j 2^K / n}
// and the table's construction gives bitwise the same values for every K (the
// angles reduce to the same fractions), so results do not depend on K. A table
// that is outgrown is kept until the process ends: plans made earlier still use it.
struct SharedTable {
    int device;
    Precision prec;
    int logK;
    void *ptr;
};
std::mutex g_tables_mutex;
std::vector<SharedTable> g_tables;

hipError_t upload_table(void **ptr, int logK, fftu_dtype dtype)
{
    const std::vector<double> t64 = make_table_f64(logK);
    const uint64_t bytes = (uint64_t(1) << logK) * (dtype == FFTU_C128 ? 16 : 8);
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) return e;
    if (dtype == FFTU_C128) {
        e = hipMemcpy(*ptr, t64.data(), bytes, hipMemcpyHostToDevice);
    } else {
        std::vector<float> t32(t64.size());
        for (size_t i = 0; i < t64.size(); ++i) t32[i] = float(t64[i]);   // rounded once
        e = hipMemcpy(*ptr, t32.data(), bytes, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        (void)hipFree(*ptr);
        *ptr = nullptr;
    }
    return e;
}

hipError_t upload_table_general(void **ptr, int64_t T, fftu_dtype dtype)
{
    const std::vector<double> t64 = make_table_general(T);
    const uint64_t bytes = uint64_t(T) * (dtype == FFTU_C128 ? 16 : 8);
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) return e;
    if (dtype == FFTU_C128) {
        e = hipMemcpy(*ptr, t64.data(), bytes, hipMemcpyHostToDevice);
    } else {
        std::vector<float> t32(t64.size());
        for (size_t i = 0; i < t64.size(); ++i) t32[i] = float(t64[i]);   // rounded once
        e = hipMemcpy(*ptr, t32.data(), bytes, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        (void)hipFree(*ptr);
        *ptr = nullptr;
    }
    return e;
}

// Shared tables of mixed-radix external plans: one per (device, precision, T), exact T.
struct SharedTableT {
    int device;
    Precision prec;
    int64_t T;
    void *ptr;
};
std::vector<SharedTableT> g_tables_T;

hipError_t shared_table_exact(int device, fftu_dtype dtype, int64_t T, void **ptr)
{
    const Precision prec = dtype == FFTU_C128 ? Precision::F64 : Precision::F32;
    std::lock_guard<std::mutex> lock(g_tables_mutex);
    for (const SharedTableT &t : g_tables_T)
        if (t.device == device && t.prec == prec && t.T == T) {
            *ptr = t.ptr;
            return hipSuccess;
        }
    void *p = nullptr;
    hipError_t e = upload_table_general(&p, T, dtype);
    if (e != hipSuccess) return e;
    g_tables_T.push_back({device, prec, T, p});
    *ptr = p;
    return hipSuccess;
}

hipError_t shared_table(int device, fftu_dtype dtype, int need_log, void **ptr, int *logK)
{
    const Precision prec = dtype == FFTU_C128 ? Precision::F64 : Precision::F32;
    std::lock_guard<std::mutex> lock(g_tables_mutex);
    SharedTable *best = nullptr;
    for (SharedTable &t : g_tables)
        if (t.device == device && t.prec == prec && (!best || t.logK > best->logK)) best = &t;
    if (best && best->logK >= need_log) {
        *ptr = best->ptr;
        *logK = best->logK;
        return hipSuccess;
    }
    const int K = std::max(need_log, 12);
    void *p = nullptr;
    hipError_t e = upload_table(&p, K, dtype);
    if (e != hipSuccess) return e;
    g_tables.push_back({device, prec, K, p});
    *ptr = p;
    *logK = K;
    return hipSuccess;
}

fftu_plan_s *build_mixed_plan(int d, const int64_t n[], const int64_t p[], fftu_dtype dtype, fftu_direction direction,
                              bool external, int device)
{
    MixedPlan mp;
    if (!plan_mixed(d, n, p, dtype, mp)) {
        record(FFTU_ERROR_UNSUPPORTED);
        return nullptr;
    }
    fftu_plan_s *pl = new (std::nothrow) fftu_plan_s();
    if (!pl) {
        record(FFTU_ERROR_OUT_OF_MEMORY);
        return nullptr;
    }
    pl->d = d;
    for (int l = 0; l < d; ++l) {
        pl->n[l] = n[l];
        pl->p[l] = p[l];
    }
    pl->dtype = dtype;
    pl->dir = direction;
    pl->prec = dtype == FFTU_C128 ? Precision::F64 : Precision::F32;
    pl->esize = dtype == FFTU_C128 ? 16 : 8;
    pl->device = device;
    pl->external = external;
    pl->mixed = true;
    pl->ms0 = mp.s0;
    pl->ms2 = mp.s2;
    pl->mg = mp.g;
    pl->table_T = mp.T;
    pl->grid.N = mp.g.N;
    pl->grid.M = mp.g.M;
    pl->grid.d = d;
    pl->mfused = mp.fused;
    pl->mx = mp.mx;
    pl->mxs = mp.mxs;
    pl->launches = int(mp.s0.size() + 1 + (mp.fused ? 0 : mp.s2.size()));
    const std::string t = dtype == FFTU_C128 ? "double" : "float";
    for (size_t i = 0; i < mp.s0.size(); ++i) pl->launch_names.push_back("fftu::k_mline<" + t + ">");
    if (mp.mx) {
        auto sv = [](int v) { return std::to_string(v); };
        const fftu::MxSplit &x = mp.mxs;
        pl->launch_names.push_back("fftu::k_mxexchange<" + t + ", " + sv(x.nr) + ", " + sv(x.nr ? x.lpr : 0) + ", " +
                                   sv(x.nh) + ", " + sv(x.nh ? x.lph : 0) + ", " +
                                   (fftu::mx_rows_staged(mp.g, x, pl->esize) ? "true>" : "false>"));
    } else if (mp.fused) {
        const bool tl = fftu::mexchange_table_in_lds(mp.g.P, mp.T, int(pl->esize));
        pl->launch_names.push_back("fftu::k_mexchange<" + t + (tl ? ", true>" : ", false>"));
    } else {
        pl->launch_names.push_back("fftu::k_mpermute<" + t + ">");
        for (size_t i = 0; i < mp.s2.size(); ++i) pl->launch_names.push_back("fftu::k_mline<" + t + ">");
    }
    hipError_t e = hipSuccess;
    if (external) {
        e = shared_table_exact(device, dtype, mp.T, &pl->table);
    } else {
        pl->table_bytes = uint64_t(mp.T) * pl->esize;
        pl->ws_bytes = uint64_t(mp.g.N) * pl->esize;
        e = upload_table_general(&pl->table, mp.T, dtype);
        if (e == hipSuccess) e = hipMalloc(&pl->ws, pl->ws_bytes);
    }
    if (e != hipSuccess) {
        const fftu_status st = from_hip(e);
        if (!external && pl->table) (void)hipFree(pl->table);
        if (pl->ws) (void)hipFree(pl->ws);
        delete pl;
        record(st);
        return nullptr;
    }
    record(FFTU_SUCCESS);
    return pl;
}

fftu_plan_s *build_gc_plan(int d, const int64_t n[], const int64_t p[], fftu_dtype dtype, fftu_direction direction,
                           bool external, int device)
{
    GcPlan gp;
    if (!plan_gc(d, n, p, dtype, gp)) {
        record(FFTU_ERROR_UNSUPPORTED);
        return nullptr;
    }
    fftu_plan_s *pl = new (std::nothrow) fftu_plan_s();
    if (!pl) {
        record(FFTU_ERROR_OUT_OF_MEMORY);
        return nullptr;
    }
    pl->d = d;
    for (int l = 0; l < d; ++l) {
        pl->n[l] = n[l];
        pl->p[l] = p[l];
    }
    pl->dtype = dtype;
    pl->dir = direction;
    pl->prec = dtype == FFTU_C128 ? Precision::F64 : Precision::F32;
    pl->esize = dtype == FFTU_C128 ? 16 : 8;
    pl->device = device;
    pl->external = external;
    pl->gc = true;
    pl->gc_H = gp.H;
    pl->gphase = gp.phase;
    pl->gphase2 = gp.phase2;
    pl->gc_pow2 = gp.pow2;
    pl->gc_last_logg = gp.last_logg;
    pl->gput = gp.put;
    pl->table_T = gp.T;
    pl->grid.N = gp.N;
    pl->grid.M = gp.M;
    pl->grid.d = d;
    const std::string t = dtype == FFTU_C128 ? "double" : "float";
    for (int c = 0; c <= gp.H; ++c) {
        if (c == gp.H && gp.last_logg > 0) break;
        if (gp.pow2) {
            for (const PassDesc &pd : gp.phase2[size_t(c)]) pl->launch_names.push_back(pass_kernel_name(pd, dtype));
        } else {
            for (size_t i = 0; i < gp.phase[size_t(c)].size(); ++i) pl->launch_names.push_back("fftu::k_mline<" + t + ">");
        }
        fftu::GputTileDesc tl{};
        if (c + 1 == gp.H && gp.last_logg > 0)
            pl->launch_names.push_back("fftu::k_gplast<" + t + ", " + std::to_string(gp.last_logg) + ">");
        else if (c < gp.H && fftu::gput_tiling(gp.put[size_t(c)], int(pl->esize), tl) && tl.K >= 8)
            pl->launch_names.push_back("fftu::k_gputt<" + t + ", " + std::to_string(1 << (tl.K - 8)) + ">");
        else if (c < gp.H)
            pl->launch_names.push_back("fftu::k_gput<" + t + ">");
    }
    pl->launches = int(pl->launch_names.size());
    hipError_t e = hipSuccess;
    if (external) {
        e = shared_table_exact(device, dtype, gp.T, &pl->table);
    } else {
        pl->table_bytes = uint64_t(gp.T) * pl->esize;
        pl->ws_bytes = uint64_t(gp.N) * pl->esize;
        e = upload_table_general(&pl->table, gp.T, dtype);
        if (e == hipSuccess) e = hipMalloc(&pl->ws, pl->ws_bytes);
    }
    if (e != hipSuccess) {
        const fftu_status st = from_hip(e);
        if (!external && pl->table) (void)hipFree(pl->table);
        if (pl->ws) (void)hipFree(pl->ws);
        delete pl;
        record(st);
        return nullptr;
    }
    record(FFTU_SUCCESS);
    return pl;
}

fftu_plan_s *build_plan(int d, const int64_t n[], const int64_t p[], fftu_dtype dtype, fftu_direction direction,
                        bool external)
{
    fftu_status s = validate(d, n, p, dtype, direction);
    if (s != FFTU_SUCCESS) {
        record(s);
        return nullptr;
    }
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) {
        record(FFTU_ERROR_DEVICE);
        return nullptr;
    }
    if (plan_is_group_cyclic(d, n, p)) return build_gc_plan(d, n, p, dtype, direction, external, device);
    if (plan_is_mixed(d, n, p)) return build_mixed_plan(d, n, p, dtype, direction, external, device);
    Geometry G = geometry(d, n, p);
    void *shared = nullptr;
    if (external) {
        int logK = 0;
        hipError_t e = shared_table(device, dtype, G.lognmax, &shared, &logK);
        if (e != hipSuccess) {
            record(from_hip(e));
            return nullptr;
        }
        G.lognmax = logK;
    }
    fftu_plan_s *pl = new (std::nothrow) fftu_plan_s();
    if (!pl) {
        record(FFTU_ERROR_OUT_OF_MEMORY);
        return nullptr;
    }
    pl->d = d;
    for (int l = 0; l < d; ++l) {
        pl->n[l] = n[l];
        pl->p[l] = p[l];
    }
    pl->dtype = dtype;
    pl->dir = direction;
    pl->prec = dtype == FFTU_C128 ? Precision::F64 : Precision::F32;
    pl->esize = dtype == FFTU_C128 ? 16 : 8;
    pl->device = device;
    pl->external = external;
    pl->grid = make_grid(G);
    pl->s0 = plan_s0(G, dtype);
    pl->s2 = plan_s2(G, dtype);
    ExchangeSplit sp;
    pl->fused = exchange_split(G, dtype, &sp);
    if (pl->fused) pl->ex = make_exchange(G, pl->grid, sp, dtype);
    pl->lastx = plan_lastx(G, pl->grid, dtype, pl->s0x, pl->lx);
    if (pl->lastx) {
        fftu_plan_info info{};
        fill_info(G, pl->s0x, true, 0, dtype, &info, true);
        pl->launches = info.launches;
        for (const PassDesc &pd : pl->s0x) pl->launch_names.push_back(pass_kernel_name(pd, dtype));
        pl->launch_names.push_back(lastx_kernel_name(pl->lx, dtype));
    } else {
        fftu_plan_info info{};
        fill_info(G, pl->s0, pl->fused, pl->s2.size(), dtype, &info);
        pl->launches = info.launches;
        pl->ttrans = !pl->fused && transpose_exchange(G);
        pl->ttrans_ld = pl->fused ? 0 : transpose_fused_ld(G);
        if (pl->ttrans_ld > 0) {
            pl->s0t = plan_s0(G, dtype, true);
            pl->s2t = plan_s2(G, dtype, true);
        }
        for (const PassDesc &pd : (pl->ttrans_ld > 0 ? pl->s0t : pl->s0))
            pl->launch_names.push_back(pass_kernel_name(pd, dtype));
        if (pl->fused) {
            pl->launch_names.push_back(exchange_kernel_name(pl->ex, dtype));
        } else {
            const std::string t = dtype == FFTU_C128 ? "double" : "float";
            if (pl->ttrans) {
                pl->launch_names.push_back("fftu::k_ttranspose<" + t + ", " + std::to_string(pl->ttrans_ld) + ">");
            } else {
                pl->launch_names.push_back("fftu::k_twiddle<" + t + ">");
                pl->launch_names.push_back("fftu::k_permute<" + t + ">");
            }
            for (const PassDesc &pd : (pl->ttrans_ld > 0 ? pl->s2t : pl->s2))
                pl->launch_names.push_back(pass_kernel_name(pd, dtype));
        }
    }
    if (external) {
        pl->table = shared;      // not owned
        record(FFTU_SUCCESS);
        return pl;
    }
    pl->table_bytes = (uint64_t(1) << G.lognmax) * pl->esize;
    pl->ws_bytes = uint64_t(pl->grid.N) * pl->esize;
    hipError_t e = upload_table(&pl->table, G.lognmax, dtype);
    if (e == hipSuccess) e = hipMalloc(&pl->ws, pl->ws_bytes);
    if (e != hipSuccess) {
        fftu_status st = from_hip(e);
        if (pl->table) (void)hipFree(pl->table);
        if (pl->ws) (void)hipFree(pl->ws);
        delete pl;
        record(st);
        return nullptr;
    }
    record(FFTU_SUCCESS);
    return pl;
}

}  // namespace

extern "C" {

const char *fftu_version(void) { return "fftu 0.1"; }

const char *fftu_status_string(fftu_status s)
{
    switch (s) {
    case FFTU_SUCCESS: return "FFTU_SUCCESS";
    case FFTU_ERROR_INVALID_VALUE: return "FFTU_ERROR_INVALID_VALUE";
    case FFTU_ERROR_NOT_DIVISIBLE: return "FFTU_ERROR_NOT_DIVISIBLE";
    case FFTU_ERROR_UNSUPPORTED: return "FFTU_ERROR_UNSUPPORTED";
    case FFTU_ERROR_OUT_OF_MEMORY: return "FFTU_ERROR_OUT_OF_MEMORY";
    case FFTU_ERROR_DEVICE: return "FFTU_ERROR_DEVICE";
    }
    return "FFTU_UNKNOWN_STATUS";
}

fftu_status fftu_last_error(void) { return g_last; }

fftu_status fftu_set_tuning(fftu_tune_param param, int value)
{
    const int i = int(param);
    if (i < 0 || i >= FFTU_TUNE_COUNT) return record(FFTU_ERROR_INVALID_VALUE);
    if (value != -1 && (value < g_tune_min[i] || value > g_tune_max[i])) return record(FFTU_ERROR_INVALID_VALUE);
    g_tune[i].store(value, std::memory_order_relaxed);
    return record(FFTU_SUCCESS);
}

int fftu_get_tuning(fftu_tune_param param)
{
    const int i = int(param);
    if (i < 0 || i >= FFTU_TUNE_COUNT) {
        record(FFTU_ERROR_INVALID_VALUE);
        return -1;
    }
    record(FFTU_SUCCESS);
    return knob(i);
}

fftu_status fftu_check(int d, const int64_t n[], const int64_t p[], fftu_dtype dtype, fftu_direction direction)
{
    return record(validate(d, n, p, dtype, direction));
}

fftu_status fftu_describe(int d, const int64_t n[], const int64_t p[], fftu_dtype dtype, fftu_direction direction,
                          fftu_plan_info *info)
{
    fftu_status s = validate(d, n, p, dtype, direction);
    if (s != FFTU_SUCCESS) return record(s);
    if (!info) return record(FFTU_ERROR_INVALID_VALUE);
    if (plan_is_group_cyclic(d, n, p)) {
        GcPlan gp;
        if (!plan_gc(d, n, p, dtype, gp)) return record(FFTU_ERROR_UNSUPPORTED);
        fill_info_gc(gp, d, dtype, info);
        return record(FFTU_SUCCESS);
    }
    if (plan_is_mixed(d, n, p)) {
        MixedPlan mp;
        if (!plan_mixed(d, n, p, dtype, mp)) return record(FFTU_ERROR_UNSUPPORTED);
        fill_info_mixed(mp, dtype, info);
        return record(FFTU_SUCCESS);
    }
    const Geometry G = geometry(d, n, p);
    std::vector<PassDesc> s0x;
    fftu::LastxDesc lx;
    if (plan_lastx(G, make_grid(G), dtype, s0x, lx)) {
        fill_info(G, s0x, true, 0, dtype, info, true);
        return record(FFTU_SUCCESS);
    }
    const auto s0 = plan_s0(G, dtype);
    ExchangeSplit sp;
    const bool fused = exchange_split(G, dtype, &sp);
    const auto s2 = plan_s2(G, dtype);
    fill_info(G, s0, fused, s2.size(), dtype, info);
    return record(FFTU_SUCCESS);
}

fftu_plan_t fftu_plan(int d, const int64_t n[], const int64_t p[], fftu_dtype dtype, fftu_direction direction)
{
    return build_plan(d, n, p, dtype, direction, false);
}

fftu_plan_t fftu_plan_real(int d, const int64_t n[], const int64_t p[], fftu_dtype dtype, fftu_direction direction)
{
    if (d < 1 || d > FFTU_MAX_DIMS || !n || !p) {
        record(d > FFTU_MAX_DIMS ? FFTU_ERROR_UNSUPPORTED : FFTU_ERROR_INVALID_VALUE);
        return nullptr;
    }
    if (n[d - 1] < 2 || n[d - 1] % 2 || p[d - 1] < 1 || (n[d - 1] / 2) % p[d - 1]) {
        record(n[d - 1] >= 2 && n[d - 1] % 2 == 0 && p[d - 1] >= 1 ? FFTU_ERROR_NOT_DIVISIBLE
                                                                      : FFTU_ERROR_INVALID_VALUE);
        return nullptr;
    }
    int64_t np[fftu::kMaxDims];
    for (int l = 0; l < d; ++l) np[l] = n[l];
    np[d - 1] = n[d - 1] / 2;
    fftu_plan_s *rc = build_plan(d, np, p, dtype, direction, false);
    if (!rc) return nullptr;
    fftu_plan_s *pl = new (std::nothrow) fftu_plan_s();
    if (!pl) {
        fftu_destroy(rc);
        record(FFTU_ERROR_OUT_OF_MEMORY);
        return nullptr;
    }
    pl->real = true;
    pl->rc = rc;
    pl->d = d;
    for (int l = 0; l < d; ++l) {
        pl->n[l] = n[l];
        pl->p[l] = p[l];
    }
    pl->dtype = dtype;
    pl->dir = direction;
    pl->prec = rc->prec;
    pl->esize = rc->esize;
    pl->device = rc->device;
    fftu::RealDesc &rd = pl->rd;
    rd.d = d;
    rd.h = int32_t(n[d - 1] / 2);
    int64_t P = 1, Pp = 1, Nh = 1, Np = 1;
    for (int l = 0; l < d; ++l) {
        rd.n[l] = int32_t(np[l]);
        rd.p[l] = int32_t(p[l]);
        rd.m[l] = int32_t(np[l] / p[l]);
        P *= p[l];
        Nh *= np[l];
        if (l < d - 1) {
            Pp *= p[l];
            Np *= n[l];
        }
    }
    rd.Nh = Nh;
    rd.Mh = Nh / P;
    rd.Mp = Np / Pp;
    pl->real_in_elems = direction == FFTU_FORWARD ? Nh : Nh + Np;
    pl->real_out_elems = direction == FFTU_FORWARD ? Nh + Np : Nh;
    pl->grid.N = Nh;
    const std::string t = dtype == FFTU_C128 ? "double" : "float";
    const std::string dd = ", " + std::to_string(d) + ">";
    if (direction == FFTU_INVERSE) pl->launch_names.push_back("fftu::k_rmerge<" + t + dd);
    for (const std::string &k : rc->launch_names) pl->launch_names.push_back(k);
    if (direction == FFTU_FORWARD) pl->launch_names.push_back("fftu::k_rsplit<" + t + dd);
    pl->launches = int(pl->launch_names.size());
    pl->table_bytes = uint64_t(n[d - 1]) * pl->esize;
    hipError_t e = upload_table_general(&pl->rtable, n[d - 1], dtype);
    if (e != hipSuccess) {
        fftu_destroy(pl);
        record(from_hip(e));
        return nullptr;
    }
    record(FFTU_SUCCESS);
    return pl;
}

namespace {
// The DST's signal signs (negated once per dimension with natural index m_l >= n_l / 2;
// on the packed array, packed index >= n_d / 4 along the last dimension) depend only on
// the local index when every local side m_l of the packed array is even: m_l >= n_l / 2
// exactly when i_l >= m_l / 2, the top bit of i_l's field in the local index where the
// sides are powers of two. They go into the complex transform's first pass (as the
// parity of the local index bits under one mask) when that pass is a line pass;
// returns whether they did.
uint64_t dst_sign_mask(const fftu_plan_s *cp, int d, const int64_t n[], const int64_t p[])
{
    uint64_t mask = 0;
    int off = 0;
    int64_t M = 1;
    for (int l = d - 1; l >= 0; --l) {
        const int64_t nl = l == d - 1 ? n[l] / 2 : n[l];
        if (nl % p[l]) return 0;
        const int64_t ml = nl / p[l];
        if (ml < 2 || !is_pow2(ml)) return 0;
        const int lg = ilog2(ml);
        mask |= uint64_t(1) << (off + lg - 1);
        off += lg;
        M *= ml;
    }
    return (M == cp->grid.M && off <= 62) ? mask : 0;
}

// Inverse: the signs go into the complex transform's last kernel when that is the
// fused exchange or k_lastx (k_exchange_sign / k_lastx_sign negate their outputs by
// the same parity).
bool fuse_dst_signs_inverse(fftu_plan_s *rp, int d, const int64_t n[], const int64_t p[])
{
    fftu_plan_s *cp = rp ? rp->rc : nullptr;
    if (!cp || cp->gc || cp->mixed || cp->is_batch || cp->ttrans || !(cp->fused || cp->lastx)) return false;
    // the fused exchange, or k_lastx (the innermost lines with the exchange)
    const std::string xname = cp->lastx ? "fftu::k_lastx<" : "fftu::k_exchange<";
    if (cp->launch_names.empty() || cp->launch_names.back().compare(0, xname.size(), xname) != 0) return false;
    if (rp->launch_names.empty() || rp->launch_names.back() != cp->launch_names.back()) return false;
    const uint64_t mask = dst_sign_mask(cp, d, n, p);
    if (!mask) return false;
    if (cp->lastx)
        cp->lx.ex.sign_mask = mask;
    else
        cp->ex.sign_mask = mask;
    const std::string renamed = (cp->lastx ? "fftu::k_lastx_sign<" : "fftu::k_exchange_sign<") +
                                cp->launch_names.back().substr(xname.size());
    cp->launch_names.back() = renamed;
    rp->launch_names.back() = renamed;
    return true;
}

bool fuse_dst_signs(fftu_plan_s *rp, int d, const int64_t n[], const int64_t p[])
{
    fftu_plan_s *cp = rp ? rp->rc : nullptr;
    if (!cp || cp->gc || cp->mixed || cp->is_batch || cp->launch_names.empty()) return false;
    std::vector<PassDesc> *first = nullptr;
    if (cp->lastx)
        first = cp->s0x.empty() ? nullptr : &cp->s0x;
    else
        first = cp->ttrans_ld > 0 ? &cp->s0t : &cp->s0;
    if (!first || first->empty()) return false;
    PassDesc &pd = (*first)[0];
    if (pd.kind != fftu::kLineStrided && pd.kind != fftu::kLineContig && pd.kind != fftu::kLineStaged) return false;
    const std::string lname = "fftu::k_line<";
    if (cp->launch_names[0].compare(0, lname.size(), lname) != 0) return false;
    const uint64_t mask = dst_sign_mask(cp, d, n, p);
    if (!mask) return false;
    pd.sign_mask = mask;
    cp->launch_names[0] = "fftu::k_line_sign<" + cp->launch_names[0].substr(lname.size());
    return true;
}
}  // namespace

fftu_plan_t fftu_plan_r2r(int d, const int64_t n[], const int64_t p[], fftu_dtype dtype, fftu_r2r_kind kind,
                          fftu_direction direction)
{
    if (d < 1 || !n || !p || (kind != FFTU_DCT && kind != FFTU_DST)) {
        record(FFTU_ERROR_INVALID_VALUE);
        return nullptr;
    }
    if (d > fftu::kR2RMaxDims) {
        record(FFTU_ERROR_UNSUPPORTED);
        return nullptr;
    }
    for (int l = 0; l < d; ++l)
        if (n[l] < 2 || n[l] % 2 || p[l] < 1 || n[l] >= (int64_t(1) << 30)) {
            record(FFTU_ERROR_INVALID_VALUE);
            return nullptr;
        }
    // the signal's real transform (its own checks: p | n, p_d | n_d / 2, the grid)
    fftu_plan_s *rc = fftu_plan_real(d, n, p, dtype, direction);
    if (!rc) return nullptr;
    fftu_plan_s *pl = new (std::nothrow) fftu_plan_s();
    if (!pl) {
        fftu_destroy(rc);
        record(FFTU_ERROR_OUT_OF_MEMORY);
        return nullptr;
    }
    pl->r2r = true;
    pl->r2r_kind = kind;
    pl->rc = rc;
    if (kind == FFTU_DST)
        pl->r2r_sign_fused = direction == FFTU_FORWARD ? fuse_dst_signs(rc, d, n, p) : fuse_dst_signs_inverse(rc, d, n, p);
    pl->d = d;
    int64_t T4 = 1, groups = 1, P = 1, N = 1;
    for (int l = 0; l < d; ++l) {
        pl->n[l] = n[l];
        pl->p[l] = p[l];
        T4 = lcm64(T4, 4 * n[l]);
        groups *= n[l] / 2 + 1;
        P *= p[l];
        N *= n[l];
    }
    pl->dtype = dtype;
    pl->dir = direction;
    pl->prec = rc->prec;
    pl->esize = rc->esize;
    pl->device = rc->device;
    pl->grid.N = N / 2;
    fftu::R2RDesc &g = pl->r2d;
    g.d = d;
    g.dst = kind == FFTU_DST ? 1 : 0;
    for (int l = 0; l < d; ++l) {
        g.n[l] = int32_t(n[l]);
        g.p[l] = int32_t(p[l]);
        g.m[l] = int32_t(n[l] / p[l]);
        g.tstep[l] = int32_t(T4 / (4 * n[l]));
    }
    g.M = N / P;
    g.groups = groups;
    g.rd = rc->rd;
    const std::string t = dtype == FFTU_C128 ? "double" : "float";
    const std::string dd = std::to_string(d);
    const bool dst = kind == FFTU_DST;
    if (direction == FFTU_FORWARD) {
        // the complex transform of the packed signal, then the split and the coefficients in one pass
        if (dst && !pl->r2r_sign_fused) pl->launch_names.push_back("fftu::k_r2rsign<" + t + ", " + std::to_string(d) + ">");
        for (const std::string &k : rc->rc->launch_names) pl->launch_names.push_back(k);
        const bool rows = fftu::r2rpost_rows_lds(g, dtype == FFTU_C128 ? sizeof(double) : sizeof(float)) > 0;
        pl->launch_names.push_back((rows ? "fftu::k_r2rpost_rows<" : "fftu::k_r2rpost<") + t + ", " + dd + ">");
    } else if (fftu::r2rpre_merge_lds(g, pl->esize) > 0) {
        // the spectrum and the merge in one pass, then the inverse complex transform
        pl->r2r_pre_merge = true;
        pl->launch_names.push_back("fftu::k_r2rpre_merge<" + t + ", " + dd + ">");
        for (const std::string &k : rc->rc->launch_names) pl->launch_names.push_back(k);
        if (dst && !pl->r2r_sign_fused) pl->launch_names.push_back("fftu::k_r2rsign<" + t + ", " + std::to_string(d) + ">");
    } else {
        pl->launch_names.push_back("fftu::k_r2rpre<" + t + ", " + dd + (fftu::r2rpre_rows(g) ? ", true>" : ", false>"));
        for (const std::string &k : rc->launch_names) pl->launch_names.push_back(k);
        if (dst && !pl->r2r_sign_fused) pl->launch_names.push_back("fftu::k_r2rsign<" + t + ", " + std::to_string(d) + ">");
    }
    pl->launches = int(pl->launch_names.size());
    pl->table_T = T4;
    pl->table_bytes = uint64_t(T4) * pl->esize;
    // the spectrum: the half spectrum and the Nyquist plane
    pl->ws_bytes = uint64_t(rc->real_in_elems > rc->real_out_elems ? rc->real_in_elems : rc->real_out_elems) *
                   pl->esize;
    hipError_t e = T4 < (int64_t(1) << 26) ? upload_table_general(&pl->rtable, T4, dtype) : hipErrorInvalidValue;
    if (e == hipSuccess) e = hipMalloc(&pl->ws, pl->ws_bytes);
    if (e != hipSuccess) {
        const fftu_status st = T4 < (int64_t(1) << 26) ? from_hip(e) : FFTU_ERROR_UNSUPPORTED;
        fftu_destroy(pl);
        record(st);
        return nullptr;
    }
    record(FFTU_SUCCESS);
    return pl;
}

fftu_plan_t fftu_plan_external(int d, const int64_t n[], const int64_t p[], fftu_dtype dtype,
                               fftu_direction direction)
{
    return build_plan(d, n, p, dtype, direction, true);
}

}  // extern "C"

namespace fftu {
// The work list of a batch (host side; see fftu_batch.hip): one descriptor per
// (stage, transform) in stage-major order, the prefix sums of their work items,
// and the descriptor each one waits for.
fftu_status build_batch_worklist(int count, const int d[], const int64_t *const n[], const int64_t *const p[],
                                 fftu_dtype dtype, fftu_direction direction, BatchWorklist &wl)
{
    if (count < 1 || !d || !n || !p) return FFTU_ERROR_INVALID_VALUE;
    for (int f = 0; f < count; ++f) {
        fftu_status s = validate(d[f], n[f], p[f], dtype, direction);
        if (s != FFTU_SUCCESS) return s;
        // batches: powers of two with one exchange only
        if (plan_is_mixed(d[f], n[f], p[f]) || plan_is_group_cyclic(d[f], n[f], p[f])) return FFTU_ERROR_UNSUPPORTED;
    }
    const size_t esize = dtype == FFTU_C128 ? 16 : 8;
    const int inv = direction == FFTU_INVERSE ? 1 : 0;
    // per-transform stages: line passes of Superstep 0, then the fused exchange
    struct Member {
        std::vector<PassDesc> s0;
        ExchangeDesc ex;
        int64_t M;
    };
    std::vector<Member> mem(static_cast<size_t>(count));
    int lognmax = 0, smax = 0;
    uint64_t ws_total = 0;
    uint32_t tile_lds = 0;
    wl = BatchWorklist{};
    for (int f = 0; f < count; ++f) {
        const Geometry G = geometry(d[f], n[f], p[f]);
        lognmax = std::max(lognmax, G.lognmax);
        const GridDesc g = make_grid(G);
        Member &m = mem[size_t(f)];
        m.M = g.M;
        // as plan_s0: the two innermost dimensions share a k_group2 pass when their
        // planes are small, every other dimension gets a line pass
        std::vector<int> dims;   // dimensions with m_l > 1, innermost first
        for (int l = G.d - 1; l >= 0; --l)
            if (G.logm[l] > 0) dims.push_back(l);
        auto outer_of = [&](int l) {
            int logA = G.logP;
            for (int j = 0; j < l; ++j) logA += G.logm[j];
            return logA;
        };
        size_t first_line = 0;
        if (dims.size() >= 2) {
            PassDesc pd;
            const int li = dims[0], lo = dims[1];
            if (make_group2_pass(outer_of(lo), G.logm[lo], G.logm[li], dtype, G.lognmax, pd) &&
                pd.threads <= kBatchThreads) {
                const uint32_t tw_bytes = ((uint32_t(1) << G.logm[lo]) + (uint32_t(1) << G.logm[li])) * uint32_t(esize);
                tile_lds = std::max(tile_lds, uint32_t(pd.lds_bytes - tw_bytes));
                m.s0.push_back(pd);
                first_line = 2;
            }
        }
        for (size_t i = first_line; i < dims.size(); ++i) {
            const int l = dims[i];
            int logB = 0;
            for (int j = l + 1; j < G.d; ++j) logB += G.logm[j];
            PassDesc pd;
            if (G.logm[l] > kBatchMaxLogLine || !make_line_pass(outer_of(l), G.logm[l], logB, dtype, G.lognmax, pd, 8) ||
                pd.threads > kBatchThreads)
                return FFTU_ERROR_UNSUPPORTED;
            tile_lds = std::max(tile_lds, uint32_t(pd.lds_bytes - (uint32_t(1) << G.logm[l]) * esize));
            m.s0.push_back(pd);
        }
        ExchangeSplit sp;
        if (m.s0.empty() || !exchange_split(G, dtype, &sp) || !batch_exchange_ok(sp)) return FFTU_ERROR_UNSUPPORTED;
        m.ex = make_exchange(G, g, sp, dtype);
        m.s0.front().conj_in = inv;
        m.ex.g.conj_out = inv;
        m.ex.g.scale = inv ? 1.0 / double(g.N) : 1.0;
        wl.N.push_back(g.N);
        wl.ws.push_back(ws_total);
        ws_total += uint64_t(g.N);
        smax = std::max(smax, int(m.s0.size()) + 1);
    }
    std::vector<int> last_desc(size_t(count), -1);
    wl.starts.assign(1, 0);
    for (int s = 0; s < smax; ++s) {
        for (int f = 0; f < count; ++f) {
            const Member &m = mem[size_t(f)];
            const int ns0 = int(m.s0.size());
            if (s > ns0) continue;
            BatchStage st{};
            int64_t tile_elems;
            if (s < ns0) {
                st.kind = m.s0[size_t(s)].kind;
                st.pd = m.s0[size_t(s)];
                st.tiles = st.pd.tiles;
                tile_elems = int64_t(1) << (st.pd.logW + st.pd.logG);   // W lines of L, or W planes of L1 L2
            } else {
                st.kind = kExchangeStage;
                st.ex = m.ex;
                const int64_t ngroups = (m.M + 63) / 64;
                st.tiles = (ngroups + 3) / 4;             // 4 groups of 64 local indices (all P sources) per tile
                tile_elems = int64_t(256) << (st.ex.nr * st.ex.lpr);
            }
            const int64_t per = std::max<int64_t>(1, (int64_t(1) << kBatchItemLog) / tile_elems);
            st.per_item = int32_t(per);
            const int64_t items = (st.tiles + per - 1) / per;
            // every stage indexes the batch's one table of omega_{2^lognmax}
            st.pd.lognmax = lognmax;
            st.ex.g.lognmax = lognmax;
            st.member = f;
            st.io = (s == 0 ? 1 : 0) | (s == ns0 ? 2 : 0);
            wl.stages.push_back(st);
            wl.member.push_back(f);
            wl.first.push_back(s == 0 ? 1 : 0);
            wl.last.push_back(s == ns0 ? 1 : 0);
            wl.dep.push_back(last_desc[size_t(f)]);
            last_desc[size_t(f)] = int(wl.stages.size()) - 1;
            wl.starts.push_back(wl.starts.back() + items);
        }
    }
    wl.lognmax = lognmax;
    wl.items = wl.starts.back();
    wl.lds = uint32_t(kBatchMaxLine) * uint32_t(esize) + tile_lds;
    wl.ws_total = ws_total;
    return FFTU_SUCCESS;
}
}  // namespace fftu

extern "C" {

fftu_plan_t fftu_plan_batch(int count, const int d[], const int64_t *const n[], const int64_t *const p[],
                            fftu_dtype dtype, fftu_direction direction)
{
    fftu::BatchWorklist wl;
    fftu_status bs = fftu::build_batch_worklist(count, d, n, p, dtype, direction, wl);
    if (bs != FFTU_SUCCESS) {
        record(bs);
        return nullptr;
    }
    fftu_plan_s *pl = new (std::nothrow) fftu_plan_s();
    if (!pl) {
        record(FFTU_ERROR_OUT_OF_MEMORY);
        return nullptr;
    }
    pl->is_batch = true;
    pl->count = count;
    pl->dtype = dtype;
    pl->dir = direction;
    pl->prec = dtype == FFTU_C128 ? Precision::F64 : Precision::F32;
    pl->esize = dtype == FFTU_C128 ? 16 : 8;
    pl->hstages = wl.stages;
    pl->stage_member = wl.member;
    pl->stage_first = wl.first;
    pl->stage_last = wl.last;
    pl->member_N = wl.N;
    pl->member_ws = wl.ws;
    pl->batch_items = wl.items;
    pl->batch_lds = wl.lds;
    const int lognmax = wl.lognmax;
    const uint64_t ws_total = wl.ws_total;
    const std::vector<int64_t> &starts = wl.starts;
    const std::vector<int32_t> &dep = wl.dep;
    hipError_t e = hipGetDevice(&pl->device);
    const int64_t L = int64_t(1) << lognmax;
    const std::vector<double> t64 = make_table_f64(lognmax);
    pl->table_bytes = uint64_t(L) * pl->esize;
    pl->ws_bytes = ws_total * pl->esize;
    const size_t K = pl->hstages.size();
    if (e == hipSuccess) e = hipMalloc(&pl->table, pl->table_bytes);
    if (e == hipSuccess) e = hipMalloc(&pl->ws, pl->ws_bytes);
    if (e == hipSuccess) e = hipMalloc(&pl->dstages, K * sizeof(fftu::BatchStage));
    if (e == hipSuccess) e = hipMalloc(&pl->dstarts, (K + 1) * sizeof(int64_t));
    if (e == hipSuccess) e = hipMalloc(&pl->ddep, K * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&pl->ddone, K * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&pl->dnext, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc(&pl->derror, sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&pl->dbind, size_t(count) * sizeof(fftu::BatchBind));
    if (e == hipSuccess) {
        // stages between a transform's first and last read and write its workspace;
        // the caller's buffers come from the bind array
        for (size_t k = 0; k < K; ++k) {
            const int f = pl->stage_member[k];
            char *ws = static_cast<char *>(pl->ws) + pl->member_ws[size_t(f)] * pl->esize;
            fftu::BatchStage &st = pl->hstages[k];
            st.src = pl->stage_first[k] ? nullptr : ws;
            st.dst = pl->stage_last[k] ? nullptr : static_cast<void *>(ws);
        }
        e = hipMemcpy(pl->dstages, pl->hstages.data(), K * sizeof(fftu::BatchStage), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemcpy(pl->dstarts, starts.data(), (K + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(pl->ddep, dep.data(), K * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        if (dtype == FFTU_C128) {
            e = hipMemcpy(pl->table, t64.data(), pl->table_bytes, hipMemcpyHostToDevice);
        } else {
            std::vector<float> t32(t64.size());
            for (size_t i = 0; i < t64.size(); ++i) t32[i] = float(t64[i]);
            e = hipMemcpy(pl->table, t32.data(), pl->table_bytes, hipMemcpyHostToDevice);
        }
    }
    int cus = 0, clock_khz = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, pl->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, pl->device);
    pl->batch_wait_ticks = int64_t(clock_khz > 0 ? clock_khz : 100000) * 2000;   // 2 s
    if (e != hipSuccess) {
        fftu_status st = from_hip(e);
        free_batch(pl);
        if (pl->table) (void)hipFree(pl->table);
        if (pl->ws) (void)hipFree(pl->ws);
        delete pl;
        record(st);
        return nullptr;
    }
    const int64_t resident = int64_t(fftu::batch_blocks_per_cu(pl->prec, pl->batch_lds)) * int64_t(cus);
    pl->batch_blocks = uint32_t(std::max<int64_t>(1, std::min<int64_t>(resident, pl->batch_items)));
    pl->launches = 2;
    pl->launch_names = {"fftu::k_batch_reset", std::string("fftu::k_batch<") +
                                                   (dtype == FFTU_C128 ? "double" : "float") + ">"};
    int64_t Ntot = 0;
    for (int64_t v : pl->member_N) Ntot += v;
    pl->grid.N = Ntot;
    pl->d = 0;
    record(FFTU_SUCCESS);
    return pl;
}

fftu_plan_t fftu_plan_batch_external(int count, const int d[], const int64_t *const n[], const int64_t *const p[],
                                     fftu_dtype dtype, fftu_direction direction)
{
    fftu::BatchWorklist wl;
    fftu_status bs = fftu::build_batch_worklist(count, d, n, p, dtype, direction, wl);
    if (bs != FFTU_SUCCESS) {
        record(bs);
        return nullptr;
    }
    int device = 0, cus = 0, clock_khz = 0;
    if (hipGetDevice(&device) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess) {
        record(FFTU_ERROR_DEVICE);
        return nullptr;
    }
    void *table = nullptr;
    int logK = 0;
    hipError_t e = shared_table(device, dtype, wl.lognmax, &table, &logK);
    if (e != hipSuccess) {
        record(from_hip(e));
        return nullptr;
    }
    fftu_plan_s *pl = new (std::nothrow) fftu_plan_s();
    if (!pl) {
        record(FFTU_ERROR_OUT_OF_MEMORY);
        return nullptr;
    }
    pl->is_batch = true;
    pl->external = true;
    pl->count = count;
    pl->dtype = dtype;
    pl->dir = direction;
    pl->prec = dtype == FFTU_C128 ? Precision::F64 : Precision::F32;
    pl->esize = dtype == FFTU_C128 ? 16 : 8;
    pl->device = device;
    pl->table = table;                      // shared, not owned
    pl->hstages = wl.stages;
    for (fftu::BatchStage &st : pl->hstages) {
        // the shared table is omega_{2^logK}, logK >= lognmax: the same entries at a finer stride
        st.pd.lognmax = logK;
        st.ex.g.lognmax = logK;
    }
    pl->stage_member = wl.member;
    pl->stage_first = wl.first;
    pl->stage_last = wl.last;
    pl->member_N = wl.N;
    pl->member_ws = wl.ws;
    pl->hstarts = wl.starts;
    pl->hdep = wl.dep;
    pl->batch_items = wl.items;
    pl->batch_lds = wl.lds;
    pl->batch_wait_ticks = int64_t(clock_khz > 0 ? clock_khz : 100000) * 2000;   // 2 s
    const int64_t resident = int64_t(fftu::batch_blocks_per_cu(pl->prec, pl->batch_lds)) * int64_t(cus);
    pl->batch_blocks = uint32_t(std::max<int64_t>(1, std::min<int64_t>(resident, pl->batch_items)));
    pl->launches = 2;
    pl->launch_names = {"fftu::k_batch_reset", std::string("fftu::k_batch<") +
                                                   (dtype == FFTU_C128 ? "double" : "float") + ">"};
    int64_t Ntot = 0;
    for (int64_t v : pl->member_N) Ntot += v;
    pl->grid.N = Ntot;
    pl->ws_bytes = 0;
    record(FFTU_SUCCESS);
    return pl;
}

size_t fftu_batch_workspace_bytes(fftu_plan_t plan)
{
    if (!plan || !plan->is_batch || !plan->external) {
        record(FFTU_ERROR_INVALID_VALUE);
        return 0;
    }
    record(FFTU_SUCCESS);
    return batch_ws_layout(plan).total;
}

size_t fftu_batch_staging_bytes(fftu_plan_t plan)
{
    if (!plan || !plan->is_batch || !plan->external) {
        record(FFTU_ERROR_INVALID_VALUE);
        return 0;
    }
    record(FFTU_SUCCESS);
    const BatchWsLayout lay = batch_ws_layout(plan);
    return lay.staged - lay.stages;
}

fftu_status fftu_execute_batch_ws(fftu_plan_t plan, const void *const in[], void *const out[], void *workspace,
                                  void *host_staging, hipStream_t stream)
{
    if (!plan || !plan->is_batch || !plan->external || !workspace || !host_staging || !aligned(workspace, 256))
        return record(FFTU_ERROR_INVALID_VALUE);
    fftu_status s = check_batch_args(plan, in, out);
    if (s != FFTU_SUCCESS) return record(s);
    const BatchWsLayout lay = batch_ws_layout(plan);
    const uintptr_t w0 = reinterpret_cast<uintptr_t>(workspace), w1 = w0 + lay.total;
    for (int f = 0; f < plan->count; ++f) {
        // the workspace must overlap no buffer
        const uintptr_t bytes = uintptr_t(plan->member_N[size_t(f)]) * plan->esize;
        for (const void *b : {in[f], static_cast<const void *>(out[f])}) {
            const uintptr_t a = reinterpret_cast<uintptr_t>(b);
            if (a < w1 && w0 < a + bytes) return record(FFTU_ERROR_INVALID_VALUE);
        }
    }
    char *ws = static_cast<char *>(workspace);
    // the image of [stages | starts | dep | bind] for these buffers and this workspace,
    // laid out as in the workspace from offset lay.stages on
    char *img = static_cast<char *>(host_staging) - lay.stages;
    fftu::BatchStage *st = reinterpret_cast<fftu::BatchStage *>(img + lay.stages);
    const size_t K = plan->hstages.size();
    for (size_t k = 0; k < K; ++k) {
        st[k] = plan->hstages[k];
        const int f = plan->stage_member[k];
        char *mws = ws + plan->member_ws[size_t(f)] * plan->esize;
        st[k].src = plan->stage_first[k] ? nullptr : mws;
        st[k].dst = plan->stage_last[k] ? nullptr : static_cast<void *>(mws);
    }
    std::memcpy(img + lay.starts, plan->hstarts.data(), (K + 1) * sizeof(int64_t));
    std::memcpy(img + lay.dep, plan->hdep.data(), K * sizeof(int32_t));
    fftu::BatchBind *bind = reinterpret_cast<fftu::BatchBind *>(img + lay.bind);
    for (int f = 0; f < plan->count; ++f) bind[f] = {in[f], out[f]};
    hipError_t e = hipMemcpyAsync(ws + lay.stages, img + lay.stages, lay.staged - lay.stages, hipMemcpyHostToDevice,
                                  stream);
    if (e != hipSuccess) return record(from_hip(e));
    fftu::BatchDesc bd{};
    bd.nstages = int32_t(K);
    bd.wait_limit = plan->batch_wait_ticks;
    bd.nitems = plan->batch_items;
    bd.stages = reinterpret_cast<const fftu::BatchStage *>(ws + lay.stages);
    bd.starts = reinterpret_cast<const int64_t *>(ws + lay.starts);
    bd.dep = reinterpret_cast<const int32_t *>(ws + lay.dep);
    bd.bind = reinterpret_cast<const fftu::BatchBind *>(ws + lay.bind);
    bd.done = reinterpret_cast<int32_t *>(ws + lay.done);
    bd.next = reinterpret_cast<unsigned long long *>(ws + lay.next);
    bd.error = reinterpret_cast<int32_t *>(ws + lay.error);
    e = fftu::launch_batch_reset(bd, stream);
    if (e == hipSuccess)
        e = fftu::launch_batch(plan->prec, bd, plan->table, plan->batch_blocks, plan->batch_lds, stream);
    if (e != hipSuccess) return record(from_hip(e));
    plan->last_ws = workspace;
    return record(FFTU_SUCCESS);
}

fftu_status fftu_execute_batch(fftu_plan_t plan, const void *const in[], void *const out[], hipStream_t stream)
{
    if (plan && plan->external) return record(FFTU_ERROR_INVALID_VALUE);   // needs fftu_execute_batch_ws
    if (!plan || !plan->is_batch || !in || !out) return record(FFTU_ERROR_INVALID_VALUE);
    if (!same_binding(plan, in, out)) {
        fftu_status s = check_batch_args(plan, in, out);
        if (s == FFTU_SUCCESS) s = enqueue_bind(plan, in, out, stream);
        if (s != FFTU_SUCCESS) return record(s);
        plan->bound_in.assign(in, in + plan->count);
        plan->bound_out.assign(out, out + plan->count);
    }
    Marker mk(plan, stream);
    return record(enqueue_batch(plan, stream, &mk));
}

fftu_status fftu_fill_uniform(void *out, int64_t count, fftu_dtype dtype, uint32_t key0, uint32_t key1,
                              uint64_t counter_base, hipStream_t stream)
{
    if (count < 0 || (count > 0 && !out) || (dtype != FFTU_C64 && dtype != FFTU_C128))
        return record(FFTU_ERROR_INVALID_VALUE);
    if (count > 0 && !aligned(out, dtype == FFTU_C128 ? 16 : 8)) return record(FFTU_ERROR_INVALID_VALUE);
    const fftu::Precision prec = dtype == FFTU_C128 ? fftu::Precision::F64 : fftu::Precision::F32;
    return record(from_hip(fftu::launch_fill_uniform(prec, out, count, key0, key1, counter_base, stream)));
}

fftu_status fftu_batch_error(fftu_plan_t plan, int *flag)
{
    if (!plan || !plan->is_batch || !flag) return record(FFTU_ERROR_INVALID_VALUE);
    const void *src = plan->derror;
    if (plan->external) {
        if (!plan->last_ws) return record(FFTU_ERROR_INVALID_VALUE);
        src = static_cast<const char *>(plan->last_ws) + batch_ws_layout(plan).error;
    }
    int32_t v = 0;
    hipError_t e = hipMemcpy(&v, src, sizeof(v), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return record(from_hip(e));
    *flag = v;
    return record(FFTU_SUCCESS);
}

fftu_graph_t fftu_graph_capture(fftu_plan_t plan, int count, const void *const in[], void *const out[])
{
    if (!plan || !in || !out || count < 0 || (count > 0) != plan->is_batch || (count > 0 && count != plan->count) ||
        (plan->is_batch && plan->external)) {
        record(FFTU_ERROR_INVALID_VALUE);
        return nullptr;
    }
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        record(FFTU_ERROR_DEVICE);
        return nullptr;
    }
    fftu_status st = count > 0 ? check_batch_args(plan, in, out) : FFTU_SUCCESS;
    fftu_graph_s *gr = nullptr;
    if (st == FFTU_SUCCESS) {
        gr = new (std::nothrow) fftu_graph_s();
        if (!gr) st = FFTU_ERROR_OUT_OF_MEMORY;
    }
    if (st == FFTU_SUCCESS && count > 0) {
        gr->batch = plan;
        gr->in.assign(in, in + count);
        gr->out.assign(out, out + count);
    }
    if (st == FFTU_SUCCESS) {
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const int saved_max = plan->timing_max;
            plan->timing_max = 0;   // no timing events inside a graph
            // a batch graph binds its own buffers first, so each replay runs on them
            // whatever the plan ran on in between
            if (count > 0) st = enqueue_bind(plan, in, out, s);
            if (st == FFTU_SUCCESS) st = count > 0 ? enqueue_batch(plan, s) : fftu_execute(plan, in[0], out[0], s);
            plan->timing_max = saved_max;
            hipError_t e2 = hipStreamEndCapture(s, &gr->graph);
            if (st == FFTU_SUCCESS && e2 != hipSuccess) st = from_hip(e2);
        } else {
            st = from_hip(e);
        }
        if (st == FFTU_SUCCESS) st = from_hip(hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0));
    }
    (void)hipStreamDestroy(s);
    if (st != FFTU_SUCCESS) {
        if (gr) {
            if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
            if (gr->graph) (void)hipGraphDestroy(gr->graph);
            delete gr;
        }
        record(st);
        return nullptr;
    }
    record(FFTU_SUCCESS);
    return gr;
}

fftu_status fftu_graph_launch(fftu_graph_t graph, hipStream_t stream)
{
    if (!graph || !graph->exec) return record(FFTU_ERROR_INVALID_VALUE);
    fftu_status st = from_hip(hipGraphLaunch(graph->exec, stream));
    if (st == FFTU_SUCCESS && graph->batch) {
        // the replay leaves the plan's device list holding the graph's buffers
        graph->batch->bound_in = graph->in;
        graph->batch->bound_out = graph->out;
    }
    return record(st);
}

void fftu_graph_destroy(fftu_graph_t graph)
{
    if (!graph) return;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
    record(FFTU_SUCCESS);
}

fftu_status fftu_get_plan_info(fftu_plan_t plan, fftu_plan_info *info)
{
    if (!plan || !info) return record(FFTU_ERROR_INVALID_VALUE);
    if (plan->r2r) {
        // the real plan of the signal, plus the coefficient step (and the sign pass of a DST)
        fftu_status st = fftu_get_plan_info(plan->rc, info);
        if (st != FFTU_SUCCESS) return st;
        info->launches = plan->launches;
        info->table_bytes += plan->table_bytes;
        info->workspace_bytes += plan->ws_bytes;
        return record(FFTU_SUCCESS);
    }
    if (plan->real) {
        // the complex plan of the packed array, plus the split or merge pass
        fftu_status st = fftu_get_plan_info(plan->rc, info);
        if (st != FFTU_SUCCESS) return st;
        info->N = 2 * plan->rd.Nh;
        info->M = info->N / info->P;
        info->launches += 1;
        info->table_bytes += plan->table_bytes;
        return record(FFTU_SUCCESS);
    }
    if (plan->gc) {
        GcPlan gp;
        gp.H = plan->gc_H;
        gp.T = plan->table_T;
        gp.N = plan->grid.N;
        gp.M = plan->grid.M;
        gp.P = plan->grid.N / plan->grid.M;
        gp.phase = plan->gphase;
        gp.phase2 = plan->gphase2;
        gp.pow2 = plan->gc_pow2;
        gp.last_logg = plan->gc_last_logg;
        gp.put = plan->gput;
        fill_info_gc(gp, plan->d, plan->dtype, info);
        return record(FFTU_SUCCESS);
    }
    if (plan->mixed) {
        MixedPlan mp;
        mp.s0 = plan->ms0;
        mp.s2 = plan->ms2;
        mp.g = plan->mg;
        mp.T = plan->table_T;
        mp.fused = plan->mfused;
        fill_info_mixed(mp, plan->dtype, info);
        return record(FFTU_SUCCESS);
    }
    const Geometry G = geometry(plan->d, plan->n, plan->p);
    if (plan->lastx)
        fill_info(G, plan->s0x, true, 0, plan->dtype, info, true);
    else
        fill_info(G, plan->s0, plan->fused, plan->s2.size(), plan->dtype, info);
    return record(FFTU_SUCCESS);
}

const char *fftu_launch_name(fftu_plan_t plan, int i)
{
    if (!plan || i < 0 || i >= int(plan->launch_names.size())) {
        record(FFTU_ERROR_INVALID_VALUE);
        return nullptr;
    }
    record(FFTU_SUCCESS);
    return plan->launch_names[size_t(i)].c_str();
}

size_t fftu_plan_device_bytes(fftu_plan_t plan)
{
    if (!plan) {
        record(FFTU_ERROR_INVALID_VALUE);
        return 0;
    }
    // a real or DCT / DST plan also owns the plan it runs on
    size_t bytes = 0;
    for (const fftu_plan_s *q = plan; q; q = q->rc) bytes += size_t(q->table_bytes + q->ws_bytes);
    record(FFTU_SUCCESS);
    return bytes;
}

fftu_status fftu_execute(fftu_plan_t plan, const void *in, void *out, hipStream_t stream)
{
    if (plan && plan->external) return record(FFTU_ERROR_INVALID_VALUE);   // needs fftu_execute_ws
    return record(execute_with(plan, in, out, plan ? plan->ws : nullptr, stream));
}

fftu_status fftu_execute_ws(fftu_plan_t plan, const void *in, void *out, void *workspace, hipStream_t stream)
{
    fftu_status s = check_exec_args(plan, in, out);
    if (s != FFTU_SUCCESS) return record(s);
    if (!workspace || !aligned(workspace, plan->esize)) return record(FFTU_ERROR_INVALID_VALUE);
    const char *w = static_cast<const char *>(workspace);
    const size_t bytes = size_t(plan->grid.N) * plan->esize;
    for (const void *buf : {in, static_cast<const void *>(out)}) {
        const char *b = static_cast<const char *>(buf);
        if (w < b + bytes && b < w + bytes) return record(FFTU_ERROR_INVALID_VALUE);   // overlaps a buffer
    }
    return record(execute_with(plan, in, out, workspace, stream));
}

fftu_plan_t fftu_plan_convolution(int d, const int64_t n[], const int64_t p[], fftu_dtype dtype)
{
    fftu_plan_s *fwd = build_plan(d, n, p, dtype, FFTU_FORWARD, false);
    if (!fwd) return nullptr;
    fftu_plan_s *inv = build_plan(d, n, p, dtype, FFTU_INVERSE, true);
    if (!inv) {
        const fftu_status st = fftu_last_error();
        fftu_destroy(fwd);
        record(st);
        return nullptr;
    }
    fwd->conv_inv = inv;
    if (fwd->lastx) fwd->launch_names.back() = lastx_kernel_name(fwd->lx, dtype, true);
    record(FFTU_SUCCESS);
    return fwd;
}

fftu_status fftu_execute_convolution(fftu_plan_t plan, const void *in, const void *filter_hat, void *out,
                                     hipStream_t stream)
{
    if (!plan || !plan->conv_inv || !filter_hat || !aligned(filter_hat, plan->esize))
        return record(FFTU_ERROR_INVALID_VALUE);
    fftu_status s = check_exec_args(plan, in, out);
    if (s != FFTU_SUCCESS) return record(s);
    const char *h = static_cast<const char *>(filter_hat);
    const char *o = static_cast<const char *>(out);
    const size_t bytes = size_t(plan->grid.N) * plan->esize;
    if (h < o + bytes && o < h + bytes) return record(FFTU_ERROR_INVALID_VALUE);   // out must not overlap the filter
    s = execute_with(plan, in, out, plan->ws, stream, filter_hat);
    if (s != FFTU_SUCCESS) return record(s);
    return record(execute_with(plan->conv_inv, out, out, plan->ws, stream));
}

fftu_status fftu_pointwise_mul(const void *a, const void *b, void *out, int64_t count, fftu_dtype dtype, double scale,
                               hipStream_t stream)
{
    if (count < 0 || (count > 0 && (!a || !b || !out)) || (dtype != FFTU_C64 && dtype != FFTU_C128))
        return record(FFTU_ERROR_INVALID_VALUE);
    const size_t es = dtype == FFTU_C128 ? 16 : 8;
    if (count > 0 && (!aligned(a, es) || !aligned(b, es) || !aligned(out, es))) return record(FFTU_ERROR_INVALID_VALUE);
    const fftu::Precision prec = dtype == FFTU_C128 ? fftu::Precision::F64 : fftu::Precision::F32;
    return record(from_hip(fftu::launch_pointwise(prec, a, b, out, count, scale, stream)));
}

}  // extern "C"

namespace {

// The transform of `plan` with workspace `ws`; mul (optional) multiplies the
// output pointwise (fused into the exchange, or a separate pass when the
// exchange is not fused).
// Mixed-radix passes from `in` into `out` (the first reads in, the rest work in
// place on out); conj on the chain's first load and last store, scale on the last.
fftu_status run_mixed_passes(const fftu_plan_s *pl, const std::vector<fftu::MixedPassDesc> &passes, const void *in,
                             void *out, int conj_first, int conj_last, double scale_last, hipStream_t stream,
                             Marker *mk = nullptr)
{
    if (passes.empty()) {
        if (in != out)
            return from_hip(hipMemcpyAsync(out, in, size_t(pl->grid.N) * pl->esize, hipMemcpyDeviceToDevice, stream));
        return FFTU_SUCCESS;
    }
    const void *src = in;
    for (size_t i = 0; i < passes.size(); ++i) {
        fftu::MixedPassDesc pd = passes[i];
        pd.conj_in = (i == 0) ? conj_first : 0;
        pd.conj_out = (i + 1 == passes.size()) ? conj_last : 0;
        pd.scale = (i + 1 == passes.size()) ? scale_last : 1.0;
        hipError_t e = fftu::launch_mline(pl->prec, src, out, pd, pl->table, stream);
        if (e != hipSuccess) return from_hip(e);
        if (mk) mk->mark();
        src = out;
    }
    return FFTU_SUCCESS;
}

// The mixed-radix transform: Superstep 0 passes (in -> ws, then in place), the
// twiddle and the permutation in one pass (ws -> out), Superstep 2 passes in
// place on out; conj(F(conj x))/N for the inverse; mul as in execute_with.
fftu_status execute_mixed(fftu_plan_s *plan, const void *in, void *out, void *ws, hipStream_t stream,
                          const void *mul, Marker &mk)
{
    const int inv = plan->dir == FFTU_INVERSE ? 1 : 0;
    const double scale = inv ? 1.0 / double(plan->mg.N) : 1.0;
    fftu_status s = run_mixed_passes(plan, plan->ms0, in, ws, inv, 0, 1.0, stream, &mk);
    if (s != FFTU_SUCCESS) return s;
    fftu::MixedGridDesc g = plan->mg;
    g.conj_in = g.conj_out = 0;
    g.twiddle = 1;
    g.scale = 1.0;
    g.mul = nullptr;
    if (plan->mfused) {
        g.conj_in = plan->ms0.empty() ? inv : 0;
        g.conj_out = inv;
        g.scale = scale;
        g.mul = mul;
        const void *src = ws;
        if (plan->ms0.empty() && in != out) src = in;
        hipError_t e = plan->mx ? fftu::launch_mxexchange(plan->prec, src, out, g, plan->mxs, plan->table, stream)
                                : fftu::launch_mexchange(plan->prec, src, out, g, plan->table, stream);
        if (e == hipSuccess) mk.mark();
        return from_hip(e);
    }
    if (plan->ms2.empty()) {
        g.conj_out = inv;
        g.scale = scale;
    }
    hipError_t e = fftu::launch_mpermute(plan->prec, ws, out, g, plan->table, stream);
    if (e != hipSuccess) return from_hip(e);
    mk.mark();
    if (!plan->ms2.empty()) {
        s = run_mixed_passes(plan, plan->ms2, out, out, 0, inv, scale, stream, &mk);
        if (s != FFTU_SUCCESS) return s;
    }
    if (!mul) return FFTU_SUCCESS;
    return from_hip(fftu::launch_pointwise(plan->prec, out, mul, out, plan->mg.N, 1.0, stream));
}

// Computation phase c of a group-cyclic plan.
bool gc_phase_empty(const fftu_plan_s *pl, int c)
{
    return pl->gc_pow2 ? pl->gphase2[size_t(c)].empty() : pl->gphase[size_t(c)].empty();
}

fftu_status run_gc_phase(const fftu_plan_s *pl, int c, const void *in, void *out, int conj_first, int conj_last,
                         double scale_last, hipStream_t stream, Marker *mk = nullptr)
{
    if (pl->gc_pow2) return run_passes(pl, pl->gphase2[size_t(c)], in, out, conj_first, conj_last, scale_last, stream, mk);
    return run_mixed_passes(pl, pl->gphase[size_t(c)], in, out, conj_first, conj_last, scale_last, stream, mk);
}

// Grids beyond p_max: computation phase 0 (reads `in`), then H times a k_gput
// (twiddle and Put, out of place) and the next phase's passes (in place); with
// power-of-two sides the last Put and phase H run as one k_gplast. The buffers
// alternate between `out` and the workspace so that the last Put lands in `out`:
// phase c runs in `out` when H - c is even.
fftu_status execute_gc(fftu_plan_s *plan, const void *in, void *out, void *ws, hipStream_t stream, const void *mul,
                       Marker &mk)
{
    const int inv = plan->dir == FFTU_INVERSE ? 1 : 0;
    const double scale = inv ? 1.0 / double(plan->grid.N) : 1.0;
    const int H = plan->gc_H;
    auto buf = [&](int c) -> void * { return ((H - c) % 2 == 0) ? out : ws; };
    const bool last_empty = gc_phase_empty(plan, H);
    fftu_status s = run_gc_phase(plan, 0, in, buf(0), inv, 0, 1.0, stream, &mk);
    if (s != FFTU_SUCCESS) return s;
    for (int c = 0; c < H; ++c) {
        fftu::GroupPutDesc g = plan->gput[size_t(c)];
        g.conj_in = (c == 0 && gc_phase_empty(plan, 0)) ? inv : 0;
        g.conj_out = 0;
        g.scale = 1.0;
        if (c == H - 1 && plan->gc_last_logg > 0) {
            // the last Put and phase H's length-p_h FFTs in one pass, the chain's last store
            g.conj_out = inv;
            g.scale = scale;
            hipError_t e = fftu::launch_gplast(plan->prec, buf(c), buf(c + 1), g, plan->table, stream);
            if (e != hipSuccess) return from_hip(e);
            mk.mark();
            break;
        }
        if (c == H - 1 && last_empty) {
            g.conj_out = inv;
            g.scale = scale;
        }
        hipError_t e = fftu::launch_gput(plan->prec, buf(c), buf(c + 1), g, plan->table, stream);
        if (e != hipSuccess) return from_hip(e);
        mk.mark();
        const bool last = c + 1 == H;
        s = run_gc_phase(plan, c + 1, buf(c + 1), buf(c + 1), 0, last ? inv : 0, last ? scale : 1.0, stream, &mk);
        if (s != FFTU_SUCCESS) return s;
    }
    if (!mul) return FFTU_SUCCESS;
    return from_hip(fftu::launch_pointwise(plan->prec, out, mul, out, plan->grid.N, 1.0, stream));
}

fftu_status execute_real(fftu_plan_s *plan, const void *in, void *out, hipStream_t stream, Marker &mk);
fftu_status execute_r2r(fftu_plan_s *plan, const void *in, void *out, hipStream_t stream, Marker &mk);

fftu_status execute_with(fftu_plan_s *plan, const void *in, void *out, void *ws, hipStream_t stream, const void *mul,
                         Marker *outer)
{
    if (plan && plan->r2r) {
        // N reals on each side
        const size_t rsize = plan->esize / 2, bytes = size_t(2 * plan->grid.N) * rsize;
        if (!in || !out || !aligned(in, rsize) || !aligned(out, rsize)) return FFTU_ERROR_INVALID_VALUE;
        const char *a = static_cast<const char *>(in);
        const char *b = static_cast<const char *>(out);
        if (in != out && a < b + bytes && b < a + bytes) return FFTU_ERROR_INVALID_VALUE;   // partial overlap
        Marker mk(plan, stream);
        mk.mark();
        return execute_r2r(plan, in, out, stream, mk);
    }
    if (plan && plan->real) {
        if (!in || !out || !aligned(in, plan->esize) || !aligned(out, plan->esize)) return FFTU_ERROR_INVALID_VALUE;
        if (in != out) {
            const char *a = static_cast<const char *>(in);
            const char *b = static_cast<const char *>(out);
            if (a < b + plan->real_out_elems * plan->esize && b < a + plan->real_in_elems * plan->esize)
                return FFTU_ERROR_INVALID_VALUE;   // partial overlap
        }
        Marker mk(plan, stream);
        mk.mark();
        return execute_real(plan, in, out, stream, mk);
    }
    fftu_status s = check_exec_args(plan, in, out);
    if (s != FFTU_SUCCESS) return s;
    Marker own(plan, stream);
    Marker &mk = outer ? *outer : own;
    if (!outer) mk.mark();   // the start event (an outer marker has recorded its own)
    if (plan->gc) return execute_gc(plan, in, out, ws, stream, mul, mk);
    if (plan->mixed) return execute_mixed(plan, in, out, ws, stream, mul, mk);
    const int inv = plan->dir == FFTU_INVERSE ? 1 : 0;
    const double scale = inv ? 1.0 / double(plan->grid.N) : 1.0;
    const void *src = in;
    if (plan->lastx) {
        if (!plan->s0x.empty()) {
            s = run_passes(plan, plan->s0x, in, ws, inv, 0, 1.0, stream, &mk);
            if (s != FFTU_SUCCESS) return s;
            src = ws;
        } else if (in == out) {
            // k_lastx reads every block of a tile before it writes: not in place
            hipError_t e = hipMemcpyAsync(ws, in, plan->grid.N * plan->esize, hipMemcpyDeviceToDevice, stream);
            if (e != hipSuccess) return from_hip(e);
            src = ws;
        }
        fftu::LastxDesc lx = plan->lx;
        lx.conj_in = plan->s0x.empty() ? inv : 0;
        lx.ex.g.conj_in = 0;
        lx.ex.g.conj_out = inv;
        lx.ex.g.scale = scale;
        lx.ex.mul = mul;
        if (mul) {   // the multiplying instantiation keeps the table in HBM
            lx.table_lds = 0;
            lx.lds_bytes = fftu::lastx_lds_bytes(lx.logl, fftu::lastx_loge(lx.logl, lx.ex.nr * lx.ex.lpr),
                                                 int(plan->esize), lx.lognt);
        }
        hipError_t e = fftu::launch_lastx(plan->prec, src, out, lx, plan->table, stream);
        if (e == hipSuccess) mk.mark();
        return from_hip(e);
    }
    // with ttrans_ld, k_ttranspose runs the innermost dimension's passes of Supersteps 0 and 2
    const std::vector<PassDesc> &s0 = plan->ttrans_ld > 0 ? plan->s0t : plan->s0;
    const std::vector<PassDesc> &s2 = plan->ttrans_ld > 0 ? plan->s2t : plan->s2;
    if (!s0.empty()) {
        s = run_passes(plan, s0, in, ws, inv, 0, 1.0, stream, &mk);
        if (s != FFTU_SUCCESS) return s;
        src = ws;
    } else if (in == out) {
        // the exchange below must not read and write the same buffer
        hipError_t e = hipMemcpyAsync(ws, in, plan->grid.N * plan->esize, hipMemcpyDeviceToDevice, stream);
        if (e != hipSuccess) return from_hip(e);
        src = ws;
    }
    const int conj_first = s0.empty() ? inv : 0;
    if (plan->fused) {
        ExchangeDesc ex = plan->ex;
        ex.g.conj_in = conj_first;
        ex.g.conj_out = inv;
        ex.g.scale = scale;
        ex.mul = mul;
        hipError_t e = fftu::launch_exchange(plan->prec, src, out, ex, plan->table, stream);
        if (e == hipSuccess) mk.mark();
        return from_hip(e);
    }
    GridDesc g = plan->grid;
    g.conj_in = conj_first;
    hipError_t e;
    if (plan->ttrans) {
        // src is the workspace, or the input when it differs from out; the last kernel
        // when no Superstep-2 pass follows
        if (s2.empty()) {
            g.conj_out = inv;
            g.scale = scale;
        }
        e = fftu::launch_ttranspose(plan->prec, src, out, g, plan->ttrans_ld, plan->table, stream);
    } else {
        e = fftu::launch_twiddle(plan->prec, src, ws, g, plan->table, stream);
        if (e == hipSuccess) {
            mk.mark();
            e = fftu::launch_permute(plan->prec, ws, out, plan->grid, stream);
        }
    }
    if (e != hipSuccess) return from_hip(e);
    mk.mark();
    s = run_passes(plan, s2, out, out, 0, inv, scale, stream, &mk);
    if (s != FFTU_SUCCESS || !mul) return s;
    return from_hip(fftu::launch_pointwise(plan->prec, out, mul, out, plan->grid.N, 1.0, stream));
}

}  // namespace

namespace {
// Real-input transforms: forward = the complex transform of the packed array into
// the output, then the split in place; inverse = the merge into the output, then
// the inverse complex transform in place.
// DCT / DST: forward = [signs, unless the complex transform's first pass applies
// them] -> complex transform of the packed signal into the workspace -> split and
// coefficients in one pass; inverse = spectrum from the coefficients -> inverse
// real transform -> [signs, unless its last kernel applies them] (in place on the
// output).
fftu_status execute_r2r(fftu_plan_s *plan, const void *in, void *out, hipStream_t stream, Marker &mk)
{
    fftu_plan_s *rp = plan->rc;
    const bool dst = plan->r2r_kind == FFTU_DST;
    hipError_t e = hipSuccess;
    if (plan->dir == FFTU_FORWARD) {
        const void *sig = in;
        if (dst && !plan->r2r_sign_fused) {
            e = fftu::launch_r2r_sign(plan->prec, in, out, plan->r2d, stream);
            if (e != hipSuccess) return from_hip(e);
            mk.mark();
            sig = out;
        }
        fftu_status s = execute_with(rp->rc, sig, plan->ws, rp->rc->ws, stream, nullptr, &mk);
        if (s != FFTU_SUCCESS) return s;
        e = fftu::launch_r2r_post(plan->prec, plan->ws, out, plan->r2d, plan->rtable, stream);
        if (e == hipSuccess) mk.mark();
        return from_hip(e);
    }
    fftu_status s;
    if (plan->r2r_pre_merge) {
        // the packed spectrum into the output (into the spectrum workspace when the call
        // is in place: other workgroups still read the coefficients), then the inverse
        // complex transform from there into the output
        void *z = in == out ? plan->ws : out;
        e = fftu::launch_r2r_pre_merge(plan->prec, in, z, plan->r2d, plan->rtable, stream);
        if (e != hipSuccess) return from_hip(e);
        mk.mark();
        s = execute_with(rp->rc, z, out, rp->rc->ws, stream, nullptr, &mk);
    } else {
        e = fftu::launch_r2r_pre(plan->prec, in, plan->ws, plan->r2d, plan->rtable, stream);
        if (e != hipSuccess) return from_hip(e);
        mk.mark();
        s = execute_real(rp, plan->ws, out, stream, mk);
    }
    if (s != FFTU_SUCCESS || !dst || plan->r2r_sign_fused) return s;
    e = fftu::launch_r2r_sign(plan->prec, out, out, plan->r2d, stream);
    if (e == hipSuccess) mk.mark();
    return from_hip(e);
}

fftu_status execute_real(fftu_plan_s *plan, const void *in, void *out, hipStream_t stream, Marker &mk)
{
    fftu_plan_s *rc = plan->rc;
    if (plan->dir == FFTU_FORWARD) {
        fftu_status s = execute_with(rc, in, out, rc->ws, stream, nullptr, &mk);
        if (s != FFTU_SUCCESS) return s;
        hipError_t e = fftu::launch_rsplit(plan->prec, out, plan->rd, plan->rtable, stream);
        if (e == hipSuccess) mk.mark();
        return from_hip(e);
    }
    hipError_t e = fftu::launch_rmerge(plan->prec, in, out, plan->rd, plan->rtable, stream);
    if (e != hipSuccess) return from_hip(e);
    mk.mark();
    return execute_with(rc, out, out, rc->ws, stream, nullptr, &mk);
}
}  // namespace

namespace fftu {
bool plan_is_batch(const fftu_plan_s *plan) { return plan->is_batch; }
int plan_device(const fftu_plan_s *plan) { return plan->device; }
size_t plan_workspace_bytes(const fftu_plan_s *plan) { return size_t(plan->grid.N) * plan->esize; }
fftu_status record_status(fftu_status s) { return record(s); }
}  // namespace fftu

extern "C" {

fftu_status fftu_timing_begin(fftu_plan_t plan, int max_calls)
{
    if (!plan || max_calls < 1) return record(FFTU_ERROR_INVALID_VALUE);
    for (hipEvent_t ev : plan->events) (void)hipEventDestroy(ev);
    plan->events.clear();
    const size_t count = size_t(max_calls) * size_t(plan->launches + 1);
    plan->events.reserve(count);
    for (size_t i = 0; i < count; ++i) {
        hipEvent_t ev;
        hipError_t e = hipEventCreate(&ev);
        if (e != hipSuccess) {
            for (hipEvent_t x : plan->events) (void)hipEventDestroy(x);
            plan->events.clear();
            plan->timing_max = 0;
            return record(from_hip(e));
        }
        plan->events.push_back(ev);
    }
    plan->timing_max = max_calls;
    plan->timing_used = 0;
    return record(FFTU_SUCCESS);
}

fftu_status fftu_timing_end(fftu_plan_t plan, float *avg_ms, int capacity, int *nkernels, int *ncalls)
{
    if (!plan || plan->timing_max == 0) return record(FFTU_ERROR_INVALID_VALUE);
    const int L = plan->launches;
    std::vector<double> sum(size_t(L), 0.0);
    fftu_status st = FFTU_SUCCESS;
    for (int c = 0; c < plan->timing_used && st == FFTU_SUCCESS; ++c) {
        for (int i = 0; i < L; ++i) {
            hipEvent_t a = plan->events[size_t(c) * size_t(L + 1) + size_t(i)];
            hipEvent_t b = plan->events[size_t(c) * size_t(L + 1) + size_t(i + 1)];
            float ms = 0.f;
            hipError_t e = hipEventSynchronize(b);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
            if (e != hipSuccess) {
                st = from_hip(e);
                break;
            }
            sum[size_t(i)] += ms;
        }
    }
    const int used = plan->timing_used;
    for (int i = 0; avg_ms && i < L && i < capacity; ++i) avg_ms[i] = used ? float(sum[size_t(i)] / used) : 0.f;
    if (nkernels) *nkernels = L;
    if (ncalls) *ncalls = used;
    for (hipEvent_t ev : plan->events) (void)hipEventDestroy(ev);
    plan->events.clear();
    plan->timing_max = 0;
    plan->timing_used = 0;
    return record(st);
}

fftu_status fftu_stage_local_fft(fftu_plan_t plan, const void *in, void *out, hipStream_t stream)
{
    fftu_status s = check_exec_args(plan, in, out);
    if (s != FFTU_SUCCESS) return record(s);
    if (plan->gc) return record(FFTU_ERROR_INVALID_VALUE);   // several supersteps: fftu_stage_superstep
    const int inv = plan->dir == FFTU_INVERSE ? 1 : 0;
    if (plan->mixed) return record(run_mixed_passes(plan, plan->ms0, in, out, inv, inv, 1.0, stream));
    return record(run_passes(plan, plan->s0, in, out, inv, inv, 1.0, stream));
}

fftu_status fftu_stage_twiddle(fftu_plan_t plan, const void *in, void *out, hipStream_t stream)
{
    fftu_status s = check_exec_args(plan, in, out);
    if (s != FFTU_SUCCESS) return record(s);
    if (plan->gc) return record(FFTU_ERROR_INVALID_VALUE);   // several supersteps: fftu_stage_superstep
    if (plan->mixed) {
        fftu::MixedGridDesc mg = plan->mg;
        mg.conj_in = mg.conj_out = plan->dir == FFTU_INVERSE ? 1 : 0;
        mg.scale = 1.0;
        return record(from_hip(fftu::launch_mtwiddle(plan->prec, in, out, mg, plan->table, stream)));
    }
    GridDesc g = plan->grid;
    g.conj_in = g.conj_out = plan->dir == FFTU_INVERSE ? 1 : 0;
    return record(from_hip(fftu::launch_twiddle(plan->prec, in, out, g, plan->table, stream)));
}

fftu_status fftu_stage_exchange(fftu_plan_t plan, const void *in, void *out, hipStream_t stream)
{
    fftu_status s = check_exec_args(plan, in, out);
    if (s != FFTU_SUCCESS) return record(s);
    if (plan->gc) return record(FFTU_ERROR_INVALID_VALUE);   // several supersteps: fftu_stage_superstep
    if (in == out) return record(FFTU_ERROR_INVALID_VALUE);
    if (plan->mixed) {
        fftu::MixedGridDesc mg = plan->mg;
        mg.conj_in = mg.conj_out = 0;
        mg.twiddle = 0;
        mg.scale = 1.0;
        return record(from_hip(fftu::launch_mpermute(plan->prec, in, out, mg, plan->table, stream)));
    }
    return record(from_hip(fftu::launch_permute(plan->prec, in, out, plan->grid, stream)));
}

fftu_status fftu_stage_remaining_fft(fftu_plan_t plan, const void *in, void *out, hipStream_t stream)
{
    fftu_status s = check_exec_args(plan, in, out);
    if (s != FFTU_SUCCESS) return record(s);
    if (plan->gc) return record(FFTU_ERROR_INVALID_VALUE);   // several supersteps: fftu_stage_superstep
    const int inv = plan->dir == FFTU_INVERSE ? 1 : 0;
    if (plan->mixed) return record(run_mixed_passes(plan, plan->ms2, in, out, inv, inv, 1.0, stream));
    return record(run_passes(plan, plan->s2, in, out, inv, inv, 1.0, stream));
}

fftu_status fftu_stage_superstep(fftu_plan_t plan, int phase, int part, const void *in, void *out, hipStream_t stream)
{
    fftu_status s = check_exec_args(plan, in, out);
    if (s != FFTU_SUCCESS) return record(s);
    const int H = plan->gc ? plan->gc_H : 1;
    const bool ok = (part == 0 && phase >= 0 && phase <= H) || ((part == 1 || part == 2) && phase >= 0 && phase < H);
    if (!ok) return record(FFTU_ERROR_INVALID_VALUE);
    if (!plan->gc) {
        // one superstep: Algorithm 2.3's stages
        if (part == 0) return phase == 0 ? fftu_stage_local_fft(plan, in, out, stream)
                                         : fftu_stage_remaining_fft(plan, in, out, stream);
        return part == 1 ? fftu_stage_twiddle(plan, in, out, stream) : fftu_stage_exchange(plan, in, out, stream);
    }
    const int inv = plan->dir == FFTU_INVERSE ? 1 : 0;
    if (part == 0) return record(run_gc_phase(plan, phase, in, out, inv, inv, 1.0, stream));
    fftu::GroupPutDesc g = plan->gput[size_t(phase)];
    g.scale = 1.0;
    if (part == 1) {
        g.permute = 0;                  // the twiddle alone, element by element
        g.conj_in = g.conj_out = inv;
    } else {
        if (in == out) return record(FFTU_ERROR_INVALID_VALUE);
        g.twiddle = 0;                  // the Put alone: pure data movement
        g.conj_in = g.conj_out = 0;
    }
    return record(from_hip(fftu::launch_gput(plan->prec, in, out, g, plan->table, stream)));
}

void fftu_destroy(fftu_plan_t plan)
{
    if (!plan) return;
    if (plan->conv_inv) {
        fftu_destroy(plan->conv_inv);
        plan->conv_inv = nullptr;
    }
    if (plan->rc) {
        fftu_destroy(plan->rc);
        plan->rc = nullptr;
    }
    int cur = 0;
    const bool have_cur = hipGetDevice(&cur) == hipSuccess;
    if (have_cur && cur != plan->device) (void)hipSetDevice(plan->device);
    for (hipEvent_t ev : plan->events) (void)hipEventDestroy(ev);
    free_batch(plan);
    if (plan->table && !plan->external) (void)hipFree(plan->table);
    if (plan->ws) (void)hipFree(plan->ws);
    if (plan->rtable) (void)hipFree(plan->rtable);
    if (have_cur && cur != plan->device) (void)hipSetDevice(cur);
    delete plan;
    record(FFTU_SUCCESS);
}

}  // extern "C"
