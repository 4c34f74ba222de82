// Host-only check of the planner under AddressSanitizer: fftu_api.cpp is linked
// with launchers that do nothing, and every plan in the list is described and
// created (creation stops at the first HIP call when no device is present).
// Prints one line per case: status of fftu_describe, fftu_plan's status.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "fftu_internal.hpp"

namespace fftu {
hipError_t launch_pass(Precision, const void *, void *, const PassDesc &pd, const void *, hipStream_t)
{
    if (pd.kind == kPair) {
        // a compiled pair of line lengths, whole tiles of columns inside B, LDS within the CU
        const int esize = pd.threads == 256 ? 16 : 8;
        const int lognt = __builtin_ctz(unsigned(pd.threads));
        if (pd.naxes != 2 || pd.loglen[0] < kPairMinLogL || pd.loglen[0] > kPairMaxLogL ||
            pd.loglen[1] < kPairMinLogL || pd.loglen[1] > kPairMaxLogL) std::abort();
        if (lognt != pair_lognt(pd.loglen[0], pd.loglen[1], pd.logB, esize)) std::abort();
        if (pd.logW != pair_logw(pd.loglen[0], pd.loglen[1], lognt) || pd.logB < pd.logW ||
            pd.logTPA != pd.logB - pd.logW || pd.tiles > pair_max_tiles(lognt) ||
            pd.lds_bytes != pair_lds_bytes(pd.loglen[0], pd.loglen[1], lognt, esize) ||
            pd.lds_bytes > (lognt == 10 ? 160u : 80u) * 1024u)
            std::abort();
        return hipSuccess;
    }
    if (pd.kind == kLong) {
        // a compiled line length, rows of at most 4 W columns, LDS within the CU
        const int esize = pd.lds_bytes == long_lds_bytes(pd.loglen[0], 16) ? 16 : 8;
        if (pd.naxes != 1 || pd.loglen[0] < kLongMinLogL || pd.loglen[0] > kLongMaxLogL ||
            pd.logW != long_logw(pd.loglen[0], esize) || pd.logB > pd.logW + 2 || pd.tiles > kLongMaxTiles ||
            pd.lds_bytes != long_lds_bytes(pd.loglen[0], esize) || pd.lds_bytes > 160u * 1024u ||
            pd.threads != kLongThreads)
            std::abort();
        return hipSuccess;
    }
    // every tile of the pass must fit the LDS tile the kernel is compiled for
    if ((int64_t(1) << (pd.logG + pd.logW)) > (int64_t(1) << kLogTileF32)) std::abort();
    return hipSuccess;
}
hipError_t launch_twiddle(Precision, const void *, void *, const GridDesc &, const void *, hipStream_t)
{
    return hipSuccess;
}
hipError_t launch_permute(Precision, const void *, void *, const GridDesc &, hipStream_t) { return hipSuccess; }
hipError_t launch_ttranspose(Precision, const void *in, void *out, const GridDesc &g, int ld, const void *, hipStream_t)
{
    if (ld < 0 || ld > 5 || (ld > 0 && g.logm[g.d - 1] != ld)) std::abort();
    // every q_l = 1, a whole number of 64 x 64 tiles, distinct buffers
    for (int l = 0; l < g.d; ++l)
        if (g.logm[l] != g.logp[l]) std::abort();
    const int logM = g.logmstride[0] + g.logm[0];
    if (logM < 6 || g.N != (int64_t(1) << (2 * logM)) || in == out) std::abort();
    return hipSuccess;
}
hipError_t launch_exchange(Precision, const void *, void *, const ExchangeDesc &ex, const void *, hipStream_t)
{
    if (ex.nh * ex.lph > kExchangeMaxWaveBits || ex.nr * ex.lpr > kExchangeRegBitsF32) std::abort();
    return hipSuccess;
}
hipError_t launch_lastx(Precision, const void *, void *, const LastxDesc &lx, const void *, hipStream_t)
{
    // a compiled split, a tile that divides the block, LDS within the CU, no input conjugation in the exchange
    const ExchangeDesc &ex = lx.ex;
    if (!lastx_split_ok(lx.logl, ex.nr, ex.lpr, ex.nh, ex.lph, lx.lognt) || ex.g.conj_in != 0) std::abort();
    if (lx.lognt != kLastxLogThreads && !lastx_split_needs_1024(lx.logl, ex.nr, ex.lpr, ex.nh, ex.lph)) std::abort();
    const int logp = ex.nr * ex.lpr + ex.nh * ex.lph;
    const int logrw = lx.lognt - (lx.logl - lastx_loge(lx.logl, ex.nr * ex.lpr)) - logp;
    if ((lx.tiles << (logrw + lx.logl)) != ex.g.M || lx.lds_bytes > 160 * 1024) std::abort();
    if (lx.table_lds && (ex.mul || lx.lds_bytes > kLastxTableLdsMax)) std::abort();
    if (ex.g.logm[ex.g.d - 1] != lx.logl) std::abort();
    return hipSuccess;
}
hipError_t launch_batch_reset(const BatchDesc &, hipStream_t) { return hipSuccess; }
hipError_t launch_rsplit(Precision, void *, const RealDesc &rd, const void *, hipStream_t)
{
    if (rd.d < 1 || rd.Nh < 1 || rd.h < 1) std::abort();
    return hipSuccess;
}
hipError_t launch_rmerge(Precision, const void *, void *, const RealDesc &rd, const void *, hipStream_t)
{
    if (rd.d < 1 || rd.Nh < 1 || rd.h < 1) std::abort();
    return hipSuccess;
}
hipError_t launch_gput(Precision, const void *in, void *out, const GroupPutDesc &g, const void *, hipStream_t)
{
    if (g.d < 1 || g.d > kMaxDims || g.N < 1 || g.M < 1 || g.T < 1 || (g.permute && in == out)) std::abort();
    int64_t P = 1, M = 1;
    for (int l = 0; l < g.d; ++l) {
        const GroupPutDim &D = g.dim[l];
        if (D.m < 1 || D.p < 1 || D.mode < 0 || D.mode > 2) std::abort();
        if (D.mode != 0 && (D.pi < 1 || D.p % D.pi || D.ni != D.pi * D.m || g.T % D.ni || D.tstep != g.T / D.ni))
            std::abort();
        if (D.mode == 1 && D.pn * D.m != D.pi) std::abort();
        if (D.mode == 2 && (D.q * D.pi != D.m || int64_t(D.mh) * D.pi != D.p)) std::abort();
        P *= D.p;
        M *= D.m;
    }
    if (M != g.M || P * M != g.N) std::abort();
    return hipSuccess;
}
hipError_t launch_gplast(Precision prec, const void *in, void *out, const GroupPutDesc &g, const void *t,
                         hipStream_t st)
{
    int logg = 0;
    for (int l = 0; l < g.d; ++l) {
        const GroupPutDim &D = g.dim[l];
        if (D.mode == 1) std::abort();             // the last Put: every dimension in mode 0 or 2
        if (D.mode == 2) logg += __builtin_ctz(unsigned(D.pi));
        if ((D.m & (D.m - 1)) || (D.p & (D.p - 1))) std::abort();
    }
    if (logg < 1 || logg > kGplastMaxLogG) std::abort();
    return launch_gput(prec, in, out, g, t, st);
}
bool gput_tiling(const GroupPutDesc &, int, GputTileDesc &) { return false; }
hipError_t launch_mxexchange(Precision, const void *in, void *out, const MixedGridDesc &g, const MxSplit &sp,
                             const void *, hipStream_t)
{
    if (in == out || g.d < 1 || g.P < 2 || (int64_t(1) << (sp.nr * sp.lpr + sp.nh * sp.lph)) != g.P) std::abort();
    return hipSuccess;
}
hipError_t launch_r2r_post(Precision, const void *, void *, const R2RDesc &g, const void *, hipStream_t)
{
    if (g.d < 1 || g.d > kR2RMaxDims || g.groups < 1) std::abort();
    return hipSuccess;
}
hipError_t launch_r2r_pre(Precision, const void *, void *, const R2RDesc &g, const void *, hipStream_t)
{
    if (g.d < 1 || g.d > kR2RMaxDims || g.groups < 1) std::abort();
    return hipSuccess;
}
hipError_t launch_r2r_pre_merge(Precision, const void *, void *, const R2RDesc &g, const void *, hipStream_t)
{
    if (g.d < 2 || g.d > kR2RMaxDims || g.groups < 1 || r2rpre_merge_lds(g, 16) == 0) std::abort();
    return hipSuccess;
}
hipError_t launch_r2r_sign(Precision, const void *, void *, const R2RDesc &g, hipStream_t)
{
    if (g.d < 1 || g.d > kR2RMaxDims) std::abort();
    return hipSuccess;
}
hipError_t launch_batch_bind(BatchBind *, const BindChunk &c, hipStream_t)
{
    if (c.count < 1 || c.count > kBindChunk || c.first < 0) std::abort();
    return hipSuccess;
}
hipError_t launch_fill_uniform(Precision, void *, int64_t, uint32_t, uint32_t, uint64_t, hipStream_t) { return hipSuccess; }
hipError_t launch_pointwise(Precision, const void *, const void *, void *, int64_t, double, hipStream_t) { return hipSuccess; }
hipError_t launch_mline(Precision prec, const void *, void *, const MixedPassDesc &pd, const void *, hipStream_t)
{
    // the tile fits the prefetch registers and its LDS; the tiles cover the lines
    const int64_t pre = prec == Precision::F64 ? kMixedPreF64 : kMixedPreF32;
    const int64_t esize = prec == Precision::F64 ? 16 : 8;
    int64_t prod = 1;
    for (int s = 0; s < pd.nstages; ++s) prod *= pd.radix[s];
    if (pd.nstages < 1 || prod != pd.L || int64_t(pd.W) * pd.L > pre * kMixedThreads ||
        (2 * pd.W * pd.pitch + pd.L) * esize != int64_t(pd.lds_bytes) || pd.tiles != (pd.A * pd.B + pd.W - 1) / pd.W)
        std::abort();
    return hipSuccess;
}
hipError_t launch_mtwiddle(Precision, const void *, void *, const MixedGridDesc &, const void *, hipStream_t) { return hipSuccess; }
hipError_t launch_mpermute(Precision, const void *, void *, const MixedGridDesc &, const void *, hipStream_t) { return hipSuccess; }
hipError_t launch_mexchange(Precision, const void *, void *, const MixedGridDesc &g, const void *, hipStream_t)
{
    if (g.P > kMexMaxP || g.T > (int64_t(1) << 24)) std::abort();
    for (int l = 0; l < g.d; ++l)
        if (!mexchange_radix_ok(g.p[l])) std::abort();
    return hipSuccess;
}
hipError_t launch_batch(Precision, const BatchDesc &bd, const void *, uint32_t, uint32_t, hipStream_t)
{
    if (bd.nstages < 1 || bd.nitems < 1) std::abort();
    return hipSuccess;
}
int batch_blocks_per_cu(Precision, uint32_t) { return 1; }
}  // namespace fftu

// Emulates the persistent batch kernel's schedule on the work list: `nwg`
// workgroups take items from one counter in order, wait until the item's
// dependency descriptor has finished every item, and finish after a random
// number of steps. Fails on a deadlock, a miscount or an out-of-range tile.
static int emulate_schedule(const fftu::BatchWorklist &wl, int nwg, unsigned seed)
{
    const int K = int(wl.stages.size());
    std::vector<int> done(size_t(K), 0), handed(size_t(K), 0);
    struct WG {
        int64_t item = -1;
        int k = -1;
        int left = 0;
        bool finished = false;
    };
    std::vector<WG> wgs(static_cast<size_t>(nwg));
    int64_t next = 0, completed = 0;
    unsigned rng = seed;
    auto rnd = [&]() { rng = rng * 1664525u + 1013904223u; return rng >> 8; };
    for (int64_t step = 0; step < 100000000; ++step) {
        bool all_done = true;
        for (WG &w : wgs) {
            if (w.finished) continue;
            all_done = false;
            if (w.item < 0) {
                w.item = next++;
                if (w.item >= wl.items) {
                    w.finished = true;
                    continue;
                }
                int lo = 0, hi = K - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (wl.starts[size_t(mid)] <= w.item) lo = mid;
                    else hi = mid - 1;
                }
                w.k = lo;
                const int64_t t = w.item - wl.starts[size_t(lo)];
                const fftu::BatchStage &st = wl.stages[size_t(lo)];
                if (st.per_item < 1 || t * st.per_item >= st.tiles) return 101;
                if (st.kind == fftu::kExchangeStage) {
                    const int64_t M = st.ex.g.M;
                    if (st.tiles * 4 * 64 < M || (st.tiles - 1) * 4 * 64 >= M) return 100;
                } else if (st.tiles != st.pd.tiles) {
                    return 104;
                }
                handed[size_t(lo)]++;
                w.left = -1;   // not started: waiting on the dependency
            }
            if (w.left < 0) {
                const int dep = wl.dep[size_t(w.k)];
                if (dep >= 0 && done[size_t(dep)] < int(wl.starts[size_t(dep) + 1] - wl.starts[size_t(dep)])) continue;
                w.left = int(rnd() % 5);
            }
            if (w.left-- == 0) {
                done[size_t(w.k)]++;
                ++completed;
                w.item = -1;
            }
        }
        if (all_done) break;
    }
    if (completed != wl.items) return 102;
    for (int k = 0; k < K; ++k)
        if (done[size_t(k)] != int(wl.starts[size_t(k) + 1] - wl.starts[size_t(k)]) || handed[size_t(k)] != done[size_t(k)])
            return 103;
    return 0;
}

static int check_worklists()
{
    int bad = 0;
    unsigned rng = 12345u;
    for (int trial = 0; trial < 6; ++trial) {
        const int count = trial == 0 ? 1 : 3 + 40 * trial;
        std::vector<std::vector<int64_t>> ns, ps;
        std::vector<int> d;
        for (int f = 0; f < count; ++f) {
            std::vector<int64_t> n(3), p(3, 2);
            for (int l = 0; l < 3; ++l) {
                rng = rng * 1664525u + 1013904223u;
                n[size_t(l)] = int64_t(1) << (4 + (rng >> 8) % 5);   // 16 .. 256
            }
            ns.push_back(n);
            ps.push_back(p);
            d.push_back(3);
        }
        std::vector<const int64_t *> np, pp;
        for (int f = 0; f < count; ++f) {
            np.push_back(ns[size_t(f)].data());
            pp.push_back(ps[size_t(f)].data());
        }
        for (fftu_dtype dt : {FFTU_C64, FFTU_C128}) {
            fftu::BatchWorklist wl;
            if (fftu::build_batch_worklist(count, d.data(), np.data(), pp.data(), dt, FFTU_FORWARD, wl) !=
                FFTU_SUCCESS) {
                ++bad;
                continue;
            }
            for (int nwg : {1, 3, 64, 700}) {
                const int r = emulate_schedule(wl, nwg, 7u + unsigned(trial));
                std::printf("worklist count=%d dt=%d items=%lld wgs=%d -> %d\n", count, int(dt),
                            (long long)wl.items, nwg, r);
                if (r) ++bad;
            }
        }
    }
    return bad;
}

// Batch plans: the planner builds every descriptor before its first HIP call.
static int check_batches()
{
    const int64_t n1[3] = {16, 256, 64}, p1[3] = {2, 2, 2};
    const int64_t n2[3] = {256, 16, 32}, p2[3] = {2, 2, 2};
    const int64_t n3[2] = {64, 128}, p3[2] = {2, 2};
    const int64_t n4[3] = {1024, 16, 16}, p4[3] = {2, 2, 2};   // local length 512: outside a batch
    const int d[3] = {3, 3, 2};
    const int64_t *ns[3] = {n1, n2, n3}, *ps[3] = {p1, p2, p3};
    int bad = 0;
    for (fftu_dtype dt : {FFTU_C64, FFTU_C128}) {
        fftu_plan_t pl = fftu_plan_batch(3, d, ns, ps, dt, FFTU_FORWARD);
        std::printf("batch plan=%d\n", int(fftu_last_error()));
        if (pl) fftu_destroy(pl);
        else if (fftu_last_error() != FFTU_ERROR_DEVICE) ++bad;
    }
    const int d4[1] = {3};
    const int64_t *ns4[1] = {n4}, *ps4[1] = {p4};
    if (fftu_plan_batch(1, d4, ns4, ps4, FFTU_C64, FFTU_FORWARD) || fftu_last_error() != FFTU_ERROR_UNSUPPORTED) ++bad;
    return bad;
}

int main()
{
    struct Case {
        std::vector<int64_t> n, p;
    };
    const std::vector<Case> cases = {
        {{512, 512, 512}, {4, 4, 4}}, {{64, 64, 64}, {8, 8, 2}}, {{4, 4, 4, 4, 4, 4, 4, 4}, {2, 2, 2, 2, 2, 2, 2, 2}},
        {{1024, 1024, 1024}, {32, 32, 32}}, {{1}, {1}}, {{2048}, {1}}, {{4096}, {64}}, {{64, 64, 64, 64, 64}, {2, 2, 2, 2, 2}},
        {{16, 16}, {4, 4}}, {{8, 1, 4}, {2, 1, 1}}, {{1 << 22, 64}, {2048, 8}}, {{256, 256, 256, 256}, {16, 16, 16, 16}},
        // k_pair, k_long and k_ttranspose plans
        {{16, 16, 16, 32, 64}, {2, 2, 2, 2, 2}}, {{64, 64, 32, 64}, {2, 2, 2, 2}}, {{32, 32, 64, 128}, {1, 1, 1, 1}},
        {{1 << 24, 64}, {4096, 8}}, {{8192, 16}, {2, 2}}, {{4096, 32}, {2, 2}}, {{8, 4096, 16}, {2, 2, 2}},
        {{1024, 64}, {32, 8}}, {{64, 64, 64}, {8, 8, 8}},
        // mixed radix (factors 2, 3, 5, 7), and one side with a factor 11 (unsupported)
        {{60, 60}, {2, 2}}, {{49, 27, 8}, {7, 3, 2}}, {{1000}, {10}}, {{126, 12, 1}, {3, 2, 1}}, {{44, 12}, {2, 2}},
        // grids beyond p_max: group-cyclic levels, several supersteps
        {{512, 512, 512}, {32, 32, 32}}, {{16, 16}, {8, 2}}, {{1024}, {64}}, {{64, 64, 64}, {16, 16, 8}},
        {{8, 27}, {4, 9}}, {{16}, {8}},
        // complex128 lines of 4096 (k_long with one line per tile) in both supersteps
        {{1 << 24, 2}, {4096, 1}},
    };
    int bad = 0;
    for (const Case &c : cases) {
        for (fftu_dtype dt : {FFTU_C64, FFTU_C128}) {
            fftu_plan_info info{};
            fftu_status s = fftu_describe(int(c.n.size()), c.n.data(), c.p.data(), dt, FFTU_FORWARD, &info);
            fftu_plan_t pl = fftu_plan(int(c.n.size()), c.n.data(), c.p.data(), dt, FFTU_INVERSE);
            fftu_status ps = fftu_last_error();
            if (pl) {
                std::vector<char> dummy(16);
                fftu_execute(pl, dummy.data(), dummy.data() + 8, nullptr);
                fftu_destroy(pl);
            }
            std::printf("describe=%d plan=%d launches=%d\n", int(s), int(ps), info.launches);
            if (s != FFTU_SUCCESS && s != FFTU_ERROR_UNSUPPORTED) ++bad;
        }
    }
    return bad + check_batches() + check_worklists();
}
