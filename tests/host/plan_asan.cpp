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
    // every tile of the pass must fit the LDS tile the kernel is compiled for
    if ((int64_t(1) << (pd.logG + pd.logW)) > (int64_t(1) << kLogTileF32)) std::abort();
    return hipSuccess;
}
hipError_t launch_twiddle(Precision, const void *, void *, const GridDesc &, const void *, hipStream_t)
{
    return hipSuccess;
}
hipError_t launch_permute(Precision, const void *, void *, const GridDesc &, hipStream_t) { return hipSuccess; }
hipError_t launch_exchange(Precision, const void *, void *, const ExchangeDesc &ex, const void *, hipStream_t)
{
    if (ex.nh * ex.lph > kExchangeMaxWaveBits || ex.nr * ex.lpr > kExchangeRegBitsF32) std::abort();
    return hipSuccess;
}
hipError_t launch_batch(Precision, const BatchDesc &bd, const void *, uint32_t, uint32_t, hipStream_t)
{
    if (bd.nstages < 1 || bd.nitems < 1) std::abort();
    return hipSuccess;
}
int batch_blocks_per_cu(Precision, uint32_t) { return 1; }
}  // namespace fftu

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
    return bad + check_batches();
}
