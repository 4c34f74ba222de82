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
}  // namespace fftu

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
    return bad;
}
