// k_lastx for complex128 (see fftu_lastx.hpp), and the launcher for both types.
#include "fftu_lastx.hpp"

namespace fftu {

hipError_t launch_lastx_f64(const void *in, void *out, const LastxDesc &lx, const void *table, hipStream_t stream)
{
    return launch_lastx_t<double>(in, out, lx, table, stream);
}

hipError_t launch_lastx(Precision prec, const void *in, void *out, const LastxDesc &lx, const void *table,
                        hipStream_t stream)
{
    return prec == Precision::F64 ? launch_lastx_f64(in, out, lx, table, stream)
                                  : launch_lastx_f32(in, out, lx, table, stream);
}

}  // namespace fftu
