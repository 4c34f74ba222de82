// k_lastx for complex64 (see fftu_lastx.hpp).
#include "fftu_lastx.hpp"

namespace fftu {

hipError_t launch_lastx_f32(const void *in, void *out, const LastxDesc &lx, const void *table, hipStream_t stream)
{
    return launch_lastx_t<float>(in, out, lx, table, stream);
}

}  // namespace fftu
