// Pointwise product of two arrays in the same layout: out[i] = a[i] b[i] scale.
//
// The transform starts and ends in the same cyclic distribution (Algorithm 2.3
// of arXiv 2203.11795), so a product of two spectra, e.g. between a forward and
// an inverse transform in a circular convolution, needs no reordering: it is
// elementwise in the buffer layout. HBM bound: 3 N b bytes per launch.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fftu_device.hpp"
#include "fftu_internal.hpp"

namespace fftu {

namespace {

template <typename T>
__global__ __launch_bounds__(256) void k_pointwise(const cx<T> *a, const cx<T> *b,
                                                   cx<T> *out, int64_t count, T scale)
{
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += stride) {
        cx<T> v = cmul(a[i], b[i]);
        if (scale != T(1)) v = {v.x * scale, v.y * scale};
        out[i] = v;
    }
}

}  // namespace

hipError_t launch_pointwise(Precision prec, const void *a, const void *b, void *out, int64_t count, double scale,
                            hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    const int64_t want = (count + 255) / 256;
    const uint32_t blocks = uint32_t(want < (int64_t(1) << 16) ? want : (int64_t(1) << 16));
    if (prec == Precision::F64)
        hipLaunchKernelGGL(k_pointwise<double>, dim3(blocks), dim3(256), 0, stream,
                           static_cast<const cx<double> *>(a), static_cast<const cx<double> *>(b),
                           static_cast<cx<double> *>(out), count, scale);
    else
        hipLaunchKernelGGL(k_pointwise<float>, dim3(blocks), dim3(256), 0, stream, static_cast<const cx<float> *>(a),
                           static_cast<const cx<float> *>(b), static_cast<cx<float> *>(out), count, float(scale));
    return hipGetLastError();
}

}  // namespace fftu
