// Device input generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC'11), counter-based, so element e of a
// buffer is a pure function of (key, e) and the same stream can be reproduced
// anywhere (a host implementation of the same definition reproduces it bit for
// bit).
//
// One Philox round on a 4 x 32-bit counter (c0, c1, c2, c3) with key (k0, k1):
//   (h0, l0) = M0 * c0, (h1, l1) = M1 * c2 (64-bit products split in halves),
//   (c0, c1, c2, c3) <- (h1 ^ c1 ^ k0, l1, h0 ^ c3 ^ k1, l0),
// and between rounds the key is bumped by the Weyl constants (W0, W1).
// Ten rounds.
//
// Element e of the buffer uses counter (e mod 2^32, e div 2^32, 0, 0) and maps
// the four output words x0..x3 to a complex value with components in [-1, 1):
//   complex64:  re = (x0 >> 8) 2^-23 - 1, im = (x1 >> 8) 2^-23 - 1
//   complex128: re = (x0 2^21 + (x1 >> 11)) 2^-52 - 1, im = (x2 2^21 + (x3 >> 11)) 2^-52 - 1
// Every step is exact (integers below 2^24 or 2^53 scaled by powers of two).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fftu_device.hpp"
#include "fftu_internal.hpp"

namespace fftu {

namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

__device__ __forceinline__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        const uint64_t p0 = uint64_t(kPhiloxM0) * c[0];
        const uint64_t p1 = uint64_t(kPhiloxM1) * c[2];
        const uint32_t n0 = uint32_t(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = uint32_t(p0 >> 32) ^ c[3] ^ k1;
        c[1] = uint32_t(p1);
        c[3] = uint32_t(p0);
        c[0] = n0;
        c[2] = n2;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill_uniform(cx<T> *out, int64_t count, uint32_t k0, uint32_t k1,
                                                      uint64_t base)
{
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < count; e += stride) {
        const uint64_t ctr = base + uint64_t(e);
        uint32_t c[4] = {uint32_t(ctr), uint32_t(ctr >> 32), 0u, 0u};
        philox4x32_10(c, k0, k1);
        cx<T> v;
        if constexpr (sizeof(T) == 4) {
            v.x = float(int32_t(c[0] >> 8)) * 0x1p-23f - 1.0f;
            v.y = float(int32_t(c[1] >> 8)) * 0x1p-23f - 1.0f;
        } else {
            v.x = double(int64_t((uint64_t(c[0]) << 21) | (c[1] >> 11))) * 0x1p-52 - 1.0;
            v.y = double(int64_t((uint64_t(c[2]) << 21) | (c[3] >> 11))) * 0x1p-52 - 1.0;
        }
        out[e] = v;
    }
}

}  // namespace

hipError_t launch_fill_uniform(Precision prec, void *out, int64_t count, uint32_t k0, uint32_t k1, uint64_t base,
                               hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    const int64_t want = (count + 255) / 256;
    const uint32_t blocks = uint32_t(want < (int64_t(1) << 16) ? want : (int64_t(1) << 16));
    if (prec == Precision::F64)
        hipLaunchKernelGGL(k_fill_uniform<double>, dim3(blocks), dim3(256), 0, stream, static_cast<cx<double> *>(out),
                           count, k0, k1, base);
    else
        hipLaunchKernelGGL(k_fill_uniform<float>, dim3(blocks), dim3(256), 0, stream, static_cast<cx<float> *>(out),
                           count, k0, k1, base);
    return hipGetLastError();
}

}  // namespace fftu
