// The real-input transform in the cyclic distribution (the real-to-complex FFT
// that arXiv 2203.11795, Section 6, names as the method's next transform, built
// from 1-D pieces dimension by dimension).
//
// Layout: the real array X of n_1 x ... x n_d (n_d even) travels as its packed
// complex view z[j', j] = X[j', 2j] + i X[j', 2j + 1] of shape n' = (n_1, ...,
// n_{d-1}, h), h = n_d / 2, in the cyclic distribution over p. Its transform Z =
// F(z) (the complex path of the library) gives the spectrum of X through the even
// and odd halves of the last dimension: with E = (Z[k] + conj Z[-k]) / 2 and
// O = (Z[k] - conj Z[-k]) / (2i) (indices negated mod n' in every dimension),
//     Y[k', k] = E + omega_{n_d}^k O,   Y[k', h] = E[k', 0] - O[k', 0].
// The output is the half spectrum Y[k', k], k < h, in the cyclic layout of n'
// over p (the layout of the input), then the Nyquist plane Y[k', h] cyclic over
// (p_1, ..., p_{d-1}). The inverse runs the other way: Z = E + i O with
// E = (Y[k] + Y[k + h]) / 2, O = (Y[k] - Y[k + h]) omega_{n_d}^{-k} / 2, where
// Y[k', k + h] = conj Y[-k', h - k] for 0 < k < h and the plane for k = 0; then
// the inverse complex transform of Z (times 1 / (N/2)) is z, the packed result.
//
// Both steps are one pass each. A thread takes an element and its partner (-k,
// or (-k', h - k) in the inverse), which are each other's partners, reads both
// and writes both, so the steps run in place; the thread of the lower position
// of a pair does the work.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "fftu_device.hpp"
#include "fftu_internal.hpp"

namespace fftu {

namespace {

// Global index k (natural coordinates of n') of buffer position `pos` < Nh; D = rd.d
// as a compile-time constant, so that the loops unroll and k stays in registers.
template <int D>
__device__ __forceinline__ void coords(const RealDesc &rd, int64_t pos, int32_t (&k)[kMaxDims])
{
    uint32_t r = uint32_t(pos / rd.Mh);
    uint32_t i = uint32_t(pos - int64_t(r) * rd.Mh);
#pragma unroll
    for (int l = D - 1; l >= 0; --l) {
        const uint32_t sl = r % uint32_t(rd.p[l]);
        r /= uint32_t(rd.p[l]);
        const uint32_t il = i % uint32_t(rd.m[l]);
        i /= uint32_t(rd.m[l]);
        k[l] = int32_t(sl + il * uint32_t(rd.p[l]));
    }
}

// Buffer position of global index k of n' (DIMS = D), or of the Nyquist plane's
// index k' (DIMS = D - 1, after the Nh packed elements).
template <int D, int DIMS>
__device__ __forceinline__ int64_t position(const RealDesc &rd, const int32_t (&k)[kMaxDims])
{
    uint32_t r = 0, i = 0;
#pragma unroll
    for (int l = 0; l < DIMS; ++l) {
        r = r * uint32_t(rd.p[l]) + uint32_t(k[l]) % uint32_t(rd.p[l]);
        i = i * uint32_t(rd.m[l]) + uint32_t(k[l]) / uint32_t(rd.p[l]);
    }
    return DIMS == D ? int64_t(r) * rd.Mh + i : rd.Nh + int64_t(r) * rd.Mp + i;
}

template <typename T>
__device__ __forceinline__ cx<T> half_of(cx<T> a) { return {a.x * T(0.5), a.y * T(0.5)}; }

}  // namespace

template <typename T, int D>
__global__ __launch_bounds__(256) void k_rsplit(cx<T> *buf, const RealDesc rd, const cx<T> *__restrict__ table)
{
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t pos = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; pos < rd.Nh; pos += stride) {
        int32_t k[kMaxDims], kk[kMaxDims];
        coords<D>(rd, pos, k);
        #pragma unroll
        for (int l = 0; l < D; ++l) kk[l] = k[l] == 0 ? 0 : rd.n[l] - k[l];
        const int64_t ppos = position<D, D>(rd, kk);
        if (ppos < pos) continue;                       // the partner's thread does this pair
        const cx<T> a = buf[pos], b = buf[ppos];
        // E = (a + conj b) / 2, O = (a - conj b) / (2i); at the partner conj E and conj O
        const cx<T> E = half_of(cx<T>{a.x + b.x, a.y - b.y});
        const cx<T> O = half_of(cx<T>{a.y + b.y, b.x - a.x});
        const int kd = k[D - 1], kkd = kk[D - 1];
        const cx<T> y = E + cmul(table[kd], O);
        const cx<T> Ec = {E.x, -E.y}, Oc = {O.x, -O.y};
        const cx<T> yy = Ec + cmul(table[kkd], Oc);
        buf[pos] = y;
        if (ppos != pos) buf[ppos] = yy;
        if (kd == 0) {
            // the Nyquist plane: omega_{n_d}^h = -1
            buf[position<D, D - 1>(rd, k)] = E - O;
            if (ppos != pos) buf[position<D, D - 1>(rd, kk)] = Ec - Oc;
        }
    }
}

template <typename T, int D>
__global__ __launch_bounds__(256) void k_rmerge(const cx<T> *in, cx<T> *out, const RealDesc rd,
                                                const cx<T> *__restrict__ table)
{
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t pos = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; pos < rd.Nh; pos += stride) {
        int32_t k[kMaxDims], kk[kMaxDims];
        coords<D>(rd, pos, k);
        const int kd = k[D - 1];
        if (kd == 0) {
            // Y[k', h] is the plane's element k'
            const cx<T> a = in[pos], c = in[position<D, D - 1>(rd, k)];
            const cx<T> E = half_of(a + c), O = half_of(a - c);
            out[pos] = {E.x - O.y, E.y + O.x};          // E + i O
            continue;
        }
        #pragma unroll
        for (int l = 0; l < D - 1; ++l) kk[l] = k[l] == 0 ? 0 : rd.n[l] - k[l];
        kk[D - 1] = rd.h - kd;
        const int64_t ppos = position<D, D>(rd, kk);
        if (ppos < pos) continue;
        const cx<T> a = in[pos], b = in[ppos];
        // Y[k + h] = conj b: E = (a + conj b) / 2, O = (a - conj b) omega^{-k} / 2;
        // at the partner conj E and conj O
        const cx<T> E = half_of(cx<T>{a.x + b.x, a.y - b.y});
        const cx<T> w = table[kd];
        const cx<T> O = cmul(half_of(cx<T>{a.x - b.x, a.y + b.y}), cx<T>{w.x, -w.y});
        const cx<T> z = {E.x - O.y, E.y + O.x};
        const cx<T> zz = {E.x + O.y, O.x - E.y};        // conj E + i conj O
        out[pos] = z;
        if (ppos != pos) out[ppos] = zz;
    }
}

hipError_t launch_rsplit(Precision prec, void *buf, const RealDesc &rd, const void *table, hipStream_t stream)
{
    const int64_t want = (rd.Nh + 255) / 256;
    const uint32_t blocks = uint32_t(want < 65536 ? (want > 0 ? want : 1) : 65536);
    auto go = [&](auto dc) {
        constexpr int D = decltype(dc)::value;
        if (prec == Precision::F64)
            hipLaunchKernelGGL((k_rsplit<double, D>), dim3(blocks), dim3(256), 0, stream,
                               static_cast<cx<double> *>(buf), rd, static_cast<const cx<double> *>(table));
        else
            hipLaunchKernelGGL((k_rsplit<float, D>), dim3(blocks), dim3(256), 0, stream,
                               static_cast<cx<float> *>(buf), rd, static_cast<const cx<float> *>(table));
    };
    static_assert(kMaxDims == 8, "k_rsplit / k_rmerge: one instantiation per dimension count");
    switch (rd.d) {
    case 1: go(std::integral_constant<int, 1>{}); break;
    case 2: go(std::integral_constant<int, 2>{}); break;
    case 3: go(std::integral_constant<int, 3>{}); break;
    case 4: go(std::integral_constant<int, 4>{}); break;
    case 5: go(std::integral_constant<int, 5>{}); break;
    case 6: go(std::integral_constant<int, 6>{}); break;
    case 7: go(std::integral_constant<int, 7>{}); break;
    case 8: go(std::integral_constant<int, 8>{}); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_rmerge(Precision prec, const void *in, void *out, const RealDesc &rd, const void *table,
                         hipStream_t stream)
{
    const int64_t want = (rd.Nh + 255) / 256;
    const uint32_t blocks = uint32_t(want < 65536 ? (want > 0 ? want : 1) : 65536);
    auto go = [&](auto dc) {
        constexpr int D = decltype(dc)::value;
        if (prec == Precision::F64)
            hipLaunchKernelGGL((k_rmerge<double, D>), dim3(blocks), dim3(256), 0, stream,
                               static_cast<const cx<double> *>(in), static_cast<cx<double> *>(out), rd,
                               static_cast<const cx<double> *>(table));
        else
            hipLaunchKernelGGL((k_rmerge<float, D>), dim3(blocks), dim3(256), 0, stream,
                               static_cast<const cx<float> *>(in), static_cast<cx<float> *>(out), rd,
                               static_cast<const cx<float> *>(table));
    };
    static_assert(kMaxDims == 8, "k_rsplit / k_rmerge: one instantiation per dimension count");
    switch (rd.d) {
    case 1: go(std::integral_constant<int, 1>{}); break;
    case 2: go(std::integral_constant<int, 2>{}); break;
    case 3: go(std::integral_constant<int, 3>{}); break;
    case 4: go(std::integral_constant<int, 4>{}); break;
    case 5: go(std::integral_constant<int, 5>{}); break;
    case 6: go(std::integral_constant<int, 6>{}); break;
    case 7: go(std::integral_constant<int, 7>{}); break;
    case 8: go(std::integral_constant<int, 8>{}); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fftu
