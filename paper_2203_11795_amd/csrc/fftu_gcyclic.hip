// Processor grids beyond p_max = sqrt(N) (arXiv 2203.11795, Section 2.3, the
// paragraph after eq. (2.13)): when p_l^2 does not divide n_l, the transform
// needs more than one communication superstep and the group-cyclic
// distribution (cycle c: blocks of c n / p elements, each cyclic over a group of
// c processors; x_j on P((j div (c n/p)) c + j mod c)).
//
// Per dimension, with m = n / p elements per processor, level i holds
// sub-transforms of n_i points, one per group of p_i processors (the level's
// array in the group-cyclic distribution with cycle p_i). Each level is
// Algorithm 2.2 on its groups: local F_m, the twiddle omega_{n_i}^{u k} (u = member
// of the group, k = local index), and a Put. Below the last level the Put sends
// sub-transform k of group b (the values z^(u)_k, u in [p_i]) to group b m + k of
// the next level, cyclically over its p_{i+1} = p_i / m members; the last level
// (p_h^2 | n_h) ends with Algorithm 2.2's Put and length-p_h FFTs, and its Put
// addresses the processors of the cyclic distribution directly: member rho of
// group b is processor rho m^h + rev(b), rev = the base-m digit reversal of b
// over h digits. So the transform starts and ends in the cyclic distribution.
//
// k_gput is one communication superstep for all dimensions at once (each
// dimension moves its own processor and local coordinates), gathered per output
// element: for the destination (processor r', local j') it finds the source
// (r, k) dimension by dimension, applies the level's twiddle of the source
// element (exponent reduced exactly in integers: one table entry of omega_T,
// T = lcm(n_l)), and stores. 32-bit index arithmetic: N < 2^31.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fftu_device.hpp"
#include "fftu_internal.hpp"

namespace fftu {

template <typename T>
__global__ __launch_bounds__(256) void k_gput(const cx<T> *__restrict__ in, cx<T> *__restrict__ out,
                                              const GroupPutDesc g, const cx<T> *__restrict__ table)
{
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    const T scale = static_cast<T>(g.scale);
    const uint32_t M = uint32_t(g.M);
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < g.N; i += stride) {
        uint32_t r = uint32_t(i / M);
        uint32_t j = uint32_t(i - int64_t(r) * M);
        uint32_t src_rank = 0, src_k = 0, rmul = 1, kmul = 1;
        uint32_t e = 0;                            // sum of terms below T <= 2^24, kept below T
        for (int l = g.d - 1; l >= 0; --l) {
            const GroupPutDim &D = g.dim[l];
            const uint32_t m = uint32_t(D.m), pi = uint32_t(D.pi);
            const uint32_t jl = j % m;
            j /= m;
            const uint32_t rl = r % uint32_t(D.p);
            r /= uint32_t(D.p);
            uint32_t sr = rl, sk = jl;             // source coordinates along this dimension
            uint32_t u = 0, k = 0;                 // the twiddle's member and local index
            if (D.mode == 1 && g.permute) {
                // destination: member rl mod p_{i+1} of group b' = rl div p_{i+1}, local jl;
                // it came from member u = rl mod p_{i+1} + p_{i+1} jl of group b' div m, index b' mod m
                const uint32_t pn = uint32_t(D.pn);
                const uint32_t bn = rl / pn;
                u = rl - bn * pn + pn * jl;
                k = bn % m;
                sr = (bn / m) * pi + u;
                sk = k;
            } else if (D.mode == 2 && g.permute) {
                // destination: cyclic processor rl = rho m^h + rev(b), local jl = s q + t;
                // it came from member s of group b (paper numbering b p_h + s), index rho + t p_h
                const uint32_t mh = uint32_t(D.mh), q = uint32_t(D.q);
                const uint32_t rho = rl / mh;
                uint32_t bs = rl - rho * mh, b = 0;
                for (int h = 0; h < D.h; ++h) {
                    const uint32_t dq = bs / m;
                    b = b * m + (bs - dq * m);
                    bs = dq;
                }
                const uint32_t s = jl / q;
                const uint32_t t = jl - s * q;
                u = s;
                k = rho + t * pi;
                sr = b * pi + s;
                sk = k;
            } else if (D.mode != 0) {
                u = rl % pi;                       // the twiddle alone: the element stays
                k = jl;
            }
            if (D.mode != 0) {
                e += u * k * uint32_t(D.tstep);    // u < p_i, k < m: u k < n_i, so the term is below T
                e = e >= uint32_t(g.T) ? e - uint32_t(g.T) : e;
            }
            src_rank += sr * rmul;
            src_k += sk * kmul;
            rmul *= uint32_t(D.p);
            kmul *= m;
        }
        // a gather: plain load, so that the rest of the line may still be in cache
        // when the neighbouring source elements are read
        cx<T> v = conj_if(get<true>(&in[int64_t(src_rank) * M + src_k]), g.conj_in);
        if (g.twiddle) v = cmul(v, table[e]);
        v = conj_if(v, g.conj_out);
        if (g.scale != 1.0) v = {v.x * scale, v.y * scale};
        put<false>(&out[i], v);
    }
}

hipError_t launch_gput(Precision prec, const void *in, void *out, const GroupPutDesc &g, const void *table,
                       hipStream_t stream)
{
    const int64_t want = (g.N + 255) / 256;
    const uint32_t blocks = uint32_t(want < 65536 ? (want > 0 ? want : 1) : 65536);
    if (prec == Precision::F64)
        hipLaunchKernelGGL(k_gput<double>, dim3(blocks), dim3(256), 0, stream, static_cast<const cx<double> *>(in),
                           static_cast<cx<double> *>(out), g, static_cast<const cx<double> *>(table));
    else
        hipLaunchKernelGGL(k_gput<float>, dim3(blocks), dim3(256), 0, stream, static_cast<const cx<float> *>(in),
                           static_cast<cx<float> *>(out), g, static_cast<const cx<float> *>(table));
    return hipGetLastError();
}

}  // namespace fftu
