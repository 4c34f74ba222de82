// k_exchange device code (one group of local indices at a time), shared by the
// k_exchange kernels and the persistent batch kernel. See fftu_exchange.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fftu_device.hpp"
#include "fftu_internal.hpp"

namespace fftu {

// c[l] selected by a uniform dimension index (unrolled, so c stays in registers).
__device__ __forceinline__ uint32_t pick(const uint32_t (&c)[kMaxDims], int l)
{
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < kMaxDims; ++i)
        if (l == i) r = c[i];
    return r;
}

// DFT of size 2^LPD along each of the ND digits of an index space of 2^(ND LPD)
// entries (row-major, last digit fastest), entry e at v[e * STRIDE + u], u in [NU].
template <typename T, int ND, int LPD, int STRIDE, int NU>
__device__ __forceinline__ void dft_digits(cx<T> *v)
{
    constexpr int RD = 1 << LPD;
    constexpr int N = 1 << (ND * LPD);
#pragma unroll
    for (int dd = 0; dd < ND; ++dd) {
        const int ds = 1 << (LPD * (ND - 1 - dd));
#pragma unroll
        for (int base = 0; base < N; ++base) {
            if ((base / ds) % RD != 0) continue;
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                cx<T> x[RD];
#pragma unroll
                for (int r = 0; r < RD; ++r) x[r] = v[(base + r * ds) * STRIDE + u];
                Dft<T, RD>::run(x);
#pragma unroll
                for (int r = 0; r < RD; ++r) v[(base + r * ds) * STRIDE + u] = x[r];
            }
        }
    }
}

// Offset inside a destination block of an output whose digits (row-major over
// the given dimensions, last fastest) form index e: digit of dimension l goes to
// k'_l, which moves by q_l prod_{j>l} m_j, i.e. a shift of ex.oshift[l].
template <int ND, int LPD>
__device__ __forceinline__ int64_t digit_offset(const int32_t *dims, const ExchangeDesc &ex, int e)
{
    int64_t off = 0;
#pragma unroll
    for (int dd = 0; dd < ND; ++dd) {
        const int digit = (e >> (LPD * (ND - 1 - dd))) & ((1 << LPD) - 1);
        off += int64_t(digit) << ex.oshift[dims[dd]];
    }
    return off;
}

// Conjugation, scaling and the optional pointwise product of the outputs o[i],
// stored at V[idx(i)]. MULM 0: the product when ex.mul is set, element by
// element; 1: never; 2: always, with every multiplier loaded before the first
// store (loads and stores share one wait counter, so a load issued after a
// store waits for it); 3: no product, the output negated where idx(i) has an odd
// number of bits under ex.sign_mask.
template <typename T, bool CO, int MULM, int NOUT, typename IDX>
__device__ __forceinline__ void exchange_store(cx<T> *__restrict__ V, const ExchangeDesc &ex, cx<T> (&o)[NOUT],
                                               IDX idx, bool valid)
{
    const GridDesc &g = ex.g;
    const T scale = static_cast<T>(g.scale);
    const cx<T> *mul = static_cast<const cx<T> *>(ex.mul);
    cx<T> mv[MULM == 2 ? NOUT : 1];
    if constexpr (MULM == 2) {
#pragma unroll
        for (int i = 0; i < NOUT; ++i) mv[i] = valid ? mul[idx(i)] : cx<T>{T(0), T(0)};
    }
#pragma unroll
    for (int i = 0; i < NOUT; ++i) {
        cx<T> w = conj_if(o[i], g.conj_out);
        if (g.scale != 1.0) w = {w.x * scale, w.y * scale};
        if (valid) {
            if constexpr (MULM == 2) w = cmul(w, mv[i]);
            if (MULM == 0 && mul) w = cmul(w, mul[idx(i)]);
            if constexpr (MULM == 3) {
                if (__popcll(uint64_t(idx(i)) & ex.sign_mask) & 1) w = {-w.x, -w.y};
            }
            put<CO>(&V[idx(i)], w);
        }
    }
}

// KG x 64 local indices with NT threads: gather, twiddle, transform, swap,
// transform, scatter. Thread (grp, hw, lane) handles local index k, which must
// be the same for every hw of a (grp, lane). fetch(j, hw, k, valid) returns
// Z^(s')[k] for the source s' = (hw, j). With ex.mul set, every output is
// multiplied by the element of ex.mul at the same position before it is stored
// (a pointwise product in the output layout).
template <typename T, int NR, int LPR, int NH, int LPH, int NT, bool CO, int MULM, typename FETCH>
__device__ __forceinline__ void exchange_core(cx<T> *__restrict__ V, const ExchangeDesc &ex,
                                              const cx<T> *__restrict__ table, unsigned char *smem_raw,
                                              const int64_t k, int tid, FETCH fetch)
{
    constexpr int LOGR = NR * LPR, LOGH = NH * LPH;
    constexpr int R = 1 << LOGR;
    constexpr int H = 1 << LOGH;
    constexpr int U = LOGH > 0 ? R / H : R;   // register slots per thread after the LDS swap
    constexpr int KG = (NT / 64) / H;         // groups of 64 local indices per workgroup
    const GridDesc &g = ex.g;
    cx<T> *lds = reinterpret_cast<cx<T> *>(smem_raw);
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int hw = wv & (H - 1);   // this wave's source index in the wave dimensions
    const int grp = wv >> LOGH;
    const int logM = g.logmstride[0] + g.logm[0];
    const uint32_t emask = (1u << g.lognmax) - 1;
    {
        const bool valid = k < g.M;

        // k = r + t p per dimension; c_l = k_l 2^(lognmax - logn_l) is the twiddle step of s'_l.
        uint32_t c[kMaxDims];
        int64_t rank_r = 0, dst_t = 0;
#pragma unroll
        for (int l = 0; l < kMaxDims; ++l) {
            c[l] = 0;
            if (l < g.d) {
                const int64_t kl = (k >> g.logmstride[l]) & ((int64_t(1) << g.logm[l]) - 1);
                rank_r += (kl & ((int64_t(1) << g.logp[l]) - 1)) << g.logpstride[l];
                dst_t += (kl >> g.logp[l]) << g.logmstride[l];
                c[l] = uint32_t(kl) << (g.lognmax - g.logn[l]);
            }
        }
        // Twiddle exponent of source (hw, j): sum over digits of digit * c_dim.
        uint32_t e_hi = 0;
#pragma unroll
        for (int dd = 0; dd < NH; ++dd)
            e_hi += uint32_t((hw >> (LPH * (NH - 1 - dd))) & ((1 << LPH) - 1)) * pick(c, ex.hdim[dd]);
        uint32_t cr[NR > 0 ? NR : 1];
#pragma unroll
        for (int dd = 0; dd < NR; ++dd) cr[dd] = pick(c, ex.rdim[dd]);

        // Gather Z^(s')[k] for s' = (hw, j), j in [R], and twiddle.
        cx<T> v[R];
#pragma unroll
        for (int j = 0; j < R; ++j) v[j] = fetch(j, hw, k, valid);
#pragma unroll
        for (int j = 0; j < R; ++j) {
            uint32_t e = e_hi;
#pragma unroll
            for (int dd = 0; dd < NR; ++dd) e += uint32_t((j >> (LPR * (NR - 1 - dd))) & ((1 << LPR) - 1)) * cr[dd];
            v[j] = conj_if(v[j], g.conj_in);
            if (LOGH > 0 || j > 0) v[j] = cmul(v[j], table[e & emask]);
        }

        // DFTs over the register dimensions (natural order out).
        dft_digits<T, NR, LPR, 1, 1>(v);

        const int64_t obase = (rank_r << logM) + dst_t;
        if constexpr (LOGH == 0) {
            exchange_store<T, CO, MULM>(
                V, ex, v, [&](int j) { return obase + digit_offset<NR, LPR>(ex.rdim, ex, j); }, valid);
        } else {
            // Swap through LDS: register j of wave hw goes to the wave that owns slot j
            // (complex128 in two rounds of doubles, so the swap needs 8 bytes per value).
            cx<T> w[H * U];
            if constexpr (sizeof(T) == 8) {
                T *ld = reinterpret_cast<T *>(smem_raw);
                __syncthreads();
#pragma unroll
                for (int j = 0; j < R; ++j) ld[((hw * R + j) * KG + grp) * 64 + lane] = v[j].x;
                __syncthreads();
#pragma unroll
                for (int x = 0; x < H; ++x)
#pragma unroll
                    for (int u = 0; u < U; ++u) w[x * U + u].x = ld[((x * R + hw * U + u) * KG + grp) * 64 + lane];
                __syncthreads();
#pragma unroll
                for (int j = 0; j < R; ++j) ld[((hw * R + j) * KG + grp) * 64 + lane] = v[j].y;
                __syncthreads();
#pragma unroll
                for (int x = 0; x < H; ++x)
#pragma unroll
                    for (int u = 0; u < U; ++u) w[x * U + u].y = ld[((x * R + hw * U + u) * KG + grp) * 64 + lane];
            } else {
                __syncthreads();
#pragma unroll
                for (int j = 0; j < R; ++j) lds[((hw * R + j) * KG + grp) * 64 + lane] = v[j];
                __syncthreads();
#pragma unroll
                for (int x = 0; x < H; ++x)
#pragma unroll
                    for (int u = 0; u < U; ++u) w[x * U + u] = lds[((x * R + hw * U + u) * KG + grp) * 64 + lane];
            }

            // DFTs over the wave dimensions, for each of this thread's U register outputs.
            dft_digits<T, NH, LPH, U, U>(w);

            exchange_store<T, CO, MULM>(
                V, ex, w,
                [&](int i) {
                    return obase + digit_offset<NH, LPH>(ex.hdim, ex, i / U) +
                           digit_offset<NR, LPR>(ex.rdim, ex, hw * U + i % U);
                },
                valid);
        }
    }
}

// exchange_core over kExchangeThreads threads, gathering from the S0 output Z.
template <typename T, int NR, int LPR, int NH, int LPH, bool CO = false, int MULM = 0>
__device__ __forceinline__ void exchange_group(const cx<T> *__restrict__ Z, cx<T> *__restrict__ V,
                                               const ExchangeDesc &ex, const cx<T> *__restrict__ table,
                                               unsigned char *smem_raw, int64_t gb, int tid)
{
    const int logM = ex.g.logmstride[0] + ex.g.logm[0];
    constexpr int H = 1 << (NH * LPH);
    const int64_t k = ((gb + ((tid >> 6) / H)) << 6) + (tid & 63);   // group grp = wave / H, one index per lane
    exchange_core<T, NR, LPR, NH, LPH, kExchangeThreads, CO, MULM>(
        V, ex, table, smem_raw, k, tid, [&](int j, int hw, int64_t k, bool valid) {
            const int64_t s = (int64_t(hw) << (NR * LPR)) + j;
            return valid ? get<CO>(&Z[(s << logM) + k]) : cx<T>{T(0), T(0)};
        });
}

}  // namespace fftu
