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

// Source of destination element (processor r, local j) of one communication
// superstep, dimension by dimension, and the exponent of the level's twiddle of
// that source element over T (each term below T, the sum reduced below T).
// Shared by the kernels and the host, which derives the tiling of a power-of-two
// Put from it.
__host__ __device__ inline void gput_source(const GroupPutDesc &g, uint32_t r, uint32_t j, uint32_t &src_rank,
                                            uint32_t &src_k, uint32_t &e)
{
    uint32_t rmul = 1, kmul = 1;
    src_rank = src_k = e = 0;
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
}

template <typename T>
__global__ __launch_bounds__(256) void k_gput(const cx<T> *__restrict__ in, cx<T> *__restrict__ out,
                                              const GroupPutDesc g, const cx<T> *__restrict__ table)
{
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    const T scale = static_cast<T>(g.scale);
    const uint32_t M = uint32_t(g.M);
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < g.N; i += stride) {
        const uint32_t r = uint32_t(i / M);
        const uint32_t j = uint32_t(i - int64_t(r) * M);
        uint32_t src_rank, src_k, e;
        gput_source(g, r, j, src_rank, src_k, e);
        // a gather: plain load, so that the rest of the line may still be in cache
        // when the neighbouring source elements are read
        cx<T> v = conj_if(get<true>(&in[int64_t(src_rank) * M + src_k]), g.conj_in);
        if (g.twiddle) v = cmul(v, table[e]);
        v = conj_if(v, g.conj_out);
        if (g.scale != 1.0) v = {v.x * scale, v.y * scale};
        put<false>(&out[i], v);
    }
}

// With every side a power of two a Put is a permutation of the bits of the buffer
// index (processor bits, then local bits): mode 1 swaps a processor digit with the
// local index, mode 2 moves digits and reverses the base-m digits of the group.
// k_gputt moves it in tiles through LDS, both sides in runs: a tile is the 2^K
// elements that differ in a set X of destination bits holding the lowest A
// destination bits and the images of the lowest B source bits. Threads load in
// source order (runs of 2^B elements), store to LDS in destination order, and
// after a barrier store in destination order (runs of 2^A elements). The tiles
// enumerate the other bits (tile bit k: destination bit ydst[k], source bit
// ysrc[k]). The twiddle exponent of an element follows from its source
// coordinates: sum over dimensions of (source processor digit mod p_i) x
// (source local index) x T / n_i, reduced mod T (a power of two).
template <typename T, int EPT>
__global__ __launch_bounds__(256) void k_gputt(const cx<T> *__restrict__ in, cx<T> *__restrict__ out,
                                               const GroupPutDesc g, const GputTileDesc tl,
                                               const cx<T> *__restrict__ table)
{
    constexpr int NT = 256;
    extern __shared__ unsigned char smem_raw[];
    cx<T> *lds = reinterpret_cast<cx<T> *>(smem_raw);
    const int tid = threadIdx.x;
    const T scale = static_cast<T>(g.scale);
    const uint32_t M = uint32_t(g.M), tmask = uint32_t(g.T) - 1;
    const int logM = __builtin_ctz(M);
    // this thread's offsets inside a tile: load element t = tid + e NT (source order),
    // store element t (destination order)
    uint32_t soff[EPT], slot[EPT], doff[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const uint32_t t = uint32_t(tid + e * NT);
        uint32_t so = 0, sl = 0, dof = 0;
        for (int i = 0; i < tl.K; ++i) {
            const uint32_t bit = (t >> i) & 1u;
            so |= bit << tl.lsrc[i];
            sl |= bit << tl.dslot[i];
            dof |= bit << tl.xdst[i];
        }
        soff[e] = so;
        slot[e] = sl + (sl >> tl.pad_shift);
        doff[e] = dof;
    }
    for (int64_t tile = blockIdx.x; tile < tl.ntiles; tile += gridDim.x) {
        int64_t sbase = 0, dbase = 0;
        for (int k = 0; k < tl.ntb; ++k)
            if ((tile >> k) & 1) {
                sbase |= int64_t(1) << tl.ysrc[k];
                dbase |= int64_t(1) << tl.ydst[k];
            }
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int64_t si = sbase | soff[e];
            cx<T> v = conj_if(get(&in[si]), g.conj_in);
            // no branch around the table load (entry 0 = 1 exactly without a twiddle), so
            // that the loads of the EPT elements issue back to back
            uint32_t rank = uint32_t(si >> logM), loc = uint32_t(si) & (M - 1);
            uint32_t ex = 0;
#pragma unroll
            for (int l = kMaxDims - 1; l >= 0; --l) {
                if (l >= g.d) continue;
                const GroupPutDim &D = g.dim[l];
                const uint32_t sr = rank & uint32_t(D.p - 1), sk = loc & uint32_t(D.m - 1);
                rank >>= __builtin_ctz(uint32_t(D.p));
                loc >>= __builtin_ctz(uint32_t(D.m));
                if (D.mode != 0) ex += (sr & uint32_t(D.pi - 1)) * sk * uint32_t(D.tstep);
            }
            v = cmul(v, table[g.twiddle ? ex & tmask : 0u]);
            lds[slot[e]] = v;
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const uint32_t t = uint32_t(tid + e * NT);
            cx<T> w = conj_if(lds[t + (t >> tl.pad_shift)], g.conj_out);
            if (g.scale != 1.0) w = {w.x * scale, w.y * scale};
            put<false>(&out[dbase | doff[e]], w);
        }
        __syncthreads();
    }
}

namespace {

// In-register DFT along bits [POS, POS + R) of the group index (natural order).
template <typename T, int LOGG, int POS, int R>
__device__ __forceinline__ void dft_axis(cx<T> (&v)[1 << LOGG])
{
    if constexpr (POS + R <= LOGG) {
        constexpr int G = 1 << LOGG, L = 1 << R;
#pragma unroll
        for (int base = 0; base < G; ++base) {
            if ((base >> POS) & (L - 1)) continue;
            cx<T> x[L];
#pragma unroll
            for (int i = 0; i < L; ++i) x[i] = v[base + (i << POS)];
            Dft<T, L>::run(x);
#pragma unroll
            for (int i = 0; i < L; ++i) v[base + (i << POS)] = x[i];
        }
    }
}

template <typename T, int LOGG, int POS>
__device__ __forceinline__ void dft_axis_r(cx<T> (&v)[1 << LOGG], int r)
{
    switch (r) {
    case 1: dft_axis<T, LOGG, POS, 1>(v); break;
    case 2: dft_axis<T, LOGG, POS, 2>(v); break;
    case 3: dft_axis<T, LOGG, POS, 3>(v); break;
    case 4: dft_axis<T, LOGG, POS, 4>(v); break;
    default: break;
    }
}

template <typename T, int LOGG>
__device__ __forceinline__ void dft_axis_at(cx<T> (&v)[1 << LOGG], int pos, int r)
{
    switch (pos) {
    case 0: dft_axis_r<T, LOGG, 0>(v, r); break;
    case 1: dft_axis_r<T, LOGG, 1>(v, r); break;
    case 2: dft_axis_r<T, LOGG, 2>(v, r); break;
    case 3: dft_axis_r<T, LOGG, 3>(v, r); break;
    default: break;
    }
}

}  // namespace

// The last communication superstep of a plan whose sides are powers of two, with
// the length-p_h FFTs that follow it (Algorithm 2.2's Superstep 2 of every
// dimension whose level h this is) in the same pass. Every dimension is then in
// mode 2 (its last Put) or mode 0 (done). A thread takes the G = prod p_h
// elements that one set of those FFTs combines: source local index k (per
// dimension s_k = rho + t p_h) and the source group b (mode 2) or processor
// (mode 0), all members s of the groups. It gathers them (consecutive threads
// read consecutive k of one source processor), applies the level's twiddle
// omega^(s s_k), runs the length-p_h DFTs along each dimension's s in
// registers, and stores output s' of dimension l at local s' q + t of processor
// rho m^h + rev(b). The FFT output index replaces s in place, so the
// destination is the Put's destination of the same s.
template <typename T, int LOGG>
__global__ __launch_bounds__(256) void k_gplast(const cx<T> *__restrict__ in, cx<T> *__restrict__ out,
                                                const GroupPutDesc g, const cx<T> *__restrict__ table)
{
    constexpr int G = 1 << LOGG;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    const T scale = static_cast<T>(g.scale);
    const uint32_t M = uint32_t(g.M), T_ = uint32_t(g.T);
    const int logM = __builtin_ctz(M);
    const int d = g.d;
    // bit j of the group index: the source offset, the destination offset (both uniform)
    // and the dimension that owns it
    uint32_t srcw[LOGG > 0 ? LOGG : 1], dstw[LOGG > 0 ? LOGG : 1];
    int owner[LOGG > 0 ? LOGG : 1], shift[LOGG > 0 ? LOGG : 1];
    {
        uint32_t pstride = 1, mstride = 1;
        int pos = 0;
        for (int l = d - 1; l >= 0; --l) {
            const GroupPutDim &D = g.dim[l];
            if (D.mode == 2) {
                const int r = __builtin_ctz(uint32_t(D.pi));
#pragma unroll
                for (int j = 0; j < LOGG; ++j)
                    if (j >= pos && j < pos + r) {
                        srcw[j] = (pstride << (j - pos)) * M;
                        dstw[j] = (uint32_t(D.q) * mstride) << (j - pos);
                        owner[j] = l;
                        shift[j] = j - pos;
                    }
                pos += r;
            }
            pstride *= uint32_t(D.p);
            mstride *= uint32_t(D.m);
        }
    }
    const int64_t nthreads = g.N >> LOGG;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nthreads; i += stride) {
        const uint32_t ksrc = uint32_t(i) & (M - 1);
        uint32_t rp = uint32_t(i >> logM);
        uint32_t rem = ksrc;
        uint32_t srank = 0, drank = 0, dloc = 0, pstride = 1, mstride = 1;
        uint32_t a[kMaxDims];                       // s_k T / n_h mod T: the twiddle of member s is a s
#pragma unroll
        for (int l = kMaxDims - 1; l >= 0; --l) {   // unrolled: a[] stays in registers
            a[l] = 0;
            if (l >= d) continue;
            const GroupPutDim &D = g.dim[l];
            const int logm = __builtin_ctz(uint32_t(D.m));
            const uint32_t sk = rem & uint32_t(D.m - 1);
            rem >>= logm;
            if (D.mode == 2) {
                const int logpi = __builtin_ctz(uint32_t(D.pi));
                const int logb = __builtin_ctz(uint32_t(D.p)) - logpi;
                const uint32_t b = rp & ((1u << logb) - 1);
                rp >>= logb;
                uint32_t bs = b, rv = 0;
                for (int h = 0; h < D.h; ++h) {
                    rv = (rv << logm) | (bs & uint32_t(D.m - 1));
                    bs >>= logm;
                }
                const uint32_t rho = sk & uint32_t(D.pi - 1), t = sk >> logpi;
                srank += (b << logpi) * pstride;
                drank += ((rho << (D.h * logm)) | rv) * pstride;
                dloc += t * mstride;
                a[l] = uint32_t((uint64_t(sk) * uint64_t(D.tstep)) % T_);
            } else {
                const int logp = __builtin_ctz(uint32_t(D.p));
                const uint32_t r = rp & uint32_t(D.p - 1);
                rp >>= logp;
                srank += r * pstride;
                drank += r * pstride;
                dloc += sk * mstride;
            }
            pstride *= uint32_t(D.p);
            mstride *= uint32_t(D.m);
        }
        uint32_t ew[LOGG > 0 ? LOGG : 1];
#pragma unroll
        for (int j = 0; j < LOGG; ++j) {
            // a s < T for every member s < p_h, so each weight a 2^shift is below T
            uint32_t av = 0;
#pragma unroll
            for (int l = 0; l < kMaxDims; ++l)
                if (l == owner[j]) av = a[l];
            ew[j] = av << shift[j];
        }
        const int64_t sbase = int64_t(srank) * M + ksrc;
        const int64_t dbase = int64_t(drank) * M + dloc;
        cx<T> v[G];
#pragma unroll
        for (int gi = 0; gi < G; ++gi) {
            uint32_t off = 0;
#pragma unroll
            for (int j = 0; j < LOGG; ++j)
                if ((gi >> j) & 1) off += srcw[j];
            // a gather: plain load (the neighbouring elements serve other threads)
            v[gi] = conj_if(get<true>(&in[sbase + off]), g.conj_in);
        }
        if (g.twiddle) {
#pragma unroll
            for (int gi = 1; gi < G; ++gi) {
                uint32_t e = 0;
#pragma unroll
                for (int j = 0; j < LOGG; ++j)
                    if ((gi >> j) & 1) {
                        e += ew[j];
                        e = e >= T_ ? e - T_ : e;
                    }
                v[gi] = cmul(v[gi], table[e]);
            }
        }
        // the length-p_h DFTs, one dimension at a time
        {
            int pos = 0;
            for (int l = d - 1; l >= 0; --l) {
                const GroupPutDim &D = g.dim[l];
                if (D.mode != 2) continue;
                const int r = __builtin_ctz(uint32_t(D.pi));
                dft_axis_at<T, LOGG>(v, pos, r);
                pos += r;
            }
        }
#pragma unroll
        for (int gi = 0; gi < G; ++gi) {
            uint32_t off = 0;
#pragma unroll
            for (int j = 0; j < LOGG; ++j)
                if ((gi >> j) & 1) off += dstw[j];
            cx<T> w = conj_if(v[gi], g.conj_out);
            if (g.scale != 1.0) w = {w.x * scale, w.y * scale};
            put<false>(&out[dbase + off], w);
        }
    }
}

template <typename T>
hipError_t launch_gplast_t(const void *in, void *out, const GroupPutDesc &g, const void *table, int logg,
                           hipStream_t stream)
{
    const int64_t want = ((g.N >> logg) + 255) / 256;
    const uint32_t blocks = uint32_t(want < 65536 ? (want > 0 ? want : 1) : 65536);
    const cx<T> *a = static_cast<const cx<T> *>(in), *tab = static_cast<const cx<T> *>(table);
    cx<T> *b = static_cast<cx<T> *>(out);
    switch (logg) {
    case 1: hipLaunchKernelGGL((k_gplast<T, 1>), dim3(blocks), dim3(256), 0, stream, a, b, g, tab); break;
    case 2: hipLaunchKernelGGL((k_gplast<T, 2>), dim3(blocks), dim3(256), 0, stream, a, b, g, tab); break;
    case 3: hipLaunchKernelGGL((k_gplast<T, 3>), dim3(blocks), dim3(256), 0, stream, a, b, g, tab); break;
    case 4: hipLaunchKernelGGL((k_gplast<T, 4>), dim3(blocks), dim3(256), 0, stream, a, b, g, tab); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gplast(Precision prec, const void *in, void *out, const GroupPutDesc &g, const void *table,
                         hipStream_t stream)
{
    // every side a power of two, each dimension in mode 0 or 2, G = prod p_h in 2..16
    auto pow2 = [](int64_t v) { return v > 0 && (v & (v - 1)) == 0; };
    if (g.d < 1 || g.d > kMaxDims || g.N >= (int64_t(1) << 31) || !pow2(g.M) || g.T >= (int64_t(1) << 26) ||
        !g.permute)
        return hipErrorInvalidValue;
    int logg = 0;
    for (int l = 0; l < g.d; ++l) {
        const GroupPutDim &D = g.dim[l];
        if (!pow2(D.m) || !pow2(D.p)) return hipErrorInvalidValue;
        if (D.mode == 2) {
            if (!pow2(D.pi) || !pow2(D.q) || D.pi > D.p || int64_t(D.pi) * D.q != D.m) return hipErrorInvalidValue;
            logg += __builtin_ctz(uint32_t(D.pi));
        } else if (D.mode != 0) {
            return hipErrorInvalidValue;
        }
    }
    if (logg < 1 || logg > kGplastMaxLogG) return hipErrorInvalidValue;
    return prec == Precision::F64 ? launch_gplast_t<double>(in, out, g, table, logg, stream)
                                  : launch_gplast_t<float>(in, out, g, table, logg, stream);
}

// The tiling of a Put whose index map is a bit permutation (every side and T powers
// of two, N < 2^31); false otherwise (k_gput then gathers element by element).
bool gput_tiling(const GroupPutDesc &g, int esize, GputTileDesc &tl)
{
    auto pow2 = [](int64_t v) { return v > 0 && (v & (v - 1)) == 0; };
    if (!g.permute || g.d < 1 || g.d > kMaxDims || !pow2(g.N) || !pow2(g.M) || !pow2(g.T) ||
        g.N >= (int64_t(1) << 31))
        return false;
    for (int l = 0; l < g.d; ++l)
        if (!pow2(g.dim[l].m) || !pow2(g.dim[l].p) || (g.dim[l].mode != 0 && !pow2(g.dim[l].pi))) return false;
    const int logN = __builtin_ctzll(uint64_t(g.N)), logM = __builtin_ctzll(uint64_t(g.M));
    // sigma[j]: the source bit of destination bit j
    int sigma[31], pi_of[31];
    bool seen[31] = {};
    for (int j = 0; j < logN; ++j) {
        const uint32_t i = 1u << j;
        uint32_t sr, sk, e;
        gput_source(g, i >> logM, i & uint32_t(g.M - 1), sr, sk, e);
        const uint64_t src = (uint64_t(sr) << logM) | sk;
        if (!pow2(int64_t(src)) || src >= uint64_t(g.N)) return false;
        sigma[j] = __builtin_ctzll(src);
        if (seen[sigma[j]]) return false;
        seen[sigma[j]] = true;
    }
    {
        uint32_t sr, sk, e;
        gput_source(g, 0, 0, sr, sk, e);
        if (sr || sk) return false;
    }
    for (int j = 0; j < logN; ++j) pi_of[sigma[j]] = j;
    // tiles of 1024 elements: runs of 32 both ways (complex64 tiles of 4096, runs of 64,
    // measured a third slower at 512^3 over 32^3)
    (void)esize;
    const int K = logN < kGputTileLog ? logN : kGputTileLog;
    // X: the lowest A destination bits, the images of the lowest B source bits, then
    // more destination bits from the bottom until |X| = K
    bool inx[31] = {};
    int nx = 0;
    const int A = (K + 1) / 2, B = K - A;   // runs of 2^A destination and 2^B source elements
    for (int j = 0; j < A; ++j) inx[j] = true, ++nx;
    for (int i = 0; i < B; ++i)
        if (!inx[pi_of[i]]) inx[pi_of[i]] = true, ++nx;
    for (int j = 0; j < logN && nx < K; ++j)
        if (!inx[j]) inx[j] = true, ++nx;
    // store order: destination bits of X ascending; LDS slot bit = the rank in that order
    int slot_of[31];
    int ns = 0;
    for (int j = 0; j < logN; ++j)
        if (inx[j]) {
            tl.xdst[ns] = j;
            slot_of[j] = ns++;
        }
    // load order: source bits of X ascending
    int nl = 0;
    for (int i = 0; i < logN; ++i)
        if (inx[pi_of[i]]) {
            tl.lsrc[nl] = i;
            tl.dslot[nl] = slot_of[pi_of[i]];
            ++nl;
        }
    int ny = 0;
    for (int j = 0; j < logN; ++j)
        if (!inx[j]) {
            tl.ydst[ny] = j;
            tl.ysrc[ny] = sigma[j];
            ++ny;
        }
    tl.K = K;
    tl.ntb = ny;
    tl.ntiles = int64_t(1) << ny;
    tl.pad_shift = A > 0 ? A : 31;
    return nl == K && ns == K;
}

hipError_t launch_gput(Precision prec, const void *in, void *out, const GroupPutDesc &g, const void *table,
                       hipStream_t stream)
{
    GputTileDesc tl{};
    const int esize = prec == Precision::F64 ? 16 : 8;
    // tiles of 256 elements or more (smaller arrays take the gather)
    if (gput_tiling(g, esize, tl) && tl.K >= 8) {
        const uint32_t elems = 1u << tl.K;
        const size_t lds = size_t(elems + (elems >> tl.pad_shift)) * size_t(esize);
        const int64_t want = tl.ntiles;
        const uint32_t blocks = uint32_t(want < 65536 ? want : 65536);
        const int ept = int(elems / 256);
        if (prec == Precision::F64) {
            const cx<double> *a = static_cast<const cx<double> *>(in), *tab = static_cast<const cx<double> *>(table);
            cx<double> *b = static_cast<cx<double> *>(out);
            if (ept == 16) hipLaunchKernelGGL((k_gputt<double, 16>), dim3(blocks), dim3(256), lds, stream, a, b, g, tl, tab);
            else if (ept == 8) hipLaunchKernelGGL((k_gputt<double, 8>), dim3(blocks), dim3(256), lds, stream, a, b, g, tl, tab);
            else if (ept == 4) hipLaunchKernelGGL((k_gputt<double, 4>), dim3(blocks), dim3(256), lds, stream, a, b, g, tl, tab);
            else if (ept == 2) hipLaunchKernelGGL((k_gputt<double, 2>), dim3(blocks), dim3(256), lds, stream, a, b, g, tl, tab);
            else hipLaunchKernelGGL((k_gputt<double, 1>), dim3(blocks), dim3(256), lds, stream, a, b, g, tl, tab);
            return hipGetLastError();
        } else {
            const cx<float> *a = static_cast<const cx<float> *>(in), *tab = static_cast<const cx<float> *>(table);
            cx<float> *b = static_cast<cx<float> *>(out);
            if (ept == 16) hipLaunchKernelGGL((k_gputt<float, 16>), dim3(blocks), dim3(256), lds, stream, a, b, g, tl, tab);
            else if (ept == 8) hipLaunchKernelGGL((k_gputt<float, 8>), dim3(blocks), dim3(256), lds, stream, a, b, g, tl, tab);
            else if (ept == 4) hipLaunchKernelGGL((k_gputt<float, 4>), dim3(blocks), dim3(256), lds, stream, a, b, g, tl, tab);
            else if (ept == 2) hipLaunchKernelGGL((k_gputt<float, 2>), dim3(blocks), dim3(256), lds, stream, a, b, g, tl, tab);
            else hipLaunchKernelGGL((k_gputt<float, 1>), dim3(blocks), dim3(256), lds, stream, a, b, g, tl, tab);
            return hipGetLastError();
        }
    }
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
