// Mixed-radix path of Algorithm 2.3 (arXiv 2203.11795) for sides whose prime
// factors are 2, 3, 5 and 7: the method itself only needs p_l^2 | n_l. (The
// paper's own code leaves the local FFTs to FFTW, which handles any size.)
//
//   k_mline      a pass of 1-D FFTs of length L (Superstep 0 along one local
//                dimension, or Superstep 2 along one grid dimension). W
//                consecutive lines of the (A, B) lines are loaded into LDS, transformed by mixed-radix Stockham
//                stages (radix 8, 4, 2, 7, 5, 3; stage s with radix R after
//                Ns points reads j + r L/R, twiddles by omega_{Ns R}^{r (j mod Ns)}
//                and writes (j div Ns) Ns R + j mod Ns + r Ns), ping-ponging
//                between two LDS buffers, and stored. Roots come from an LDS
//                copy of omega_L taken from the plan's FP64-generated table of
//                omega_T, T = lcm(n_l).
//   k_mtwiddle   Superstep 0's twiddle Z^(s)[k] = prod_l omega_{n_l}^{k_l s_l} Y^(s)[k],
//                the exponent reduced exactly in integers (one table entry).
//   k_mpermute   Superstep 1: W^(r)[s q + t] = Z^(s)[r + t p], per output element,
//                optionally with the twiddle of the source element applied on
//                the way (the whole transform runs twiddle and Put as one pass).
//
// The index arithmetic uses 32-bit divisions by runtime sizes, so this path
// takes N < 2^31. Loops that hold barriers run on wave-uniform values.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fftu_device.hpp"
#include "fftu_internal.hpp"

namespace fftu {

namespace {

// Roots omega_R^m, m in [R], from a table of omega_L (stride L / R): loaded once
// by a caller that runs many DFTs of size R (only the odd radices use them).
template <typename T, int R>
__device__ __forceinline__ void load_roots(cx<T> (&w)[R], const cx<T> *tw, int LperR)
{
    if constexpr (R == 3 || R == 5 || R == 7) {
#pragma unroll
        for (int m = 0; m < R; ++m) w[m] = tw[m * LperR];
    }
}

// DFT of size R on registers x[0..R-1], natural order: radix 2, 4, 8 with constant
// roots; 3, 5, 7 from omega_R^m = w[m * ws] (a load_roots array with ws = 1, or a
// table of omega_L with ws = L / R). For odd R the inputs pair as a_r = x_r +
// x_{R-r}, b_r = x_r - x_{R-r}, since omega^{(R-r) c} is the conjugate of
// omega^{r c} = C + iS: then y_c = x_0 + sum_r (C a_r + i S b_r), and y_{R-c}
// takes the same sums with the sign of the i S b_r part flipped.
template <typename T, int R>
__device__ __forceinline__ void dft_small(cx<T> (&x)[8], const cx<T> *w, int ws)
{
    if constexpr (R == 2 || R == 4 || R == 8) {
        Dft<T, R>::run(x);
    } else {
        constexpr int H = (R - 1) / 2;
        cx<T> a[H + 1], b[H + 1];
        cx<T> y0 = x[0];
#pragma unroll
        for (int r = 1; r <= H; ++r) {
            a[r] = x[r] + x[R - r];
            b[r] = x[r] - x[R - r];
            y0 = y0 + a[r];
        }
        cx<T> y[R];
        y[0] = y0;
#pragma unroll
        for (int c = 1; c <= H; ++c) {
            cx<T> A = x[0];
            T bx = T(0), by = T(0);
#pragma unroll
            for (int r = 1; r <= H; ++r) {
                const cx<T> wr = w[((r * c) % R) * ws];
                A = {A.x + wr.x * a[r].x, A.y + wr.x * a[r].y};
                bx += wr.y * b[r].x;
                by += wr.y * b[r].y;
            }
            y[c] = {A.x - by, A.y + bx};        // A + i (bx + i by)
            y[R - c] = {A.x + by, A.y - bx};
        }
#pragma unroll
        for (int c = 0; c < R; ++c) x[c] = y[c];
    }
}

// n / d for n < 2^22 and a wave-uniform d with inv = 1 / d: one float estimate,
// corrected by one step either way.
__device__ __forceinline__ int div_small(int n, int d, float inv)
{
    int q = int(float(n) * inv);
    const int r = n - q * d;
    q += r >= d ? 1 : 0;
    q -= r < 0 ? 1 : 0;
    return q;
}

// One Stockham stage of radix R over `lines` lines of length L (src -> dst in LDS;
// line w starts at w * pitch).
template <typename T, int R>
__device__ __forceinline__ void mixed_stage(const cx<T> *src, cx<T> *dst, const cx<T> *tw, int L, int pitch, int Ns,
                                            int lines, int tid, int nt)
{
    const int LR = L / R;
    const int span = L / (Ns * R);          // omega_{Ns R} = omega_L^span
    const int nb = lines * LR;
    const float inv_lr = 1.0f / float(LR), inv_ns = 1.0f / float(Ns);
    cx<T> w[R];
    load_roots<T, R>(w, tw, LR);
    for (int bi = tid; bi < nb; bi += nt) {
        const int wl = div_small(bi, LR, inv_lr);
        const int j = bi - wl * LR;
        const int jd = div_small(j, Ns, inv_ns);
        const int k = j - jd * Ns;
        const cx<T> *s = src + wl * pitch + j;
        cx<T> x[8];
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = s[r * LR];
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) x[r] = cmul(x[r], tw[r * k * span]);
        }
        dft_small<T, R>(x, w, 1);
        cx<T> *o = dst + wl * pitch + jd * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) o[r * Ns] = x[r];
    }
}

}  // namespace

template <typename T>
__global__ __launch_bounds__(kMixedThreads) void k_mline(const cx<T> *in, cx<T> *out, const MixedPassDesc pd,
                                                         const cx<T> *__restrict__ table)
{
    extern __shared__ unsigned char smem_raw[];
    __shared__ int64_t lbase[kMixedMaxW];   // strided tiles: global offset of each line's first element
    const int L = pd.L, W = pd.W;
    const int pitch = int(pd.pitch);   // strided tiles: odd, so consecutive lines fall on different LDS banks
    cx<T> *tw = reinterpret_cast<cx<T> *>(smem_raw);
    cx<T> *buf0 = tw + L;
    cx<T> *buf1 = buf0 + W * pitch;
    const int tid = threadIdx.x;
    // launch sizes in scalar registers: the tile loop holds barriers
    const int nt = __builtin_amdgcn_readfirstlane(int(blockDim.x));
    const int64_t nblocks = __builtin_amdgcn_readfirstlane(int(gridDim.x));
    for (int j = tid; j < L; j += nt) tw[j] = table[int64_t(j) * pd.tstep];
    const T scale = static_cast<T>(pd.scale);
    const uint32_t B = uint32_t(pd.B);
    for (int64_t t = blockIdx.x; t < pd.tiles; t += nblocks) {
        // the tile holds lines u0 .. u0 + lines - 1 of the A B lines (line u = a B + b);
        // `lines` is wave-uniform
        const uint32_t u0 = uint32_t(t) << pd.logW;
        const uint32_t total = uint32_t(pd.A) * B;
        const int lines = int(total - u0 < uint32_t(W) ? total - u0 : uint32_t(W));
        __syncthreads();   // twiddle copy done / previous tile's LDS reads done
        if (B != 1) {
            // line u = a B + b starts at (a L) B + b: one division per line, not per element
            for (int w = tid; w < lines; w += nt) {
                const uint32_t u = u0 + uint32_t(w);
                const uint32_t a = u / B;
                lbase[w] = int64_t(a) * L * B + (u - a * B);
            }
            __syncthreads();
        }
        const int n = lines * L;
        const float inv_lines = 1.0f / float(lines);
        // element e of the tile: LDS offset (line w, position x) and global offset. With
        // B = 1 the tile's lines are contiguous in memory and e runs along them (the LDS
        // pitch is L there); otherwise lanes run over consecutive lines (consecutive b:
        // runs of up to min(W, B) elements). e < 2^22, so the quotient comes from one
        // float estimate and a correction.
        auto where = [&](int e, int &off) -> int64_t {
            if (B == 1) {
                off = e;
                return int64_t(u0) * L + e;
            }
            const int x = div_small(e, lines, inv_lines);
            const int w = e - x * lines;
            off = w * pitch + x;
            return lbase[w] + int64_t(x) * B;
        };
        // kMixedBatch loads per thread in flight, then their LDS stores
        for (int e0 = tid; e0 < n; e0 += kMixedBatch * nt) {
            cx<T> r[kMixedBatch];
            int off[kMixedBatch];
#pragma unroll
            for (int i = 0; i < kMixedBatch; ++i) {
                const int e = e0 + i * nt;
                if (e < n) r[i] = get(&in[where(e, off[i])]);
            }
#pragma unroll
            for (int i = 0; i < kMixedBatch; ++i)
                if (e0 + i * nt < n) buf0[off[i]] = conj_if(r[i], pd.conj_in);
        }
        __syncthreads();
        cx<T> *src = buf0, *dst = buf1;
        int Ns = 1;
        for (int s = 0; s < pd.nstages; ++s) {
            switch (pd.radix[s]) {
            case 2: mixed_stage<T, 2>(src, dst, tw, L, pitch, Ns, lines, tid, nt); break;
            case 3: mixed_stage<T, 3>(src, dst, tw, L, pitch, Ns, lines, tid, nt); break;
            case 4: mixed_stage<T, 4>(src, dst, tw, L, pitch, Ns, lines, tid, nt); break;
            case 5: mixed_stage<T, 5>(src, dst, tw, L, pitch, Ns, lines, tid, nt); break;
            case 7: mixed_stage<T, 7>(src, dst, tw, L, pitch, Ns, lines, tid, nt); break;
            case 8: mixed_stage<T, 8>(src, dst, tw, L, pitch, Ns, lines, tid, nt); break;
            default: break;
            }
            __syncthreads();
            cx<T> *tmp = src;
            src = dst;
            dst = tmp;
            Ns *= pd.radix[s];
        }
        for (int e0 = tid; e0 < n; e0 += kMixedBatch * nt) {
#pragma unroll
            for (int i = 0; i < kMixedBatch; ++i) {
                const int e = e0 + i * nt;
                if (e < n) {
                    int off;
                    const int64_t addr = where(e, off);
                    cx<T> v = conj_if(src[off], pd.conj_out);
                    if (pd.scale != 1.0) v = {v.x * scale, v.y * scale};
                    put<false>(&out[addr], v);
                }
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_mtwiddle(const cx<T> *in, cx<T> *out, const MixedGridDesc g,
                                                  const cx<T> *__restrict__ table)
{
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < g.N; i += stride) {
        uint32_t rank = uint32_t(i / g.M);
        uint32_t k = uint32_t(i - int64_t(rank) * g.M);
        int64_t e = 0;
        for (int l = g.d - 1; l >= 0; --l) {
            const uint32_t sl = rank % uint32_t(g.p[l]);
            rank /= uint32_t(g.p[l]);
            const uint32_t kl = k % uint32_t(g.m[l]);
            k /= uint32_t(g.m[l]);
            e += int64_t(kl) * sl * g.tstep[l];      // k_l s_l < n_l, times T / n_l: below T
        }
        cx<T> v = conj_if(get(&in[i]), g.conj_in);
        v = cmul(v, table[e % g.T]);
        put<false>(&out[i], conj_if(v, g.conj_out));
    }
}

// With g.twiddle set, the element is also multiplied by Superstep 0's twiddle of
// its source position, omega^(sum_l k_l s_l) (the twiddle and the Put in one pass).
template <typename T>
__global__ __launch_bounds__(256) void k_mpermute(const cx<T> *in, cx<T> *out, const MixedGridDesc g,
                                                  const cx<T> *__restrict__ table)
{
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    const T scale = static_cast<T>(g.scale);
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < g.N; i += stride) {
        uint32_t r = uint32_t(i / g.M);
        uint32_t j = uint32_t(i - int64_t(r) * g.M);
        int64_t src_rank = 0, src_k = 0, rmul = 1, kmul = 1, e = 0;
        for (int l = g.d - 1; l >= 0; --l) {
            const uint32_t jl = j % uint32_t(g.m[l]);
            j /= uint32_t(g.m[l]);
            const uint32_t rl = r % uint32_t(g.p[l]);
            r /= uint32_t(g.p[l]);
            const uint32_t sl = jl / uint32_t(g.q[l]);          // j_l = s_l q_l + t_l
            const uint32_t tl = jl - sl * uint32_t(g.q[l]);
            const int64_t kl = int64_t(rl) + int64_t(tl) * g.p[l];  // k_l = r_l + t_l p_l
            src_rank += int64_t(sl) * rmul;
            src_k += kl * kmul;
            e += kl * sl * g.tstep[l];
            rmul *= g.p[l];
            kmul *= g.m[l];
        }
        cx<T> v = conj_if(get(&in[src_rank * g.M + src_k]), g.conj_in);
        if (g.twiddle) v = cmul(v, table[e % g.T]);
        v = conj_if(v, g.conj_out);
        if (g.scale != 1.0) v = {v.x * scale, v.y * scale};
        put<false>(&out[i], v);
    }
}

// Superstep 0's twiddle, Superstep 1 and Superstep 2 in one pass (the mixed-radix
// counterpart of k_exchange): for a local index k = r + t p (per dimension) the
// values Z^(s)[k] of all P sources are the inputs of one F_{p_1} x ... x F_{p_d}
// whose output k' lands in V^(r)[t + k' q] (Theorem 2.1). A workgroup takes 64
// consecutive k (one per lane) of every block: each wave gathers a share of the
// sources (one load instruction reads 64 consecutive elements of one block),
// twiddles by omega_T^e, e = sum_l s_l k_l T / n_l (each term below T, so the sum
// is reduced exactly with one quotient estimate), stores to LDS as [s][lane], runs
// the length-p_l DFTs along each grid digit of s in LDS, and scatters. The grid
// sides must be 1, 2, 3, 4, 5, 7 or 8 (one radix stage each), P <= kMexMaxP.
// TL: the twiddles come from an LDS copy of the table (when it fits beside the tile).
template <typename T, bool TL>
__global__ __launch_bounds__(kMexThreads) void k_mexchange(const cx<T> *__restrict__ in, cx<T> *__restrict__ out,
                                                           const MixedGridDesc g, const cx<T> *__restrict__ table)
{
    extern __shared__ unsigned char smem_raw[];
    constexpr int NW = kMexThreads / 64;
    const int P = int(g.P);
    cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);                     // [P][64]
    uint32_t *sdig = reinterpret_cast<uint32_t *>(buf + P * 64);         // digits of s, 4 bits each
    uint32_t *soff = sdig + P;                                          // output offset of k' = s
    cx<T> *tlds = reinterpret_cast<cx<T> *>(soff + P);                  // omega_T (TL)
    if constexpr (TL)
        for (int e = threadIdx.x; e < int(g.T); e += kMexThreads) tlds[e] = table[e];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int d = g.d;
    const uint32_t M = uint32_t(g.M);
    const uint32_t tn = uint32_t(g.T);   // table size T
    const float inv_tn = 1.0f / float(tn);
    const T scale = static_cast<T>(g.scale);
    const cx<T> *mul = static_cast<const cx<T> *>(g.mul);
    // per source s: its digits (row-major over p) and the offset sum_l s_l q_l mstride_l
    // of output k' = s inside a destination block
    for (int s = tid; s < P; s += kMexThreads) {
        uint32_t dig = 0, off = 0, mstride = 1;
        int rs = s;
        for (int l = d - 1; l >= 0; --l) {
            const int sl = rs % g.p[l];
            rs /= g.p[l];
            dig |= uint32_t(sl) << (4 * l);
            off += uint32_t(sl) * uint32_t(g.q[l]) * mstride;
            mstride *= uint32_t(g.m[l]);
        }
        sdig[s] = dig;
        soff[s] = off;
    }
    const int64_t ngroups = (int64_t(M) + 63) >> 6;
    const int64_t nblocks = __builtin_amdgcn_readfirstlane(int(gridDim.x));   // uniform loop (barriers inside)
    for (int64_t grp = blockIdx.x; grp < ngroups; grp += nblocks) {
        const uint32_t k = uint32_t(grp << 6) + uint32_t(lane);
        const bool valid = k < M;
        // digits k_l of k (row-major over m), c_l = k_l T / n_l < T / p_l, and the
        // destination of output k' = 0: block rank(r), offset sum_l t_l mstride_l
        uint32_t c[kMaxDims];
        uint32_t rank = 0, obase = 0;
        {
            uint32_t rem = valid ? k : 0, mstride = 1, pstride = 1;
#pragma unroll
            for (int l = kMaxDims - 1; l >= 0; --l) {
                c[l] = 0;
                if (l < d) {
                    const uint32_t ml = uint32_t(g.m[l]), pl = uint32_t(g.p[l]);
                    const uint32_t kl = rem % ml;
                    rem /= ml;
                    c[l] = kl * uint32_t(g.tstep[l]);
                    const uint32_t rl = kl % pl, tl = kl / pl;
                    rank += rl * pstride;
                    obase += tl * mstride;
                    mstride *= ml;
                    pstride *= pl;
                }
            }
        }
        const int64_t dbase = int64_t(rank) * M + obase;
        __syncthreads();   // the previous group is out of LDS (and the digit tables are in)
        // gather and twiddle: wave wv takes sources wv + i NW, all its loads in flight
        for (int s0 = wv; s0 < P; s0 += kMexBatch * NW) {
            cx<T> v[kMexBatch];
#pragma unroll
            for (int i = 0; i < kMexBatch; ++i) {
                const int s = s0 + i * NW;
                v[i] = (valid && s < P) ? get(&in[int64_t(s) * M + k]) : cx<T>{T(0), T(0)};
            }
#pragma unroll
            for (int i = 0; i < kMexBatch; ++i) {
                const int s = s0 + i * NW;
                if (s < P) {
                    const uint32_t dig = sdig[s];
                    uint32_t e = 0;
#pragma unroll
                    for (int l = 0; l < kMaxDims; ++l)
                        if (l < d) e += ((dig >> (4 * l)) & 15u) * c[l];
                    // e < d T: one quotient estimate and a correction each way
                    int32_t r = int32_t(e - uint32_t(float(e) * inv_tn) * tn);
                    r += r < 0 ? int32_t(tn) : 0;
                    r -= r >= int32_t(tn) ? int32_t(tn) : 0;
                    cx<T> x = conj_if(v[i], g.conj_in);
                    if (g.twiddle) x = cmul(x, TL ? tlds[r] : table[r]);
                    buf[s * 64 + lane] = x;
                }
            }
        }
        __syncthreads();
        // Superstep 2: the DFT of length p_l along digit l of s (stride pstride_l), in place
        int pstride = 1;
        for (int l = d - 1; l >= 0; --l) {
            const int pl = g.p[l];
            if (pl > 1) {
                const int nlines = P / pl;
                const int LperR = int(tn) / pl;
                for (int ln = wv; ln < nlines; ln += NW) {
                    const int sb = (ln / pstride) * pstride * pl + ln % pstride;
                    cx<T> x[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        if (i < pl) x[i] = buf[(sb + i * pstride) * 64 + lane];
                    switch (pl) {
                    case 2: dft_small<T, 2>(x, table, LperR); break;
                    case 3: dft_small<T, 3>(x, table, LperR); break;
                    case 4: dft_small<T, 4>(x, table, LperR); break;
                    case 5: dft_small<T, 5>(x, table, LperR); break;
                    case 7: dft_small<T, 7>(x, table, LperR); break;
                    default: dft_small<T, 8>(x, table, LperR); break;
                    }
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        if (i < pl) buf[(sb + i * pstride) * 64 + lane] = x[i];
                }
                __syncthreads();
            }
            pstride *= pl;
        }
        // scatter: output k' (the digits of s after the DFTs) to dbase + soff[k']
        if (valid) {
            for (int s = wv; s < P; s += NW) {
                const int64_t idx = dbase + soff[s];
                cx<T> w = conj_if(buf[s * 64 + lane], g.conj_out);
                if (g.scale != 1.0) w = {w.x * scale, w.y * scale};
                if (mul) w = cmul(w, mul[idx]);
                put<false>(&out[idx], w);
            }
        }
    }
}

namespace {

uint32_t grid_for(int64_t count)
{
    const int64_t want = (count + 255) / 256;
    return uint32_t(want < (int64_t(1) << 18) ? (want > 0 ? want : 1) : (int64_t(1) << 18));
}

}  // namespace

hipError_t launch_mline(Precision prec, const void *in, void *out, const MixedPassDesc &pd, const void *table,
                        hipStream_t stream)
{
    const uint32_t blocks = uint32_t(pd.tiles < (int64_t(1) << 20) ? pd.tiles : (int64_t(1) << 20));
    if (prec == Precision::F64)
        hipLaunchKernelGGL(k_mline<double>, dim3(blocks), dim3(kMixedThreads), pd.lds_bytes, stream,
                           static_cast<const cx<double> *>(in), static_cast<cx<double> *>(out), pd,
                           static_cast<const cx<double> *>(table));
    else
        hipLaunchKernelGGL(k_mline<float>, dim3(blocks), dim3(kMixedThreads), pd.lds_bytes, stream,
                           static_cast<const cx<float> *>(in), static_cast<cx<float> *>(out), pd,
                           static_cast<const cx<float> *>(table));
    return hipGetLastError();
}

hipError_t launch_mtwiddle(Precision prec, const void *in, void *out, const MixedGridDesc &g, const void *table,
                           hipStream_t stream)
{
    if (prec == Precision::F64)
        hipLaunchKernelGGL(k_mtwiddle<double>, dim3(grid_for(g.N)), dim3(256), 0, stream,
                           static_cast<const cx<double> *>(in), static_cast<cx<double> *>(out), g,
                           static_cast<const cx<double> *>(table));
    else
        hipLaunchKernelGGL(k_mtwiddle<float>, dim3(grid_for(g.N)), dim3(256), 0, stream,
                           static_cast<const cx<float> *>(in), static_cast<cx<float> *>(out), g,
                           static_cast<const cx<float> *>(table));
    return hipGetLastError();
}

hipError_t launch_mpermute(Precision prec, const void *in, void *out, const MixedGridDesc &g, const void *table,
                           hipStream_t stream)
{
    if (prec == Precision::F64)
        hipLaunchKernelGGL(k_mpermute<double>, dim3(grid_for(g.N)), dim3(256), 0, stream,
                           static_cast<const cx<double> *>(in), static_cast<cx<double> *>(out), g,
                           static_cast<const cx<double> *>(table));
    else
        hipLaunchKernelGGL(k_mpermute<float>, dim3(grid_for(g.N)), dim3(256), 0, stream,
                           static_cast<const cx<float> *>(in), static_cast<cx<float> *>(out), g,
                           static_cast<const cx<float> *>(table));
    return hipGetLastError();
}

hipError_t launch_mexchange(Precision prec, const void *in, void *out, const MixedGridDesc &g, const void *table,
                            hipStream_t stream)
{
    if (g.P < 1 || g.P > kMexMaxP || g.T > (int64_t(1) << 24) || g.N >= (int64_t(1) << 31) || g.d > 8)
        return hipErrorInvalidValue;
    for (int l = 0; l < g.d; ++l)
        if (!mexchange_radix_ok(g.p[l])) return hipErrorInvalidValue;
    const int64_t groups = (g.M + 63) >> 6;
    const uint32_t blocks = uint32_t(groups < (int64_t(1) << 20) ? groups : (int64_t(1) << 20));
    const size_t esize = prec == Precision::F64 ? 16 : 8;
    const size_t lds = size_t(g.P) * (64 * esize + 8);
    // the table in LDS when two workgroups per CU still fit (measured 7% faster at 480^3)
    const bool tl = mexchange_table_in_lds(g.P, g.T, int(esize));
    const size_t bytes = tl ? lds + size_t(g.T) * esize : lds;
    if (prec == Precision::F64) {
        const cx<double> *a = static_cast<const cx<double> *>(in), *tab = static_cast<const cx<double> *>(table);
        cx<double> *b = static_cast<cx<double> *>(out);
        if (tl)
            hipLaunchKernelGGL((k_mexchange<double, true>), dim3(blocks), dim3(kMexThreads), bytes, stream, a, b, g, tab);
        else
            hipLaunchKernelGGL((k_mexchange<double, false>), dim3(blocks), dim3(kMexThreads), bytes, stream, a, b, g, tab);
    } else {
        const cx<float> *a = static_cast<const cx<float> *>(in), *tab = static_cast<const cx<float> *>(table);
        cx<float> *b = static_cast<cx<float> *>(out);
        if (tl)
            hipLaunchKernelGGL((k_mexchange<float, true>), dim3(blocks), dim3(kMexThreads), bytes, stream, a, b, g, tab);
        else
            hipLaunchKernelGGL((k_mexchange<float, false>), dim3(blocks), dim3(kMexThreads), bytes, stream, a, b, g, tab);
    }
    return hipGetLastError();
}

}  // namespace fftu
