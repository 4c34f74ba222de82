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

#include <atomic>
#include <cstdint>

#include "fftu_device.hpp"
#include "fftu_exchange.hpp"
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

// Elements of a tile per thread (the tile holds at most kMixedThreads times as many).
template <typename T>
constexpr int mline_pre() { return sizeof(T) == 8 ? kMixedPreF64 : kMixedPreF32; }

// The grid is persistent (about as many workgroups as fit on the device at once):
// a workgroup loads its next tile into registers while it transforms the current
// one, so each CU keeps loads in flight through the LDS stages as well. Its
// barriers order LDS only, so that they do not wait for those loads.
template <typename T>
__global__ __launch_bounds__(kMixedThreads) void k_mline(const cx<T> *__restrict__ in, cx<T> *__restrict__ out,
                                                         const MixedPassDesc pd, const cx<T> *__restrict__ table)
{
    constexpr int PRE = mline_pre<T>();
    extern __shared__ unsigned char smem_raw[];
    __shared__ uint32_t lbase[2][kMixedMaxW];   // strided tiles: offset of each line's first element (two tiles)
    const int L = pd.L, W = pd.W;
    const int pitch = int(pd.pitch);   // strided tiles: odd, so consecutive lines fall on different LDS banks
    cx<T> *tw = reinterpret_cast<cx<T> *>(smem_raw);
    cx<T> *buf0 = tw + L;
    cx<T> *buf1 = buf0 + W * pitch;
    const int tid = threadIdx.x;
    // launch sizes in scalar registers: the tile loop holds barriers
    const int nt = __builtin_amdgcn_readfirstlane(int(blockDim.x));
    const uint32_t nblocks = __builtin_amdgcn_readfirstlane(int(gridDim.x));
    const uint32_t B = uint32_t(pd.B);
    const uint32_t total = uint32_t(pd.A) * B;    // lines
    const uint32_t tiles = uint32_t(pd.tiles);
    const T scale = static_cast<T>(pd.scale);
    auto tile_lines = [&](uint32_t t) {
        const uint32_t u0 = t << pd.logW;
        return int(total - u0 < uint32_t(W) ? total - u0 : uint32_t(W));
    };
    // line u = a B + b starts at (a L) B + b: one division per line, not per element
    auto set_lbase = [&](uint32_t t, int slot) {
        const uint32_t u0 = t << pd.logW;
        const int lines = tile_lines(t);
        for (int w = tid; w < lines; w += nt) {
            const uint32_t u = u0 + uint32_t(w);
            const uint32_t a = u / B;
            lbase[slot][w] = a * uint32_t(L) * B + (u - a * B);
        }
    };
    // element e of tile t: LDS offset (line w, position x) and global offset. With B = 1
    // the tile's lines are contiguous in memory and e runs along them (the LDS pitch is
    // L there); otherwise lanes run over consecutive lines (consecutive b: runs of up
    // to min(W, B) elements). e < 2^22, so the quotient comes from one float estimate
    // and a correction.
    auto where = [&](uint32_t t, int lines, int slot, int e, int &off) -> uint32_t {
        if (B == 1) {
            off = e;
            return (t << pd.logW) * uint32_t(L) + uint32_t(e);
        }
        const int x = div_small(e, lines, 1.0f / float(lines));
        const int w = e - x * lines;
        off = w * pitch + x;
        return lbase[slot][w] + uint32_t(x) * B;
    };
    // branch-free (elements past the tile reload element 0), so that the loads issue
    // back to back and are waited for only where the values are used
    auto prefetch = [&](cx<T> (&r)[PRE], uint32_t t, int slot) {
        const int lines = tile_lines(t);
        const int n = lines * L;
#pragma unroll
        for (int i = 0; i < PRE; ++i) {
            const int e = tid + i * nt;
            int off;
            r[i] = get(&in[where(t, lines, slot, e < n ? e : 0, off)]);
        }
    };

    for (int j = tid; j < L; j += nt) tw[j] = table[int64_t(j) * pd.tstep];
    cx<T> pre[PRE];
    int slot = 0;
    if (blockIdx.x < tiles) {
        if (B != 1) {
            set_lbase(blockIdx.x, 0);
            lds_barrier();
        }
        prefetch(pre, blockIdx.x, 0);
    }
    for (uint32_t t = blockIdx.x; t < tiles; t += nblocks) {
        const int lines = tile_lines(t);
        const int n = lines * L;
        // the next tile (the last one reloads itself: the prefetch takes no branch, so
        // its loads are waited for only where the values are used)
        const uint32_t tn = t + nblocks < tiles ? t + nblocks : t;
        lds_barrier();   // twiddle copy done / previous tile's LDS reads done
#pragma unroll
        for (int i = 0; i < PRE; ++i) {
            const int e = tid + i * nt;
            if (e < n) {
                int off;
                where(t, lines, slot, e, off);
                buf0[off] = conj_if(pre[i], pd.conj_in);
            }
        }
        if (B != 1) set_lbase(tn, slot ^ 1);
        lds_barrier();
        prefetch(pre, tn, slot ^ 1);   // in flight through the stages below
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
            lds_barrier();
            cx<T> *tmp = src;
            src = dst;
            dst = tmp;
            Ns *= pd.radix[s];
        }
#pragma unroll
        for (int i = 0; i < PRE; ++i) {
            const int e = tid + i * nt;
            if (e < n) {
                int off;
                const uint32_t addr = where(t, lines, slot, e, off);
                cx<T> v = conj_if(src[off], pd.conj_out);
                if (pd.scale != 1.0) v = {v.x * scale, v.y * scale};
                put<false>(&out[addr], v);
            }
        }
        slot ^= 1;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_mtwiddle(const cx<T> *in, cx<T> *out, const MixedGridDesc g,
                                                  const cx<T> *__restrict__ table)
{
    // N < 2^31 and T < 2^24 on this path: 32-bit index arithmetic throughout
    const uint32_t stride = gridDim.x * blockDim.x;
    const uint32_t M = uint32_t(g.M), tn = uint32_t(g.T);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < uint32_t(g.N); i += stride) {
        uint32_t rank = i / M;
        uint32_t k = i - rank * M;
        uint32_t e = 0;
        for (int l = g.d - 1; l >= 0; --l) {
            const uint32_t sl = rank % uint32_t(g.p[l]);
            rank /= uint32_t(g.p[l]);
            const uint32_t kl = k % uint32_t(g.m[l]);
            k /= uint32_t(g.m[l]);
            e += (kl * sl) * uint32_t(g.tstep[l]);  // k_l s_l < n_l, times T / n_l: below T; d T < 2^27
        }
        cx<T> v = conj_if(get(&in[i]), g.conj_in);
        v = cmul(v, table[e % tn]);
        put<false>(&out[i], conj_if(v, g.conj_out));
    }
}

// With g.twiddle set, the element is also multiplied by Superstep 0's twiddle of
// its source position, omega^(sum_l k_l s_l) (the twiddle and the Put in one pass).
template <typename T>
__global__ __launch_bounds__(256) void k_mpermute(const cx<T> *in, cx<T> *out, const MixedGridDesc g,
                                                  const cx<T> *__restrict__ table)
{
    // N < 2^31 and T < 2^24 on this path: 32-bit index arithmetic throughout
    const uint32_t stride = gridDim.x * blockDim.x;
    const uint32_t M = uint32_t(g.M), tn = uint32_t(g.T);
    const T scale = static_cast<T>(g.scale);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < uint32_t(g.N); i += stride) {
        uint32_t r = i / M;
        uint32_t j = i - r * M;
        uint32_t src_rank = 0, src_k = 0, rmul = 1, kmul = 1, e = 0;
        for (int l = g.d - 1; l >= 0; --l) {
            const uint32_t jl = j % uint32_t(g.m[l]);
            j /= uint32_t(g.m[l]);
            const uint32_t rl = r % uint32_t(g.p[l]);
            r /= uint32_t(g.p[l]);
            const uint32_t sl = jl / uint32_t(g.q[l]);          // j_l = s_l q_l + t_l
            const uint32_t tl = jl - sl * uint32_t(g.q[l]);
            const uint32_t kl = rl + tl * uint32_t(g.p[l]);     // k_l = r_l + t_l p_l
            src_rank += sl * rmul;
            src_k += kl * kmul;
            e += (kl * sl) * uint32_t(g.tstep[l]);              // below T each; d T < 2^27
            rmul *= uint32_t(g.p[l]);
            kmul *= uint32_t(g.m[l]);
        }
        cx<T> v = conj_if(get(&in[src_rank * M + src_k]), g.conj_in);
        if (g.twiddle) v = cmul(v, table[e % tn]);
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

// The mixed-radix exchange where every grid side is a power of two (the local sides
// may be any product of 2, 3, 5, 7): the structure of k_exchange (fftu_exchange.hip)
// with general index arithmetic. A group is 64 consecutive local indices k (one
// per lane) of every source block; for k = r + t p (per dimension) the P sources
// s' are the inputs of one F_{p_1} x ... x F_{p_d} whose output k' lands in
// V^(r)[t + k' q] (Theorem 2.1). The grid dimensions with p_l > 1 split into NH
// leading wave dimensions of 2^LPH and NR trailing register dimensions of 2^LPR: a
// thread holds the 2^(NR LPR) sources of one wave index in registers (each load
// instruction reads 64 consecutive elements of one block), twiddles them by
// omega_T^e, e = sum_l s'_l k_l T / n_l (every term below T, the sum reduced with one
// quotient estimate), runs the register dimensions' DFTs with compile-time roots,
// swaps through LDS so that each thread holds every wave index of some register
// outputs, runs the wave dimensions' DFTs and scatters (runs of 64 / p_d elements).
template <typename T, int NR, int LPR, int NH, int LPH, bool ROWS>
__global__ __launch_bounds__(ROWS ? kMxRowsThreads : kExchangeThreads) void k_mxexchange(
    const cx<T> *__restrict__ Z, cx<T> *__restrict__ V, const MixedGridDesc g, const MxSplit sp, const MxRows rw,
    const cx<T> *__restrict__ table)
{
    constexpr int LOGR = NR * LPR, LOGH = NH * LPH;
    constexpr int R = 1 << LOGR;
    constexpr int H = 1 << LOGH;
    constexpr int U = LOGH > 0 ? R / H : R;   // register slots per thread after the LDS swap
    constexpr int NT = ROWS ? kMxRowsThreads : kExchangeThreads;
    constexpr int KG = (NT / 64) / H;
    static_assert(!ROWS || (LOGH > 0 && NR > 0), "k_mxexchange: staged rows reuse the wave swap's LDS");
    extern __shared__ unsigned char smem_raw[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int hw = wv & (H - 1);
    const int grp = wv >> LOGH;
    const uint32_t M = uint32_t(g.M);          // N < 2^31: 32-bit indices
    const uint32_t tn = uint32_t(g.T);
    const float inv_tn = 1.0f / float(tn);
    const T scale = static_cast<T>(g.scale);
    const cx<T> *mul = static_cast<const cx<T> *>(g.mul);
    // output offset of digit 1 of each register and wave dimension: k'_l moves by
    // q_l prod_{j>l} m_j (uniform)
    uint32_t ors[NR > 0 ? NR : 1], ohs[NH > 0 ? NH : 1];
    {
        uint32_t ms = 1;
#pragma unroll
        for (int l = kMaxDims - 1; l >= 0; --l) {
            if (l >= g.d) continue;
#pragma unroll
            for (int dd = 0; dd < NR; ++dd)
                if (sp.rdim[dd] == l) ors[dd] = uint32_t(g.q[l]) * ms;
#pragma unroll
            for (int dd = 0; dd < NH; ++dd)
                if (sp.hdim[dd] == l) ohs[dd] = uint32_t(g.q[l]) * ms;
            ms *= uint32_t(g.m[l]);
        }
    }
    auto reduce = [&](uint32_t e) {
        int32_t r = int32_t(e - uint32_t(float(e) * inv_tn) * tn);
        r += r < 0 ? int32_t(tn) : 0;
        r -= r >= int32_t(tn) ? int32_t(tn) : 0;
        return uint32_t(r);
    };
    // Work item it = (row rho, chunk c): the KG*64 slots of a workgroup take columns
    // k_{d-1} in [c KG 64, (c + 1) KG 64) of source row rho, so the row's outputs (one
    // full row of m_{d-1} elements per destination block and output digit) are written
    // by one workgroup. Rows run over k_0..k_{d-2} with k_{d-2} = r + p t taken t-fastest:
    // consecutive rows fill adjacent output rows, and a block of rw.bit items per
    // workgroup keeps a cache line shared by two rows inside one workgroup.
    const uint32_t mlast = uint32_t(g.m[g.d - 1]);
    const uint32_t nblk = __builtin_amdgcn_readfirstlane(int(gridDim.x));
    for (uint32_t it0 = blockIdx.x * rw.bit; it0 < rw.W; it0 += nblk * rw.bit)
    for (uint32_t it = it0; it < it0 + rw.bit && it < rw.W; ++it) {
        const uint32_t rho = it / rw.nchunk;
        const uint32_t kd = (it - rho * rw.nchunk) * uint32_t(KG * 64) + uint32_t(grp * 64 + lane);
        const bool valid = kd < mlast;
        uint32_t kx[kMaxDims];
        {
            uint32_t rem = rho;
#pragma unroll
            for (int l = kMaxDims - 1; l >= 0; --l) {
                kx[l] = 0;
                if (l >= g.d) continue;
                if (l == g.d - 1) {
                    kx[l] = valid ? kd : 0u;
                    continue;
                }
                const uint32_t ml = uint32_t(g.m[l]);
                const uint32_t raw = rem % ml;
                rem /= ml;
                if (l == g.d - 2) {
                    const uint32_t ql = uint32_t(g.q[l]);
                    kx[l] = raw / ql + uint32_t(g.p[l]) * (raw % ql);
                } else {
                    kx[l] = raw;
                }
            }
        }
        // k (row-major over m), the twiddle steps c_l = k_l T / n_l of the register and
        // wave dimensions, the destination block r and offset t
        uint32_t cr[NR > 0 ? NR : 1], ch[NH > 0 ? NH : 1];
        uint32_t k = 0, rank_r = 0, dst_t = 0;
        {
            uint32_t ms = 1, ps = 1;
#pragma unroll
            for (int l = kMaxDims - 1; l >= 0; --l) {
                if (l >= g.d) continue;
                const uint32_t ml = uint32_t(g.m[l]), pl = uint32_t(g.p[l]);
                const uint32_t kl = kx[l];
                const uint32_t cl = kl * uint32_t(g.tstep[l]);
#pragma unroll
                for (int dd = 0; dd < NR; ++dd)
                    if (sp.rdim[dd] == l) cr[dd] = cl;
#pragma unroll
                for (int dd = 0; dd < NH; ++dd)
                    if (sp.hdim[dd] == l) ch[dd] = cl;
                k += kl * ms;
                rank_r += (kl & (pl - 1)) * ps;          // p_l a power of two
                dst_t += (kl / pl) * ms;
                ms *= ml;
                ps *= pl;
            }
        }
        uint32_t e_hi = 0;
#pragma unroll
        for (int dd = 0; dd < NH; ++dd) e_hi += uint32_t((hw >> (LPH * (NH - 1 - dd))) & ((1 << LPH) - 1)) * ch[dd];

        cx<T> v[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const uint32_t s = (uint32_t(hw) << LOGR) + uint32_t(j);
            v[j] = valid ? get(&Z[s * M + k]) : cx<T>{T(0), T(0)};
        }
#pragma unroll
        for (int j = 0; j < R; ++j) {
            uint32_t e = e_hi;
#pragma unroll
            for (int dd = 0; dd < NR; ++dd) e += uint32_t((j >> (LPR * (NR - 1 - dd))) & ((1 << LPR) - 1)) * cr[dd];
            v[j] = conj_if(v[j], g.conj_in);
            // no branch around the table load (table[0] = 1 exactly when there is no
            // twiddle), so that the R loads issue back to back
            v[j] = cmul(v[j], table[g.twiddle ? reduce(e) : 0u]);
        }
        dft_digits<T, NR, LPR, 1, 1>(v);

        const uint32_t obase = rank_r * M + dst_t;
        auto roff = [&](int j) {
            uint32_t off = 0;
#pragma unroll
            for (int dd = 0; dd < NR; ++dd) off += uint32_t((j >> (LPR * (NR - 1 - dd))) & ((1 << LPR) - 1)) * ors[dd];
            return off;
        };
        auto hoff = [&](int i) {
            uint32_t off = 0;
#pragma unroll
            for (int dd = 0; dd < NH; ++dd) off += uint32_t((i >> (LPH * (NH - 1 - dd))) & ((1 << LPH) - 1)) * ohs[dd];
            return off;
        };
        auto store = [&](uint32_t idx, cx<T> w) {
            w = conj_if(w, g.conj_out);
            if (g.scale != 1.0) w = {w.x * scale, w.y * scale};
            if (mul) w = cmul(w, mul[idx]);
            V[idx] = w;   // cached: L2 merges the partial lines of neighbouring output runs
        };
        if constexpr (LOGH == 0) {
            if (valid) {
#pragma unroll
                for (int j = 0; j < R; ++j) store(obase + roff(j), v[j]);
            }
        } else {
            // swap through LDS: register j of wave hw goes to the wave that owns slot j
            // (complex128 in two rounds of doubles)
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
                cx<T> *lds = reinterpret_cast<cx<T> *>(smem_raw);
                __syncthreads();
#pragma unroll
                for (int j = 0; j < R; ++j) lds[((hw * R + j) * KG + grp) * 64 + lane] = v[j];
                __syncthreads();
#pragma unroll
                for (int x = 0; x < H; ++x)
#pragma unroll
                    for (int u = 0; u < U; ++u) w[x * U + u] = lds[((x * R + hw * U + u) * KG + grp) * 64 + lane];
            }
            dft_digits<T, NH, LPH, U, U>(w);
            if constexpr (ROWS) {
                // One round per wave digit x: every thread puts its U outputs of that x into
                // LDS as whole rows (row = the destination block's r_d and the register digits
                // other than the last dimension's, position u_{d-1} q_{d-1} + t), and the
                // workgroup stores the rows linearly: each row, m_{d-1} elements of one
                // destination block, is written contiguously.
                constexpr int RPR = R >> LPR;                 // rows per value of r_d
                const uint32_t plast = 1u << LPR, qlast = uint32_t(g.q[g.d - 1]);
                const uint32_t rd = kx[g.d - 1] & (plast - 1), tt = kx[g.d - 1] >> LPR;
                const uint32_t rank_hi = rank_r - rd, dst_hi = dst_t - tt;   // the row's block and offset
                const uint32_t relems = uint32_t(R) * mlast;
                const float inv_m = 1.0f / float(mlast);
                cx<T> *stage = reinterpret_cast<cx<T> *>(smem_raw);
#pragma unroll
                for (int x = 0; x < H; ++x) {
                    __syncthreads();   // the swap's (or the previous round's) LDS reads are done
                    if (valid) {
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const int j = hw * U + u;
                            const uint32_t row = rd * RPR + uint32_t(j >> LPR);
                            stage[row * mlast + uint32_t(j & ((1 << LPR) - 1)) * qlast + tt] = w[x * U + u];
                        }
                    }
                    __syncthreads();
                    const uint32_t xoff = hoff(x);
                    for (uint32_t e = uint32_t(tid); e < relems; e += NT) {
                        const uint32_t row = uint32_t(div_small(int(e), int(mlast), inv_m));
                        const uint32_t pos = e - row * mlast;
                        const uint32_t r = row / RPR, jh = row % RPR;
                        store((rank_hi + r) * M + dst_hi + xoff + roff(int(jh << LPR)) + pos, stage[e]);
                    }
                }
            } else if (valid) {
#pragma unroll
                for (int i = 0; i < H * U; ++i) store(obase + hoff(i / U) + roff(hw * U + i % U), w[i]);
            }
        }
    }
}

namespace {

// Work items of k_mxexchange: rows of the last dimension cut into chunks of `slots`
// columns. Rows go to workgroups in blocks of B (and all their chunks) when a row of
// the output is not a whole number of 128-byte lines, B the fewest rows that are and
// that divide q_{d-2}; otherwise one chunk per item.
MxRows mx_rows(const MixedGridDesc &g, int slots, size_t elem)
{
    MxRows rw{};
    const int64_t mlast = g.m[g.d - 1];
    rw.nchunk = uint32_t((mlast + slots - 1) / slots);
    const uint32_t rows = uint32_t(g.M / mlast);
    rw.W = rows * rw.nchunk;
    rw.bit = 1;
    const int64_t rowbytes = mlast * int64_t(elem);
    if (g.d >= 2 && rowbytes % 128 != 0)
        for (int b = 2; b <= 8; ++b)
            if ((b * rowbytes) % 128 == 0 && g.q[g.d - 2] % b == 0) {
                rw.bit = uint32_t(b) * rw.nchunk;
                break;
            }
    return rw;
}

template <typename T, int NR, int LPR, int NH, int LPH>
hipError_t mx_launch_t(const void *in, void *out, const MixedGridDesc &g, const MxSplit &sp, const void *table,
                       hipStream_t stream)
{
    if constexpr (NH * LPH > 0 && NR > 0 && NR * LPR <= 4) {
        if (mx_rows_staged(g, sp, sizeof(cx<T>))) {
            // one row per work item; LDS: the wave swap of kMxRowsThreads threads (8-byte words),
            // which also holds the R m_{d-1} staged outputs (m_{d-1} <= 512 / H)
            MxRows rw{};
            rw.nchunk = 1;
            rw.bit = 1;
            rw.W = uint32_t(g.M / g.m[g.d - 1]);
            const uint32_t lds = uint32_t(kMxRowsThreads) * (1u << (NR * LPR)) * 8u;
            if (uint64_t(1u << (NR * LPR)) * uint64_t(g.m[g.d - 1]) * sizeof(cx<T>) > lds) return hipErrorInvalidValue;
            const uint32_t blocks = rw.W < (1u << 20) ? rw.W : (1u << 20);
            hipLaunchKernelGGL((k_mxexchange<T, NR, LPR, NH, LPH, true>), dim3(blocks), dim3(kMxRowsThreads), lds, stream,
                               static_cast<const cx<T> *>(in), static_cast<cx<T> *>(out), g, sp, rw,
                               static_cast<const cx<T> *>(table));
            return hipGetLastError();
        }
    }
    constexpr int KG = (kExchangeThreads / 64) >> (NH * LPH);
    const MxRows rw = mx_rows(g, KG * 64, sizeof(cx<T>));
    const int64_t want = (int64_t(rw.W) + rw.bit - 1) / rw.bit;
    const uint32_t blocks = uint32_t(want < (int64_t(1) << 20) ? want : (int64_t(1) << 20));
    hipLaunchKernelGGL((k_mxexchange<T, NR, LPR, NH, LPH, false>), dim3(blocks), dim3(kExchangeThreads), sp.lds_bytes,
                       stream, static_cast<const cx<T> *>(in), static_cast<cx<T> *>(out), g, sp, rw,
                       static_cast<const cx<T> *>(table));
    return hipGetLastError();
}

template <typename T, int NR, int LPR>
hipError_t mx_launch_h(const void *in, void *out, const MixedGridDesc &g, const MxSplit &sp, const void *table,
                       hipStream_t stream)
{
    constexpr int LOGR = NR * LPR;
    if (sp.nh == 0) return mx_launch_t<T, NR, LPR, 0, 0>(in, out, g, sp, table, stream);
    if constexpr (LOGR >= 1)
        if (sp.nh == 1 && sp.lph == 1) return mx_launch_t<T, NR, LPR, 1, 1>(in, out, g, sp, table, stream);
    if constexpr (LOGR >= 2) {
        if (sp.nh == 1 && sp.lph == 2) return mx_launch_t<T, NR, LPR, 1, 2>(in, out, g, sp, table, stream);
        if (sp.nh == 2 && sp.lph == 1) return mx_launch_t<T, NR, LPR, 2, 1>(in, out, g, sp, table, stream);
    }
    return hipErrorInvalidValue;
}

template <typename T, int MAXR>
hipError_t mx_launch_r(const void *in, void *out, const MixedGridDesc &g, const MxSplit &sp, const void *table,
                       hipStream_t stream)
{
    switch (sp.nr * 8 + sp.lpr) {
    case 0 * 8 + 0: return mx_launch_h<T, 0, 0>(in, out, g, sp, table, stream);
    case 1 * 8 + 1: return mx_launch_h<T, 1, 1>(in, out, g, sp, table, stream);
    case 2 * 8 + 1: return mx_launch_h<T, 2, 1>(in, out, g, sp, table, stream);
    case 3 * 8 + 1: return mx_launch_h<T, 3, 1>(in, out, g, sp, table, stream);
    case 4 * 8 + 1: return mx_launch_h<T, 4, 1>(in, out, g, sp, table, stream);
    case 1 * 8 + 2: return mx_launch_h<T, 1, 2>(in, out, g, sp, table, stream);
    case 2 * 8 + 2: return mx_launch_h<T, 2, 2>(in, out, g, sp, table, stream);
    case 1 * 8 + 3: return mx_launch_h<T, 1, 3>(in, out, g, sp, table, stream);
    case 1 * 8 + 4: return mx_launch_h<T, 1, 4>(in, out, g, sp, table, stream);
    case 5 * 8 + 1:
        if constexpr (MAXR >= 5) return mx_launch_h<T, 5, 1>(in, out, g, sp, table, stream);
        return hipErrorInvalidValue;
    case 1 * 8 + 5:
        if constexpr (MAXR >= 5) return mx_launch_h<T, 1, 5>(in, out, g, sp, table, stream);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_mxexchange(Precision prec, const void *in, void *out, const MixedGridDesc &g, const MxSplit &sp,
                             const void *table, hipStream_t stream)
{
    if (g.P < 1 || g.T >= (int64_t(1) << 24) || g.N >= (int64_t(1) << 31) || g.d < 1 || g.d > kMaxDims)
        return hipErrorInvalidValue;
    int64_t P = 1;
    for (int l = 0; l < g.d; ++l) {
        if (g.p[l] < 1 || (g.p[l] & (g.p[l] - 1)) || g.m[l] % g.p[l] || g.q[l] * g.p[l] != g.m[l]) return hipErrorInvalidValue;
        P *= g.p[l];
    }
    if (P != g.P || (int64_t(1) << (sp.nr * sp.lpr + sp.nh * sp.lph)) != P) return hipErrorInvalidValue;
    return prec == Precision::F64 ? mx_launch_r<double, kExchangeRegBitsF64>(in, out, g, sp, table, stream)
                                  : mx_launch_r<float, kExchangeRegBitsF32>(in, out, g, sp, table, stream);
}

namespace {

uint32_t grid_for(int64_t count)
{
    const int64_t want = (count + 255) / 256;
    return uint32_t(want < (int64_t(1) << 18) ? (want > 0 ? want : 1) : (int64_t(1) << 18));
}

}  // namespace

namespace {

// Persistent grid of k_mline: the workgroups that fit on the device at once (per
// device and LDS size, cached), at most one per tile.
uint32_t mline_blocks(Precision prec, const MixedPassDesc &pd)
{
    constexpr int kDevices = 64, kLdsSlots = 65;
    static std::atomic<int> cus[kDevices];
    static std::atomic<int> per_cu[2][kLdsSlots];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDevices) return 0;
    int c = cus[dev].load(std::memory_order_relaxed);
    if (c == 0) {
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1) return 0;
        cus[dev].store(c, std::memory_order_relaxed);
    }
    const int slot = int((pd.lds_bytes + 1023) / 1024);
    if (slot >= kLdsSlots) return 0;
    std::atomic<int> &cached = per_cu[prec == Precision::F64 ? 1 : 0][slot];
    int nb = cached.load(std::memory_order_relaxed);
    if (nb == 0) {
        const hipError_t e =
            prec == Precision::F64
                ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_mline<double>, kMixedThreads, uint32_t(slot) * 1024u)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_mline<float>, kMixedThreads, uint32_t(slot) * 1024u);
        if (e != hipSuccess || nb < 1) nb = 1;
        cached.store(nb, std::memory_order_relaxed);
    }
    const int64_t want = int64_t(c) * nb;
    return uint32_t(pd.tiles < want ? pd.tiles : want);
}

}  // namespace

hipError_t launch_mline(Precision prec, const void *in, void *out, const MixedPassDesc &pd, const void *table,
                        hipStream_t stream)
{
    // a tile must fit the registers of the prefetch, and the indices 32 bits
    const int pre = prec == Precision::F64 ? kMixedPreF64 : kMixedPreF32;
    if (pd.W < 1 || pd.W > kMixedMaxW || (1 << pd.logW) != pd.W || int64_t(pd.W) * pd.L > int64_t(pre) * kMixedThreads ||
        pd.A * pd.B * pd.L >= (int64_t(1) << 31) || pd.tiles != (pd.A * pd.B + pd.W - 1) / pd.W)
        return hipErrorInvalidValue;
    const uint32_t blocks = mline_blocks(prec, pd);
    if (blocks == 0) return hipErrorInvalidValue;
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
    if (g.N < 1 || g.N >= (int64_t(1) << 31) || g.T < 1 || g.T >= (int64_t(1) << 24) || g.d < 1 || g.d > kMaxDims)
        return hipErrorInvalidValue;   // the kernel's 32-bit index arithmetic
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
    if (g.N < 1 || g.N >= (int64_t(1) << 31) || g.T < 1 || g.T >= (int64_t(1) << 24) || g.d < 1 || g.d > kMaxDims)
        return hipErrorInvalidValue;   // the kernel's 32-bit index arithmetic
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
