// HIP kernels for gfx950 (MI355X) of the cyclic-to-cyclic multidimensional FFT
// (Koopman & Bisseling, arXiv 2203.11795, Algorithm 2.3).
//
//   k_pass      Superstep 0 (and the unfused Superstep 2): batched Stockham FFTs
//               along a group of consecutive dimensions, one LDS tile per
//               workgroup, coalesced HBM reads and writes.
//   k_twiddle   Superstep 0's twiddle loop, Z[k] = prod_l omega_{n_l}^{k_l s_l} Y[k].
//   k_permute   Superstep 1 on its own: W^(r)[s q + t] = Z^(s)[r + t p].
//   (k_exchange, the fused twiddle + permutation + length-p FFTs, is in fftu_exchange.hip;
//    k_line, the register-direct single-dimension pass, is in fftu_line.hip.)
//
// Inverse transforms are run as conj(F(conj(x))): conjugation is exact, so this
// equals the transform with conjugated weights. Only the first load and the last
// store of a chain conjugate.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

#include "fftu_device.hpp"
#include "fftu_internal.hpp"

namespace fftu {

// ---------------------------------------------------------------------------
// k_pass: one Stockham stage over every line of one group axis, in place in LDS.
// Stage with radix R after Ns = 2^logNs: butterfly jj reads positions
// jj + r L/R, multiplies by omega_{Ns R}^{r (jj mod Ns)}, and writes positions
// (jj div Ns) Ns R + (jj mod Ns) + r Ns. Every thread holds its butterflies'
// operands in registers across the barrier between the reads and the writes.
// ---------------------------------------------------------------------------
template <typename T>
struct TileMax {
    static constexpr int value = 1 << (sizeof(T) == 8 ? kLogTileF64 : kLogTileF32);
};

template <typename T, int R>
__device__ __forceinline__ void pass_stage(cx<T> *buf, const PassDesc &pd, int logL, int logS, int logNs,
                                           const cx<T> *__restrict__ table)
{
    constexpr int logR = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : R == 16 ? 4 : 5;
    constexpr int NU = TileMax<T>::value / R / kPassThreads > 0 ? TileMax<T>::value / R / kPassThreads : 1;
    const int logW = pd.logW;
    const int logLR = logL - logR;
    const int units = 1 << (pd.logG + logW - logR);
    const int lw = pd.lw;
    cx<T> v[NU][R];
    int base[NU], ob[NU];
#pragma unroll
    for (int it = 0; it < NU; ++it) {
        const int u = threadIdx.x + it * kPassThreads;
        if (u < units) {
            const int w = u & ((1 << logW) - 1);
            const int rest = u >> logW;
            const int jj = rest & ((1 << logLR) - 1);
            const int other = rest >> logLR;
            const int lo = other & ((1 << logS) - 1);
            const int hi = other >> logS;
            base[it] = (((hi << (logL + logS)) + lo) * lw) + w;
#pragma unroll
            for (int r = 0; r < R; ++r) v[it][r] = buf[base[it] + (((jj + (r << logLR)) << logS) * lw)];
            if (logNs > 0) {
                const int jm = jj & ((1 << logNs) - 1);
                const int sh = pd.lognmax - logNs - logR;
#pragma unroll
                for (int r = 1; r < R; ++r) v[it][r] = cmul(v[it][r], table[(r * jm) << sh]);
            }
            Dft<T, R>::run(v[it]);
            ob[it] = ((jj >> logNs) << (logNs + logR)) + (jj & ((1 << logNs) - 1));
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < NU; ++it) {
        const int u = threadIdx.x + it * kPassThreads;
        if (u < units) {
#pragma unroll
            for (int r = 0; r < R; ++r) buf[base[it] + (((ob[it] + (r << logNs)) << logS) * lw)] = v[it][r];
        }
    }
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ void pass_tile(const cx<T> *in, cx<T> *out, const PassDesc &pd,
                                          const cx<T> *__restrict__ table, cx<T> *buf, int64_t t)
{
    int64_t a_base, b_base;
    if (pd.logB >= pd.logW) {
        a_base = t >> pd.logTPA;
        b_base = (t & ((int64_t(1) << pd.logTPA) - 1)) << pd.logW;
    } else {
        a_base = t << (pd.logW - pd.logBt);
        b_base = 0;
    }
    const int64_t gbase = a_base * pd.GB + b_base;
    const int tile = 1 << (pd.logG + pd.logW);
    const int bmask = (1 << pd.logBt) - 1;
    const int gmask = (1 << pd.logG) - 1;

    // Coalesced load of the tile: element e walks memory order (outer block, group position, inner).
    for (int e = threadIdx.x; e < tile; e += kPassThreads) {
        const int b = e & bmask;
        const int pos = (e >> pd.logBt) & gmask;
        const int ap = e >> (pd.logBt + pd.logG);
        const int64_t goff = gbase + int64_t(ap) * pd.GB + (int64_t(pos) << pd.logB) + b;
        buf[pos * pd.lw + ((ap << pd.logBt) | b)] = conj_if(get(&in[goff]), pd.conj_in);
    }
    __syncthreads();

    for (int ax = 0; ax < pd.naxes; ++ax) {
        const int logL = pd.loglen[ax], logS = pd.logstride[ax];
        int logNs = 0;
        for (int st = 0; st < pd.nstages[ax]; ++st) {
            const int logR = pd.lograd[ax][st];
            switch (logR) {
            case 1: pass_stage<T, 2>(buf, pd, logL, logS, logNs, table); break;
            case 2: pass_stage<T, 4>(buf, pd, logL, logS, logNs, table); break;
            case 3: pass_stage<T, 8>(buf, pd, logL, logS, logNs, table); break;
            default: pass_stage<T, 16>(buf, pd, logL, logS, logNs, table); break;
            }
            logNs += logR;
        }
    }

    const T scale = static_cast<T>(pd.scale);
    for (int e = threadIdx.x; e < tile; e += kPassThreads) {
        const int b = e & bmask;
        const int pos = (e >> pd.logBt) & gmask;
        const int ap = e >> (pd.logBt + pd.logG);
        const int64_t goff = gbase + int64_t(ap) * pd.GB + (int64_t(pos) << pd.logB) + b;
        cx<T> v = conj_if(buf[pos * pd.lw + ((ap << pd.logBt) | b)], pd.conj_out);
        if (pd.scale != 1.0) v = {v.x * scale, v.y * scale};
        put<false>(&out[goff], v);
    }
}


template <typename T>
__global__ __launch_bounds__(kPassThreads) void k_pass(const cx<T> *in, cx<T> *out, const PassDesc pd,
                                                       const cx<T> *__restrict__ table)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);
    const int64_t nblocks = __builtin_amdgcn_readfirstlane(int(gridDim.x));   // uniform loop (barriers inside)
    for (int64_t t = blockIdx.x; t < pd.tiles; t += nblocks) {
        pass_tile(in, out, pd, table, buf, t);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Pointwise kernels over the cyclic buffer (grid-stride over N elements).
// ---------------------------------------------------------------------------

// Twiddle exponent of local index k on processor s, as a power of
// omega_{2^lognmax}: sum_l k_l s_l 2^(lognmax - logn_l), reduced mod 2^lognmax.
__device__ __forceinline__ uint32_t twiddle_exponent(const GridDesc &g, int64_t rank_s, int64_t k)
{
    uint32_t e = 0;
    for (int l = 0; l < g.d; ++l) {
        const uint32_t kl = uint32_t((k >> g.logmstride[l]) & ((int64_t(1) << g.logm[l]) - 1));
        const uint32_t sl = uint32_t((rank_s >> g.logpstride[l]) & ((int64_t(1) << g.logp[l]) - 1));
        e += (kl * sl) << (g.lognmax - g.logn[l]);
    }
    return e & ((uint32_t(1) << g.lognmax) - 1);
}

template <typename T>
__global__ __launch_bounds__(kPointwiseThreads) void k_twiddle(const cx<T> *in, cx<T> *out, const GridDesc g,
                                                               const cx<T> *__restrict__ table)
{
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    const int logM = g.logmstride[0] + g.logm[0];
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < g.N; i += stride) {
        const int64_t s = i >> logM, k = i & ((int64_t(1) << logM) - 1);
        cx<T> v = cmul(conj_if(get(&in[i]), g.conj_in), table[twiddle_exponent(g, s, k)]);
        put<false>(&out[i], conj_if(v, g.conj_out));
    }
}

// One thread per destination element (r, i): i_l = s_l q_l + t_l, so the source
// is processor s at local index r + t p.
template <typename T>
__global__ __launch_bounds__(kPointwiseThreads) void k_permute(const cx<T> *__restrict__ in, cx<T> *__restrict__ out,
                                                               const GridDesc g)
{
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    const int logM = g.logmstride[0] + g.logm[0];
    for (int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < g.N; j += stride) {
        const int64_t r = j >> logM, i = j & ((int64_t(1) << logM) - 1);
        int64_t s = 0, src = 0;
        for (int l = 0; l < g.d; ++l) {
            const int logq = g.logm[l] - g.logp[l];
            const int64_t il = (i >> g.logmstride[l]) & ((int64_t(1) << g.logm[l]) - 1);
            const int64_t sl = il >> logq, tl = il & ((int64_t(1) << logq) - 1);
            const int64_t rl = (r >> g.logpstride[l]) & ((int64_t(1) << g.logp[l]) - 1);
            s += sl << g.logpstride[l];
            src += (rl + (tl << g.logp[l])) << g.logmstride[l];
        }
        put<false>(&out[j], get(&in[(s << logM) + src]));
    }
}

// Superstep 0's twiddle and Superstep 1 together where every q_l = n_l / p_l^2 is 1.
// Then m = p, M = P and t = 0, so W^(r)[s] = Z^(s)[r]: the exchange is the transpose
// of the P x M matrix of blocks. A workgroup moves one 64 x 64 tile (processors
// s0 + ds, local indices k0 + dk) through LDS, reading rows of 64 consecutive k and
// writing rows of 64 consecutive s. The twiddle prod_l omega_{n_l}^{k_l s_l} is a
// product of one factor per dimension; within a 64-aligned tile digit l of k is
// k_l0 + dk_l with dk_l < 2^b_l (b_l of the low 6 index bits belong to dimension l,
// the same for s since m = p), so each dimension needs only 2^(2 b_l) factors. The
// workgroup builds those in LDS (k_l s_l < n_l, no reduction) instead of reading the
// table once per element. A factor omega_T^e is read as omega_T^(e - e mod 2^h)
// omega_T^(e mod 2^h), h = ceil(log2(T) / 2): both reads fall in 2^h entries that
// stay in cache, where the exponents k_l s_l of a large n_l would scatter over the
// whole table (2^24 entries for the 2^24 x 64 shape). The tile's loads are issued
// before the factors are built.
//
// LD > 0: the innermost dimension has m_d = p_d = 2^LD <= 32 points, so the tile's
// 64 consecutive local indices hold whole lines of it, and its 64 consecutive
// processors whole groups of its p_d. The kernel then also runs Superstep 0's
// length-m_d FFTs (on the rows, with the twiddle applied as each line is written
// back) and Superstep 2's length-p_d FFTs (on the columns, each line stored straight
// from registers: its outputs are consecutive s, and plain stores let L2 join the
// lanes' pieces of each line) in registers with exact roots. The local FFT
// factorises over dimensions (eq. (1.3)), as does Superstep 2's, so the other
// dimensions' passes may come before and after. It may then be the last kernel:
// the store conjugates and scales as the descriptor says.
constexpr int kTransposeTile = 64;

template <typename T, int LD>
__global__ __launch_bounds__(kPointwiseThreads) void k_ttranspose(const cx<T> *__restrict__ in,
                                                                  cx<T> *__restrict__ out, const GridDesc g,
                                                                  const cx<T> *__restrict__ table)
{
    constexpr int TT = kTransposeTile;
    extern __shared__ unsigned char smem_raw[];
    cx<T> *tile = reinterpret_cast<cx<T> *>(smem_raw);   // [ds][dk], rows of TT + 1
    cx<T> *fac = tile + TT * (TT + 1);                    // per-dimension factor tables
    const int logM = g.logmstride[0] + g.logm[0];
    const int64_t tk = int64_t(blockIdx.x) & ((int64_t(1) << (logM - 6)) - 1);
    const int64_t ts = int64_t(blockIdx.x) >> (logM - 6);
    const int64_t k0 = tk << 6, s0 = ts << 6;
    const int tid = threadIdx.x;
    const int dk = tid & (TT - 1);
    constexpr int PER = TT * TT / kPointwiseThreads;   // elements per thread
    cx<T> r[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int ds = (tid >> 6) + i * (kPointwiseThreads / TT);
        r[i] = conj_if(get(&in[((s0 + ds) << logM) + k0 + dk]), g.conj_in);
    }
    // factor tables: dimension l holds omega_{n_l}^{(k_l0 + a)(s_l0 + b)} at off_l + a 2^b_l + b,
    // b_l = the low 6 index bits that belong to dimension l, off_l = sum_{j<l} 4^b_j
    auto lowbits = [&](int l) {
        const int b = 6 - g.logmstride[l];
        return b <= 0 ? 0 : (b < g.logm[l] ? b : g.logm[l]);
    };
    int total = 0;
    for (int l = 0; l < g.d; ++l) total += 1 << (2 * lowbits(l));
    for (int i = tid; i < total; i += kPointwiseThreads) {
        int l = 0, off = 0;
        while (i >= off + (1 << (2 * lowbits(l)))) {
            off += 1 << (2 * lowbits(l));
            ++l;
        }
        const int bl = lowbits(l);
        const int a = (i - off) >> bl, b = (i - off) & ((1 << bl) - 1);
        const uint32_t kl = uint32_t((k0 >> g.logmstride[l]) & ((int64_t(1) << g.logm[l]) - 1)) + uint32_t(a);
        const uint32_t sl = uint32_t((s0 >> g.logpstride[l]) & ((int64_t(1) << g.logp[l]) - 1)) + uint32_t(b);
        const uint32_t e = (kl * sl) << (g.lognmax - g.logn[l]);
        const int h = (g.lognmax + 1) >> 1;
        fac[i] = cmul(table[e & ~((uint32_t(1) << h) - 1)], table[e & ((uint32_t(1) << h) - 1)]);
    }
    // per-element product of the factors: the loop runs over every possible dimension
    // (compile-time indices, so the per-dimension constants stay in scalar registers)
    // and stops at g.d
    auto twiddle = [&](int dkk, int dss) {
        cx<T> w = {T(1), T(0)};
        int off = 0;
#pragma unroll
        for (int l = 0; l < kMaxDims; ++l) {
            if (l >= g.d) break;
            const int bl = lowbits(l);
            const int a = (dkk >> g.logmstride[l]) & ((1 << bl) - 1);
            const int b = (dss >> g.logpstride[l]) & ((1 << bl) - 1);
            w = cmul(w, fac[off + (a << bl) + b]);
            off += 1 << (2 * bl);
        }
        return w;
    };
    if constexpr (LD > 0) {
        constexpr int R = 1 << LD, LINES = TT * TT / R, GR = TT >> LD;
#pragma unroll
        for (int i = 0; i < PER; ++i) tile[((tid >> 6) + i * (kPointwiseThreads / TT)) * (TT + 1) + dk] = r[i];
        __syncthreads();
        // rows: Superstep 0 along the innermost dimension, then the twiddle, in place
        for (int line = tid; line < LINES; line += kPointwiseThreads) {
            const int dss = line / GR, base = dss * (TT + 1) + (line % GR) * R;
            cx<T> x[R];
#pragma unroll
            for (int i = 0; i < R; ++i) x[i] = tile[base + i];
            Dft<T, R>::run(x);
#pragma unroll
            for (int i = 0; i < R; ++i) tile[base + i] = cmul(x[i], twiddle((line % GR) * R + i, dss));
        }
        __syncthreads();
        // columns: Superstep 2 along the innermost grid dimension, stored straight out (the
        // R outputs of a lane are consecutive s; plain stores let L2 join the lanes' pieces)
        const T scale = static_cast<T>(g.scale);
        for (int line = tid; line < LINES; line += kPointwiseThreads) {
            const int gg = line % GR, dkk = line / GR;
            cx<T> x[R];
#pragma unroll
            for (int i = 0; i < R; ++i) x[i] = tile[(gg * R + i) * (TT + 1) + dkk];
            Dft<T, R>::run(x);
#pragma unroll
            for (int i = 0; i < R; ++i) {
                cx<T> v = conj_if(x[i], g.conj_out);
                if (g.scale != 1.0) v = {v.x * scale, v.y * scale};
                out[((k0 + dkk) << logM) + s0 + gg * R + i] = v;
            }
        }
        return;
    } else {
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int ds = (tid >> 6) + i * (kPointwiseThreads / TT);
        tile[ds * (TT + 1) + dk] = cmul(r[i], twiddle(dk, ds));
    }
    __syncthreads();
    const int ds = tid & (TT - 1);
    const T scale = static_cast<T>(g.scale);
#pragma unroll 4
    for (int dk2 = tid >> 6; dk2 < TT; dk2 += kPointwiseThreads / TT) {
        cx<T> v = conj_if(tile[ds * (TT + 1) + dk2], g.conj_out);
        if (g.scale != 1.0) v = {v.x * scale, v.y * scale};
        put<false>(&out[((k0 + dk2) << logM) + s0 + ds], v);
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
namespace {
constexpr int64_t kMaxBlocks = int64_t(1) << 22;   // keeps blocks x threads below 2^32

template <typename T>
hipError_t launch_pass_t(const void *in, void *out, const PassDesc &pd, const void *table, hipStream_t stream)
{
    const uint32_t blocks = uint32_t(pd.tiles < kMaxBlocks ? pd.tiles : kMaxBlocks);
    hipLaunchKernelGGL(k_pass<T>, dim3(blocks), dim3(kPassThreads), pd.lds_bytes, stream,
                       static_cast<const cx<T> *>(in), static_cast<cx<T> *>(out), pd,
                       static_cast<const cx<T> *>(table));
    return hipGetLastError();
}

uint32_t pointwise_blocks(int64_t n)
{
    const int64_t want = (n + kPointwiseThreads - 1) / kPointwiseThreads;
    return uint32_t(want < 262144 ? (want > 0 ? want : 1) : 262144);
}

}  // namespace

hipError_t launch_pass(Precision prec, const void *in, void *out, const PassDesc &pd, const void *table,
                       hipStream_t stream)
{
    // the signed load exists in the line kernels only
    if (pd.sign_mask != 0 && pd.kind != kLineStrided && pd.kind != kLineContig && pd.kind != kLineStaged)
        return hipErrorInvalidValue;
    if (pd.kind == kGroup2) return launch_group2(prec, in, out, pd, table, stream);
    if (pd.kind == kPair) return launch_pair(prec, in, out, pd, stream);
    if (pd.kind == kLong) return launch_long(prec, in, out, pd, table, stream);
    if (pd.kind != kTilePass) return launch_line(prec, in, out, pd, table, stream);
    return prec == Precision::F64 ? launch_pass_t<double>(in, out, pd, table, stream)
                                  : launch_pass_t<float>(in, out, pd, table, stream);
}

hipError_t launch_twiddle(Precision prec, const void *in, void *out, const GridDesc &g, const void *table,
                          hipStream_t stream)
{
    const uint32_t blocks = pointwise_blocks(g.N);
    if (prec == Precision::F64)
        hipLaunchKernelGGL(k_twiddle<double>, dim3(blocks), dim3(kPointwiseThreads), 0, stream,
                           static_cast<const cx<double> *>(in), static_cast<cx<double> *>(out), g,
                           static_cast<const cx<double> *>(table));
    else
        hipLaunchKernelGGL(k_twiddle<float>, dim3(blocks), dim3(kPointwiseThreads), 0, stream,
                           static_cast<const cx<float> *>(in), static_cast<cx<float> *>(out), g,
                           static_cast<const cx<float> *>(table));
    return hipGetLastError();
}

hipError_t launch_permute(Precision prec, const void *in, void *out, const GridDesc &g, hipStream_t stream)
{
    const uint32_t blocks = pointwise_blocks(g.N);
    if (prec == Precision::F64)
        hipLaunchKernelGGL(k_permute<double>, dim3(blocks), dim3(kPointwiseThreads), 0, stream,
                           static_cast<const cx<double> *>(in), static_cast<cx<double> *>(out), g);
    else
        hipLaunchKernelGGL(k_permute<float>, dim3(blocks), dim3(kPointwiseThreads), 0, stream,
                           static_cast<const cx<float> *>(in), static_cast<cx<float> *>(out), g);
    return hipGetLastError();
}

// bytes of LDS for k_ttranspose: the tile and the factor tables (at most 4^6 entries)
uint32_t ttranspose_lds_bytes(const GridDesc &g, int esize)
{
    int total = 0;
    for (int l = 0; l < g.d; ++l) {
        const int b = 6 - g.logmstride[l];
        const int bl = b <= 0 ? 0 : (b < g.logm[l] ? b : g.logm[l]);
        total += 1 << (2 * bl);
    }
    return uint32_t((kTransposeTile * (kTransposeTile + 1) + total) * esize);
}

namespace {
template <typename T, int LD>
void launch_ttranspose_t(const void *in, void *out, const GridDesc &g, const void *table, int64_t tiles, uint32_t lds,
                         hipStream_t stream)
{
    hipLaunchKernelGGL((k_ttranspose<T, LD>), dim3(uint32_t(tiles)), dim3(kPointwiseThreads), lds, stream,
                       static_cast<const cx<T> *>(in), static_cast<cx<T> *>(out), g, static_cast<const cx<T> *>(table));
}

template <typename T>
hipError_t launch_ttranspose_ld(int ld, const void *in, void *out, const GridDesc &g, const void *table, int64_t tiles,
                                uint32_t lds, hipStream_t stream)
{
    switch (ld) {
    case 0: launch_ttranspose_t<T, 0>(in, out, g, table, tiles, lds, stream); break;
    case 1: launch_ttranspose_t<T, 1>(in, out, g, table, tiles, lds, stream); break;
    case 2: launch_ttranspose_t<T, 2>(in, out, g, table, tiles, lds, stream); break;
    case 3: launch_ttranspose_t<T, 3>(in, out, g, table, tiles, lds, stream); break;
    case 4: launch_ttranspose_t<T, 4>(in, out, g, table, tiles, lds, stream); break;
    case 5: launch_ttranspose_t<T, 5>(in, out, g, table, tiles, lds, stream); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
}  // namespace

hipError_t launch_ttranspose(Precision prec, const void *in, void *out, const GridDesc &g, int ld, const void *table,
                             hipStream_t stream)
{
    const int logM = g.logmstride[0] + g.logm[0];
    for (int l = 0; l < g.d; ++l)
        if (g.logm[l] != g.logp[l] || g.logmstride[l] != g.logpstride[l]) return hipErrorInvalidValue;
    if (logM < 6 || g.N != (int64_t(1) << (2 * logM)) || in == out) return hipErrorInvalidValue;
    if (ld != 0 && (ld > 5 || g.logm[g.d - 1] != ld)) return hipErrorInvalidValue;
    const int64_t tiles = int64_t(1) << (2 * logM - 12);
    if (tiles > (int64_t(1) << 31) / kPointwiseThreads) return hipErrorInvalidValue;
    const int esize = prec == Precision::F64 ? 16 : 8;
    const uint32_t lds = ttranspose_lds_bytes(g, esize);
    return prec == Precision::F64 ? launch_ttranspose_ld<double>(ld, in, out, g, table, tiles, lds, stream)
                                  : launch_ttranspose_ld<float>(ld, in, out, g, table, tiles, lds, stream);
}

}  // namespace fftu
