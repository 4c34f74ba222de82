// The DCT-II and DST-II (and their exact inverses) in the zig-zag cyclic
// distribution, on top of the real transform. arXiv 2203.11795, Section 6, names
// them as the method's next transforms, built from 1-D algorithms dimension by
// dimension, with the zig-zag cyclic distribution to exploit their symmetry.
//
// Signal side: v, the zig-zag order of x along every dimension (v[m(j)] = x[j]:
// even samples ascending, then odd samples descending), in the real transform's
// packed layout. Its DFT V gives the DCT-II coefficients through one operator per
// dimension,
//     (C f)[k] = w^k f[k] + w^-k f[n - k],   w = exp(-2 pi i / (4 n)),
// (index n - 0 read as 0): y = (C_1 x ... x C_d) V, which is real. C_l couples
// k_l and n_l - k_l only, so a thread takes the 2^d indices that are mirror images
// of one representative (k_l in [0, n_l/2]) in any subset of the dimensions,
// forms V there from the complex transform of the packed signal (the real
// transform's split, in the same pass), applies the C_l in registers and stores
// y. On a pair (a, b) = (f[k], f[n - k]):
//     C a = w^k a + w^-k b,   C b = i (w^k a - w^-k b).
// The inverse applies C_l^-1, a = w^-k (g_a - i g_b) / 2, b = w^k (g_a + i g_b) / 2
// (k = 0: a = g_a / 2), writes V on the half spectrum and the plane (the real
// transform's complex side), and the inverse real transform gives v. At k = 0 and
// k = n/2 a and b are one element: only the first copy is stored.
// DST-II: y_s[k] = DCT-II(x')[n - 1 - k] with x'[j] = (-1)^j x[j], that is
// v'[m] = v[m] for m < n/2 and -v[m] otherwise along every dimension: a sign
// pass on the signal, the DCT, and the store at n_l - 1 - k_l.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "fftu_device.hpp"
#include "fftu_internal.hpp"

namespace fftu {

namespace {

// Buffer position of natural index k of the packed array n' (DIMS = D = d), or of
// the Nyquist plane's index (DIMS = D - 1, after the Nh packed elements). Compile-time
// dimension counts: the loop unrolls and k stays in registers.
template <int D, int DIMS>
__device__ __forceinline__ int64_t spec_position(const RealDesc &rd, const int32_t (&k)[D])
{
    uint32_t r = 0, i = 0;
#pragma unroll
    for (int l = 0; l < DIMS; ++l) {
        r = r * uint32_t(rd.p[l]) + uint32_t(k[l]) % uint32_t(rd.p[l]);
        i = i * uint32_t(rd.m[l]) + uint32_t(k[l]) / uint32_t(rd.p[l]);
    }
    return DIMS == D ? int64_t(r) * rd.Mh + i : rd.Nh + int64_t(r) * rd.Mp + i;
}

// Position of coefficient index k (cyclic over p).
template <int D>
__device__ __forceinline__ int64_t coeff_position(const R2RDesc &g, const int32_t (&k)[D])
{
    uint32_t r = 0, i = 0;
#pragma unroll
    for (int l = 0; l < D; ++l) {
        r = r * uint32_t(g.p[l]) + uint32_t(k[l]) % uint32_t(g.p[l]);
        i = i * uint32_t(g.m[l]) + uint32_t(k[l]) / uint32_t(g.p[l]);
    }
    return int64_t(r) * g.M + i;
}

// The representative of group t (k_l in [0, n_l/2], last dimension fastest).
template <int D>
__device__ __forceinline__ void representative(const R2RDesc &g, int64_t t, int32_t (&k)[D])
{
#pragma unroll
    for (int l = D - 1; l >= 0; --l) {
        const int64_t span = g.n[l] / 2 + 1;
        const int64_t q = t / span;
        k[l] = int32_t(t - q * span);
        t = q;
    }
}

// Member `mask` of the group: k_l mirrored where bit l is set.
template <int D>
__device__ __forceinline__ void member(const R2RDesc &g, const int32_t (&k)[D], int mask, int32_t (&kk)[D])
{
#pragma unroll
    for (int l = 0; l < D; ++l) kk[l] = ((mask >> l) & 1) ? (k[l] == 0 ? 0 : g.n[l] - k[l]) : k[l];
}

// A member that repeats another (a mirrored self-image: k_l = 0 or n_l / 2).
template <int D>
__device__ __forceinline__ bool repeated(const R2RDesc &g, const int32_t (&k)[D], int mask)
{
    bool rep = false;
#pragma unroll
    for (int l = 0; l < D; ++l) rep = rep || (((mask >> l) & 1) && (k[l] == 0 || 2 * k[l] == g.n[l]));
    return rep;
}

template <typename T>
__device__ __forceinline__ cx<T> times_i(cx<T> a) { return {-a.y, a.x}; }

}  // namespace

// Forward: the real transform's split and the coefficients in one pass. It reads
// Z = F(z), the complex transform of the packed signal z[j', j] = v[j', 2j] +
// i v[j', 2j + 1] (shape n', h = n_d / 2), before the split into the half
// spectrum: V[k] = E + w_{n_d}^{k_d} O at every full index k, with E = (Z[k~] +
// conj Z[-k~]) / 2 and O = (Z[k~] - conj Z[-k~]) / (2i), k~ = k with k_d mod h. The
// packed indices a group needs are the mirror images of its representative in
// packed space (k_d and n_d - k_d reduce to k_d and h - k_d mod h), and -k~ is the
// image with every coordinate mirrored: the complementary member.
template <typename T, int D>
__global__ __launch_bounds__(256) void k_r2rpost(const cx<T> *__restrict__ zf, T *__restrict__ y, const R2RDesc g,
                                                 const cx<T> *__restrict__ table)
{
    constexpr int G = 1 << D;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    const int32_t h = g.rd.h;
    const int64_t wstep = 4 * int64_t(g.tstep[D - 1]);   // omega_{n_d}^e = table entry e wstep
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < g.groups; t += stride) {
        int32_t k[D];
        representative<D>(g, t, k);
        cx<T> zv[G];
#pragma unroll
        for (int mask = 0; mask < G; ++mask) {
            int32_t pk[D];
            member<D>(g, k, mask, pk);
            const int32_t base = k[D - 1] == h ? 0 : k[D - 1];
            pk[D - 1] = ((mask >> (D - 1)) & 1) ? (base == 0 ? 0 : h - base) : base;
            zv[mask] = zf[spec_position<D, D>(g.rd, pk)];
        }
        cx<T> v[G];
#pragma unroll
        for (int mask = 0; mask < G; ++mask) {
            const cx<T> a = zv[mask], b = zv[(G - 1) ^ mask];
            const cx<T> E = {(a.x + b.x) * T(0.5), (a.y - b.y) * T(0.5)};
            const cx<T> O = {(a.y + b.y) * T(0.5), (b.x - a.x) * T(0.5)};
            const int32_t kd = ((mask >> (D - 1)) & 1) ? (k[D - 1] == 0 ? 0 : g.n[D - 1] - k[D - 1]) : k[D - 1];
            v[mask] = E + cmul(table[int64_t(kd) * wstep], O);
        }
#pragma unroll
        for (int l = 0; l < D; ++l) {
            const cx<T> w = table[int64_t(k[l]) * g.tstep[l]];
            const cx<T> wc = {w.x, -w.y};
#pragma unroll
            for (int mask = 0; mask < G; ++mask) {
                if ((mask >> l) & 1) continue;
                const int mb = mask | (1 << l);
                const cx<T> a = cmul(w, v[mask]), b = cmul(wc, v[mb]);
                v[mask] = a + b;
                v[mb] = times_i(a - b);
            }
        }
#pragma unroll
        for (int mask = 0; mask < G; ++mask) {
            if (repeated<D>(g, k, mask)) continue;
            int32_t kk[D];
            member<D>(g, k, mask, kk);
            if (g.dst) {
#pragma unroll
                for (int l = 0; l < D; ++l) kk[l] = g.n[l] - 1 - kk[l];
            }
            y[coeff_position<D>(g, kk)] = v[mask].x;
        }
    }
}

// The forward pass with whole coefficient rows staged in LDS. A workgroup takes one
// row of representatives (k_0..k_{D-2} fixed, k_{D-1} in [0, n_D / 2]): lane j takes
// k_{D-1} = j < h, and the lane with j = 0 also finishes the group k_{D-1} = h, whose
// packed inputs are the same (k_D mod h = 0 for both). The row's outputs are the
// 2^(D-1) coefficient rows of its leading mirror images, every one complete over
// k_{D-1} in [0, n_D); they go into LDS as [mirror][r_D][i_D] (one element of padding
// per segment) and out as p_D contiguous runs of m_D coefficients each. The
// arithmetic per group is that of k_r2rpost.
template <typename T, int D>
__global__ __launch_bounds__(256) void k_r2rpost_rows(const cx<T> *__restrict__ zf, T *__restrict__ y, const R2RDesc g,
                                                      const cx<T> *__restrict__ table, const int64_t rows)
{
    static_assert(D >= 2, "k_r2rpost_rows: rows of the last dimension");
    constexpr int G = 1 << D, GL = 1 << (D - 1);
    extern __shared__ unsigned char smem_raw[];
    T *stage = reinterpret_cast<T *>(smem_raw);
    __shared__ int64_t rowbase[GL];
    const int tid = threadIdx.x;
    const int32_t h = g.rd.h, nd = g.n[D - 1], pd = g.p[D - 1], md = g.m[D - 1];
    const int32_t seg = md + 1, rstride = pd * seg;
    const int64_t wstep = 4 * int64_t(g.tstep[D - 1]);
    const float inv_nd = 1.0f / float(nd), inv_md = 1.0f / float(md);
    auto udiv = [](int32_t a, int32_t b, float inv) {   // a / b for a < 2^22, one float estimate, corrected
        int32_t q = int32_t(float(a) * inv);
        const int32_t r = a - q * b;
        q += r >= b ? 1 : 0;
        q -= r < 0 ? 1 : 0;
        return q;
    };
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        int32_t k[D];
        {
            int64_t t = row;
#pragma unroll
            for (int l = D - 2; l >= 0; --l) {
                const int64_t span = g.n[l] / 2 + 1;
                const int64_t q = t / span;
                k[l] = int32_t(t - q * span);
                t = q;
            }
            k[D - 1] = 0;
        }
        if (tid < GL) {
            // output position of coefficient row `tid` at k_{D-1} = 0 (-1: a repeated image)
            int32_t kk[D];
            member<D>(g, k, tid, kk);
            bool rep = false;
#pragma unroll
            for (int l = 0; l < D - 1; ++l) rep = rep || (((tid >> l) & 1) && (k[l] == 0 || 2 * k[l] == g.n[l]));
            uint32_t r = 0, i = 0;
#pragma unroll
            for (int l = 0; l < D - 1; ++l) {
                const int32_t kl = g.dst ? g.n[l] - 1 - kk[l] : kk[l];
                r = r * uint32_t(g.p[l]) + uint32_t(kl) % uint32_t(g.p[l]);
                i = i * uint32_t(g.m[l]) + uint32_t(kl) / uint32_t(g.p[l]);
            }
            rowbase[tid] = rep ? int64_t(-1) : int64_t(r) * pd * g.M + int64_t(i) * md;
        }
        for (int32_t j = tid; j < h; j += 256) {
            k[D - 1] = j;
            cx<T> zv[G];
#pragma unroll
            for (int mask = 0; mask < G; ++mask) {
                int32_t pk[D];
                member<D>(g, k, mask, pk);
                pk[D - 1] = ((mask >> (D - 1)) & 1) ? (j == 0 ? 0 : h - j) : j;
                zv[mask] = zf[spec_position<D, D>(g.rd, pk)];
            }
            // one pass for k_{D-1} = j; the lane with j = 0 makes a second for k_{D-1} = h
            const int npass = j == 0 ? 2 : 1;
#pragma unroll 1
            for (int pass = 0; pass < npass; ++pass) {
                const int32_t klast = pass ? h : j;
                int32_t kr[D];
#pragma unroll
                for (int l = 0; l < D; ++l) kr[l] = k[l];
                kr[D - 1] = klast;
                cx<T> v[G];
#pragma unroll
                for (int mask = 0; mask < G; ++mask) {
                    const cx<T> a = zv[mask], b = zv[(G - 1) ^ mask];
                    const cx<T> E = {(a.x + b.x) * T(0.5), (a.y - b.y) * T(0.5)};
                    const cx<T> O = {(a.y + b.y) * T(0.5), (b.x - a.x) * T(0.5)};
                    const int32_t kd = ((mask >> (D - 1)) & 1) ? (klast == 0 ? 0 : nd - klast) : klast;
                    v[mask] = E + cmul(table[int64_t(kd) * wstep], O);
                }
#pragma unroll
                for (int l = 0; l < D; ++l) {
                    const cx<T> w = table[int64_t(kr[l]) * g.tstep[l]];
                    const cx<T> wc = {w.x, -w.y};
#pragma unroll
                    for (int mask = 0; mask < G; ++mask) {
                        if ((mask >> l) & 1) continue;
                        const int mb = mask | (1 << l);
                        const cx<T> a = cmul(w, v[mask]), b = cmul(wc, v[mb]);
                        v[mask] = a + b;
                        v[mb] = times_i(a - b);
                    }
                }
#pragma unroll
                for (int mask = 0; mask < G; ++mask) {
                    if (repeated<D>(g, kr, mask)) continue;
                    int32_t kl = ((mask >> (D - 1)) & 1) ? (klast == 0 ? 0 : nd - klast) : klast;
                    if (g.dst) kl = nd - 1 - kl;
                    const int32_t rl = kl % pd, il = kl / pd;
                    stage[(mask & (GL - 1)) * rstride + rl * seg + il] = v[mask].x;
                }
            }
        }
        __syncthreads();
        for (int32_t e = tid; e < GL * nd; e += 256) {
            const int32_t ml = udiv(e, nd, inv_nd);
            const int32_t pos = e - ml * nd;
            const int32_t rl = udiv(pos, md, inv_md);
            const int32_t il = pos - rl * md;
            const int64_t base = rowbase[ml];
            if (base >= 0) y[base + int64_t(rl) * g.M + il] = stage[ml * rstride + rl * seg + il];
        }
        __syncthreads();
    }
}

// ROWS: one workgroup per row of representatives (k_0..k_{D-2} fixed), lane j taking
// k_{D-1} = j and the lane with j = 0 also k_{D-1} = n_D / 2, so that every wave's
// half-spectrum stores (the members with k_D < n_D / 2) start on a multiple of 64
// along the last dimension; otherwise one group per thread over all groups.
template <typename T, int D, bool ROWS>
__global__ __launch_bounds__(256) void k_r2rpre(const T *__restrict__ y, cx<T> *__restrict__ spec, const R2RDesc g,
                                                const cx<T> *__restrict__ table, const int64_t rows)
{
    constexpr int G = 1 << D;
    auto group = [&](const int32_t (&k)[D]) {
        cx<T> v[G];
#pragma unroll
        for (int mask = 0; mask < G; ++mask) {
            int32_t kk[D];
            member<D>(g, k, mask, kk);
            if (g.dst) {
#pragma unroll
                for (int l = 0; l < D; ++l) kk[l] = g.n[l] - 1 - kk[l];
            }
            v[mask] = {y[coeff_position<D>(g, kk)], T(0)};
        }
#pragma unroll
        for (int l = 0; l < D; ++l) {
            const cx<T> w = table[int64_t(k[l]) * g.tstep[l]];
            const cx<T> wc = {w.x, -w.y};
#pragma unroll
            for (int mask = 0; mask < G; ++mask) {
                if ((mask >> l) & 1) continue;
                const int mb = mask | (1 << l);
                const cx<T> a = v[mask], b = v[mb];
                if (k[l] == 0) {
                    v[mask] = {a.x * T(0.5), a.y * T(0.5)};
                    v[mb] = v[mask];
                } else {
                    const cx<T> ib = times_i(b);
                    const cx<T> lo = cmul(wc, a - ib), hi = cmul(w, a + ib);
                    v[mask] = {lo.x * T(0.5), lo.y * T(0.5)};
                    v[mb] = {hi.x * T(0.5), hi.y * T(0.5)};
                }
            }
        }
        // the half spectrum and the plane: the members with k_d <= n_d / 2
#pragma unroll
        for (int mask = 0; mask < G / 2; ++mask) {
            if (repeated<D>(g, k, mask)) continue;
            int32_t kk[D];
            member<D>(g, k, mask, kk);
            const int64_t pos = kk[D - 1] < g.rd.h ? spec_position<D, D>(g.rd, kk) : spec_position<D, D - 1>(g.rd, kk);
            spec[pos] = v[mask];
        }
    };
    if constexpr (ROWS) {
        const int32_t h = g.rd.h;
        for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
            int32_t k[D];
            int64_t t = row;
#pragma unroll
            for (int l = D - 2; l >= 0; --l) {
                const int64_t span = g.n[l] / 2 + 1;
                const int64_t q = t / span;
                k[l] = int32_t(t - q * span);
                t = q;
            }
            for (int32_t j = threadIdx.x; j <= h; j += blockDim.x) {
                k[D - 1] = j;
                group(k);
            }
        }
    } else {
        const int64_t stride = int64_t(gridDim.x) * blockDim.x;
        for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < g.groups; t += stride) {
            int32_t k[D];
            representative<D>(g, t, k);
            group(k);
        }
    }
}

// The inverse's spectrum and the real transform's merge in one pass, one workgroup per
// row of representatives as k_r2rpre's ROWS form: the half spectrum and the plane,
// Y = (C_1^-1 x ... x C_d^-1) y, of every leading mirror image of the row stay in LDS
// as [mirror][k_d] (k_d in [0, n_d / 2]), and the packed spectrum Z = E + i O is formed
// from Y at (k', k_d) and (-k', n_d / 2 - k_d), or from Y at (k', 0) and the plane at k'
// for k_d = 0, which are all in the row (E = (a + conj b) / 2, O = (a - conj b)
// omega_{n_d}^{-k_d} / 2, as the merge computes them). Z goes out in runs of m'_d
// elements per block. A mirror image that repeats another (k_l = 0 or n_l / 2) takes
// that one's values and writes nothing.
template <typename T, int D>
__global__ __launch_bounds__(256) void k_r2rpre_merge(const T *__restrict__ y, cx<T> *__restrict__ zout,
                                                      const R2RDesc g, const cx<T> *__restrict__ table,
                                                      const int64_t rows)
{
    static_assert(D >= 2, "k_r2rpre_merge: rows of the last dimension");
    constexpr int G = 1 << D, GL = 1 << (D - 1);
    extern __shared__ unsigned char smem_raw[];
    cx<T> *ys = reinterpret_cast<cx<T> *>(smem_raw);   // [GL][h + 1]
    const int tid = threadIdx.x;
    const int32_t h = g.rd.h, hp = h + 1;
    const int32_t pd = g.rd.p[D - 1], md = g.rd.m[D - 1];   // the packed last side h = p_d m'_d
    const int64_t wstep = 4 * int64_t(g.tstep[D - 1]);       // omega_{n_d}^e = table entry e wstep
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        int32_t k[D];
        {
            int64_t t = row;
#pragma unroll
            for (int l = D - 2; l >= 0; --l) {
                const int64_t span = g.n[l] / 2 + 1;
                const int64_t q = t / span;
                k[l] = int32_t(t - q * span);
                t = q;
            }
        }
        uint32_t repbits = 0;   // leading dimensions whose mirror image is the same index
#pragma unroll
        for (int l = 0; l < D - 1; ++l)
            if (k[l] == 0 || 2 * k[l] == g.n[l]) repbits |= 1u << l;
        for (int32_t j = tid; j <= h; j += blockDim.x) {
            k[D - 1] = j;
            cx<T> v[G];
#pragma unroll
            for (int mask = 0; mask < G; ++mask) {
                int32_t kk[D];
                member<D>(g, k, mask, kk);
                if (g.dst) {
#pragma unroll
                    for (int l = 0; l < D; ++l) kk[l] = g.n[l] - 1 - kk[l];
                }
                v[mask] = {y[coeff_position<D>(g, kk)], T(0)};
            }
#pragma unroll
            for (int l = 0; l < D; ++l) {
                const cx<T> w = table[int64_t(k[l]) * g.tstep[l]];
                const cx<T> wc = {w.x, -w.y};
#pragma unroll
                for (int mask = 0; mask < G; ++mask) {
                    if ((mask >> l) & 1) continue;
                    const int mb = mask | (1 << l);
                    const cx<T> a = v[mask], b = v[mb];
                    if (k[l] == 0) {
                        v[mask] = {a.x * T(0.5), a.y * T(0.5)};
                        v[mb] = v[mask];
                    } else {
                        const cx<T> ib = times_i(b);
                        const cx<T> lo = cmul(wc, a - ib), hi = cmul(w, a + ib);
                        v[mask] = {lo.x * T(0.5), lo.y * T(0.5)};
                        v[mb] = {hi.x * T(0.5), hi.y * T(0.5)};
                    }
                }
            }
            // the members with k_d <= n_d / 2 (last dimension not mirrored)
#pragma unroll
            for (int mask = 0; mask < GL; ++mask) ys[mask * hp + j] = v[mask];
        }
        __syncthreads();
        for (int32_t e = tid; e < GL * h; e += blockDim.x) {
            const int32_t ml = e / h, rem = e - ml * h;
            if (uint32_t(ml) & repbits) continue;
            const int32_t rdd = rem / md, id = rem - rdd * md;
            const int32_t kd = rdd + pd * id;
            const cx<T> a = ys[ml * hp + kd];
            cx<T> zv;
            if (kd == 0) {
                const cx<T> c = ys[ml * hp + h];
                const cx<T> E = {(a.x + c.x) * T(0.5), (a.y + c.y) * T(0.5)};
                const cx<T> O = {(a.x - c.x) * T(0.5), (a.y - c.y) * T(0.5)};
                zv = {E.x - O.y, E.y + O.x};
            } else {
                const int32_t mc = int32_t(uint32_t(ml ^ (GL - 1)) & ~repbits);   // -k'
                const cx<T> b = ys[mc * hp + (h - kd)];
                const cx<T> E = {(a.x + b.x) * T(0.5), (a.y - b.y) * T(0.5)};
                const cx<T> w = table[int64_t(kd) * wstep];
                const cx<T> O = cmul(cx<T>{(a.x - b.x) * T(0.5), (a.y + b.y) * T(0.5)}, cx<T>{w.x, -w.y});
                zv = {E.x - O.y, E.y + O.x};
            }
            int32_t kk[D];
            member<D>(g, k, ml, kk);
            kk[D - 1] = kd;
            zout[spec_position<D, D>(g.rd, kk)] = zv;
        }
        __syncthreads();
    }
}

// The signs of the DST's signal: v[m] negated once for each dimension with
// m_l >= n_l / 2 (the odd samples of x), on the packed layout.
template <typename T, int D>
__global__ __launch_bounds__(256) void k_r2rsign(const cx<T> *in, cx<T> *out, const R2RDesc g)
{
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    const RealDesc &rd = g.rd;
    for (int64_t pos = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; pos < rd.Nh; pos += stride) {
        uint32_t r = uint32_t(pos / rd.Mh);
        uint32_t i = uint32_t(pos - int64_t(r) * rd.Mh);
        T s = T(1), s0 = T(1), s1 = T(1);
#pragma unroll
        for (int l = D - 1; l >= 0; --l) {
            const uint32_t sl = r % uint32_t(rd.p[l]);
            r /= uint32_t(rd.p[l]);
            const uint32_t il = i % uint32_t(rd.m[l]);
            i /= uint32_t(rd.m[l]);
            const int32_t j = int32_t(sl + il * uint32_t(rd.p[l]));   // packed natural index
            if (l == D - 1) {
                s0 = 2 * j < rd.h ? T(1) : T(-1);                     // signal index 2j against n_d / 2
                s1 = 2 * j + 1 < rd.h ? T(1) : T(-1);
            } else if (2 * j >= g.n[l]) {
                s = -s;
            }
        }
        const cx<T> a = in[pos];
        out[pos] = {a.x * s * s0, a.y * s * s1};
    }
}

namespace {

// One thread per group or element over up to 2^22 workgroups (a grid capped at 65536
// made the sign pass's threads loop, 0.40 against 0.34 ms at 512^3).
uint32_t grid_of(int64_t count)
{
    const int64_t want = (count + 255) / 256;
    return uint32_t(want < (1 << 22) ? (want > 0 ? want : 1) : (1 << 22));
}

bool r2r_ok(const R2RDesc &g)
{
    if (g.d < 1 || g.d > kR2RMaxDims || g.d != g.rd.d || g.groups < 1) return false;
    for (int l = 0; l < g.d; ++l)
        if (g.n[l] < 2 || g.n[l] % 2 || g.p[l] < 1 || g.m[l] * g.p[l] != g.n[l] || g.tstep[l] < 1) return false;
    return true;
}

template <typename T>
hipError_t post_t(const void *spec, void *y, const R2RDesc &g, const void *table, hipStream_t stream)
{
    const cx<T> *a = static_cast<const cx<T> *>(spec), *tab = static_cast<const cx<T> *>(table);
    T *b = static_cast<T *>(y);
    const uint32_t lds = r2rpost_rows_lds(g, sizeof(T));
    if (lds > 0) {
        const int64_t rows = g.groups / (g.n[g.d - 1] / 2 + 1);
        const uint32_t blocks = uint32_t(rows < (int64_t(1) << 20) ? rows : (int64_t(1) << 20));
        switch (g.d) {
        case 2: hipLaunchKernelGGL((k_r2rpost_rows<T, 2>), dim3(blocks), dim3(256), lds, stream, a, b, g, tab, rows); break;
        case 3: hipLaunchKernelGGL((k_r2rpost_rows<T, 3>), dim3(blocks), dim3(256), lds, stream, a, b, g, tab, rows); break;
        case 4: hipLaunchKernelGGL((k_r2rpost_rows<T, 4>), dim3(blocks), dim3(256), lds, stream, a, b, g, tab, rows); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const uint32_t blocks = grid_of(g.groups);
    switch (g.d) {
    case 1: hipLaunchKernelGGL((k_r2rpost<T, 1>), dim3(blocks), dim3(256), 0, stream, a, b, g, tab); break;
    case 2: hipLaunchKernelGGL((k_r2rpost<T, 2>), dim3(blocks), dim3(256), 0, stream, a, b, g, tab); break;
    case 3: hipLaunchKernelGGL((k_r2rpost<T, 3>), dim3(blocks), dim3(256), 0, stream, a, b, g, tab); break;
    case 4: hipLaunchKernelGGL((k_r2rpost<T, 4>), dim3(blocks), dim3(256), 0, stream, a, b, g, tab); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t pre_t(const void *y, void *spec, const R2RDesc &g, const void *table, hipStream_t stream)
{
    const T *a = static_cast<const T *>(y);
    cx<T> *b = static_cast<cx<T> *>(spec);
    const cx<T> *tab = static_cast<const cx<T> *>(table);
    if (r2rpre_rows(g)) {
        const int64_t rows = g.groups / (g.n[g.d - 1] / 2 + 1);
        const uint32_t blocks = uint32_t(rows < (int64_t(1) << 20) ? rows : (int64_t(1) << 20));
        switch (g.d) {
        case 2: hipLaunchKernelGGL((k_r2rpre<T, 2, true>), dim3(blocks), dim3(256), 0, stream, a, b, g, tab, rows); break;
        case 3: hipLaunchKernelGGL((k_r2rpre<T, 3, true>), dim3(blocks), dim3(256), 0, stream, a, b, g, tab, rows); break;
        case 4: hipLaunchKernelGGL((k_r2rpre<T, 4, true>), dim3(blocks), dim3(256), 0, stream, a, b, g, tab, rows); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const uint32_t blocks = grid_of(g.groups);
    switch (g.d) {
    case 1: hipLaunchKernelGGL((k_r2rpre<T, 1, false>), dim3(blocks), dim3(256), 0, stream, a, b, g, tab, int64_t(0)); break;
    case 2: hipLaunchKernelGGL((k_r2rpre<T, 2, false>), dim3(blocks), dim3(256), 0, stream, a, b, g, tab, int64_t(0)); break;
    case 3: hipLaunchKernelGGL((k_r2rpre<T, 3, false>), dim3(blocks), dim3(256), 0, stream, a, b, g, tab, int64_t(0)); break;
    case 4: hipLaunchKernelGGL((k_r2rpre<T, 4, false>), dim3(blocks), dim3(256), 0, stream, a, b, g, tab, int64_t(0)); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

namespace {
template <typename T>
hipError_t pre_merge_t(const void *y, void *z, const R2RDesc &g, const void *table, hipStream_t stream)
{
    const uint32_t lds = r2rpre_merge_lds(g, sizeof(cx<T>));
    if (lds == 0) return hipErrorInvalidValue;
    const int64_t rows = g.groups / (g.n[g.d - 1] / 2 + 1);
    const uint32_t blocks = uint32_t(rows < (int64_t(1) << 20) ? rows : (int64_t(1) << 20));
    const T *a = static_cast<const T *>(y);
    cx<T> *b = static_cast<cx<T> *>(z);
    const cx<T> *tab = static_cast<const cx<T> *>(table);
    switch (g.d) {
    case 2: hipLaunchKernelGGL((k_r2rpre_merge<T, 2>), dim3(blocks), dim3(256), lds, stream, a, b, g, tab, rows); break;
    case 3: hipLaunchKernelGGL((k_r2rpre_merge<T, 3>), dim3(blocks), dim3(256), lds, stream, a, b, g, tab, rows); break;
    case 4: hipLaunchKernelGGL((k_r2rpre_merge<T, 4>), dim3(blocks), dim3(256), lds, stream, a, b, g, tab, rows); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
}  // namespace

hipError_t launch_r2r_pre_merge(Precision prec, const void *y, void *z, const R2RDesc &g, const void *table4,
                                hipStream_t stream)
{
    if (!r2r_ok(g)) return hipErrorInvalidValue;
    return prec == Precision::F64 ? pre_merge_t<double>(y, z, g, table4, stream) : pre_merge_t<float>(y, z, g, table4, stream);
}

hipError_t launch_r2r_post(Precision prec, const void *spec, void *y, const R2RDesc &g, const void *table4,
                           hipStream_t stream)
{
    if (!r2r_ok(g)) return hipErrorInvalidValue;
    return prec == Precision::F64 ? post_t<double>(spec, y, g, table4, stream)
                                  : post_t<float>(spec, y, g, table4, stream);
}

hipError_t launch_r2r_pre(Precision prec, const void *y, void *spec, const R2RDesc &g, const void *table4,
                          hipStream_t stream)
{
    if (!r2r_ok(g)) return hipErrorInvalidValue;
    return prec == Precision::F64 ? pre_t<double>(y, spec, g, table4, stream)
                                  : pre_t<float>(y, spec, g, table4, stream);
}

hipError_t launch_r2r_sign(Precision prec, const void *in, void *out, const R2RDesc &g, hipStream_t stream)
{
    if (!r2r_ok(g)) return hipErrorInvalidValue;
    const uint32_t blocks = grid_of(g.rd.Nh);
    auto go = [&](auto dc) {
        constexpr int D = decltype(dc)::value;
        if (prec == Precision::F64)
            hipLaunchKernelGGL((k_r2rsign<double, D>), dim3(blocks), dim3(256), 0, stream,
                               static_cast<const cx<double> *>(in), static_cast<cx<double> *>(out), g);
        else
            hipLaunchKernelGGL((k_r2rsign<float, D>), dim3(blocks), dim3(256), 0, stream,
                               static_cast<const cx<float> *>(in), static_cast<cx<float> *>(out), g);
    };
    switch (g.d) {   // r2r_ok: d <= kR2RMaxDims = 4
    case 1: go(std::integral_constant<int, 1>{}); break;
    case 2: go(std::integral_constant<int, 2>{}); break;
    case 3: go(std::integral_constant<int, 3>{}); break;
    case 4: go(std::integral_constant<int, 4>{}); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fftu
