/*
 * FP64 CPU oracle for the multidimensional DFT (Koopman & Bisseling,
 * "Minimizing communication in the multidimensional FFT", arXiv 2203.11795).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or load
 * this file: only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark use it. It shares no code, headers, tables or constants with
 * the HIP library.
 *
 * Everything here is the plain definition of the transform, written for
 * readability rather than speed:
 *   - oracle_dft_direct: the d-dimensional DFT summed term by term
 *     (Section 1, eq. (1.2)), O(N^2), for tiny arrays;
 *   - oracle_dft_points: the same sum for a chosen set of output indices,
 *     O(N) per output, for spot checks of large arrays;
 *   - oracle_fft_axes: 1-D DFTs applied along chosen axes one after the other
 *     (the row-column factorisation of Section 1.2, eq. (1.3)), each 1-D DFT
 *     computed by the textbook iterative radix-2 Cooley-Tukey FFT when its
 *     length is a power of two, and otherwise summed term by term from the
 *     1-D definition (O(L^2) per line, long double sums, exponents reduced
 *     exactly).
 *
 * Sign convention (Section 1, eq. (1.1)): omega_n = exp(-2*pi*i/n) for the
 * forward transform; sign = +1 conjugates every weight (unnormalised inverse).
 * Complex arrays are interleaved (re, im) doubles.
 *
 * Status codes: 0 success, 1 invalid argument, 3 out of memory.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double re, im;
} cplx;

static cplx c_add(cplx a, cplx b) { cplx r = {a.re + b.re, a.im + b.im}; return r; }
static cplx c_sub(cplx a, cplx b) { cplx r = {a.re - b.re, a.im - b.im}; return r; }
static cplx c_mul(cplx a, cplx b)
{
    cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    return r;
}

/* exp(sign * 2*pi*i * e / n), evaluated in long double on the exactly reduced
 * exponent e mod n; the four points e*4 == 0 (mod n) are returned exactly. */
static cplx root_of_unity(int64_t n, int64_t e, int sign)
{
    cplx w;
    e %= n;
    if (e < 0) e += n;
    if ((4 * e) % n == 0) {
        int64_t quarter = (4 * e) / n; /* 0..3 */
        static const double re4[4] = {1.0, 0.0, -1.0, 0.0};
        static const double im4[4] = {0.0, 1.0, 0.0, -1.0};
        w.re = re4[quarter];
        w.im = im4[quarter] * (double)sign;
        return w;
    }
    long double ang = 2.0L * 3.14159265358979323846264338327950288L * (long double)e / (long double)n;
    w.re = (double)cosl(ang);
    w.im = (double)(sinl(ang) * (long double)sign);
    return w;
}

static int is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * One 1-D DFT of length L (a power of two) on a contiguous buffer, in place:
 * bit-reversal permutation followed by log2(L) butterfly sweeps (radix-2
 * decimation in time). w[e] = omega_L^e for e in [L/2].
 */
static void fft1d_radix2(cplx *a, int64_t L, const cplx *w)
{
    for (int64_t i = 1, j = 0; i < L; ++i) {
        int64_t bit = L >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j |= bit;
        if (i < j) {
            cplx t = a[i];
            a[i] = a[j];
            a[j] = t;
        }
    }
    for (int64_t len = 2; len <= L; len <<= 1) {
        int64_t half = len / 2, step = L / len;
        for (int64_t base = 0; base < L; base += len) {
            for (int64_t k = 0; k < half; ++k) {
                cplx u = a[base + k];
                cplx v = c_mul(a[base + k + half], w[k * step]);
                a[base + k] = c_add(u, v);
                a[base + k + half] = c_sub(u, v);
            }
        }
    }
}

/*
 * In-place DFT along every axis a with bit a of axes_mask set, of a row-major
 * array of the given shape (eq. (1.3): the d-D DFT is the composition of 1-D
 * DFTs along each axis). Axes are processed from the last to the first.
 * nthreads <= 0 means "use the OpenMP default".
 */
/* y[k] = sum_j x[j] w[(j k) mod L] for k in [L]: the 1-D DFT of eq. (1.1) by its
 * definition, with w[e] = omega_L^e (sign included), long double sums. */
static void dft1d_direct(const cplx *x, cplx *y, int64_t L, const cplx *w)
{
    for (int64_t k = 0; k < L; ++k) {
        long double re = 0.0L, im = 0.0L;
        int64_t e = 0;                       /* (j k) mod L, advanced by k per term */
        for (int64_t j = 0; j < L; ++j) {
            re += (long double)x[j].re * w[e].re - (long double)x[j].im * w[e].im;
            im += (long double)x[j].re * w[e].im + (long double)x[j].im * w[e].re;
            e += k;
            if (e >= L) e -= L;
        }
        y[k].re = (double)re;
        y[k].im = (double)im;
    }
}

int oracle_fft_axes(int ndim, const int64_t *shape, uint32_t axes_mask, double *data, int sign,
                    int nthreads)
{
    if (ndim < 1 || ndim > 32 || !shape || !data || (sign != 1 && sign != -1)) return 1;
    int64_t total = 1;
    for (int a = 0; a < ndim; ++a) {
        if (shape[a] < 1) return 1;
        total *= shape[a];
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    cplx *x = (cplx *)data;
    for (int a = ndim - 1; a >= 0; --a) {
        if (!((axes_mask >> a) & 1u)) continue;
        int64_t L = shape[a];
        if (L == 1) continue;
        int64_t stride = 1;
        for (int b = a + 1; b < ndim; ++b) stride *= shape[b];
        int64_t outer = total / (L * stride);
        const int radix2 = is_pow2(L);
        const int64_t nw = radix2 ? L / 2 : L;
        cplx *w = (cplx *)malloc(sizeof(cplx) * (size_t)nw);
        if (!w) return 3;
        for (int64_t e = 0; e < nw; ++e) w[e] = root_of_unity(L, e, sign);
        int failed = 0;
#pragma omp parallel
        {
            cplx *line = (cplx *)malloc(sizeof(cplx) * (size_t)(2 * L));
            if (!line) {
#pragma omp atomic write
                failed = 1;
            } else {
#pragma omp for schedule(static)
                for (int64_t ln = 0; ln < outer * stride; ++ln) {
                    int64_t o = ln / stride, i = ln % stride;
                    cplx *base = x + o * L * stride + i;
                    for (int64_t j = 0; j < L; ++j) line[j] = base[j * stride];
                    if (radix2) {
                        fft1d_radix2(line, L, w);
                    } else {
                        dft1d_direct(line, line + L, L, w);
                        memcpy(line, line + L, sizeof(cplx) * (size_t)L);
                    }
                    for (int64_t j = 0; j < L; ++j) base[j * stride] = line[j];
                }
                free(line);
            }
        }
        free(w);
        if (failed) return 3;
    }
    return 0;
}

/* Multi-index of flat row-major index f. */
static void unravel(int64_t f, int ndim, const int64_t *shape, int64_t *idx)
{
    for (int a = ndim - 1; a >= 0; --a) {
        idx[a] = f % shape[a];
        f /= shape[a];
    }
}

/*
 * Direct evaluation of eq. (1.2) for every output: Y[k] = sum_j X[j] *
 * prod_l omega_{n_l}^{j_l k_l}. The exponent of each term is reduced exactly
 * in integers, as sum_l (j_l k_l mod n_l) * (N / n_l) mod N, so that a single
 * table of omega_N^e (long double) serves every term; sums are accumulated in
 * long double. Limited to N <= 16384.
 */
int oracle_dft_direct(int ndim, const int64_t *shape, const double *xin, double *yout, int sign)
{
    if (ndim < 1 || ndim > 32 || !shape || !xin || !yout || (sign != 1 && sign != -1)) return 1;
    int64_t N = 1;
    for (int a = 0; a < ndim; ++a) {
        if (shape[a] < 1) return 1;
        N *= shape[a];
    }
    if (N > 16384) return 1;
    long double *tre = (long double *)malloc(sizeof(long double) * (size_t)N);
    long double *tim = (long double *)malloc(sizeof(long double) * (size_t)N);
    int64_t *jidx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N * ndim));
    if (!tre || !tim || !jidx) {
        free(tre);
        free(tim);
        free(jidx);
        return 3;
    }
    for (int64_t e = 0; e < N; ++e) {
        long double ang = 2.0L * 3.14159265358979323846264338327950288L * (long double)e / (long double)N;
        tre[e] = cosl(ang);
        tim[e] = sinl(ang) * (long double)sign;
    }
    for (int64_t j = 0; j < N; ++j) unravel(j, ndim, shape, jidx + j * ndim);
    for (int64_t k = 0; k < N; ++k) {
        const int64_t *kk = jidx + k * ndim;
        long double sr = 0.0L, si = 0.0L;
        for (int64_t j = 0; j < N; ++j) {
            const int64_t *jj = jidx + j * ndim;
            int64_t e = 0;
            for (int a = 0; a < ndim; ++a) e = (e + ((jj[a] * kk[a]) % shape[a]) * (N / shape[a])) % N;
            long double xr = xin[2 * j], xi = xin[2 * j + 1];
            sr += xr * tre[e] - xi * tim[e];
            si += xr * tim[e] + xi * tre[e];
        }
        yout[2 * k] = (double)sr;
        yout[2 * k + 1] = (double)si;
    }
    free(tre);
    free(tim);
    free(jidx);
    return 0;
}

/*
 * eq. (1.2) for the npts outputs with flat row-major indices kflat[], O(N)
 * each. The weight of term j is the product over l of omega_{n_l}^{j_l k_l mod
 * n_l} taken from per-axis long double tables; the product and the sum are
 * formed in long double. Threads split the sum over j.
 */
int oracle_dft_points(int ndim, const int64_t *shape, const double *xin, int64_t npts,
                      const int64_t *kflat, double *yout, int sign, int nthreads)
{
    if (ndim < 1 || ndim > 32 || !shape || !xin || !kflat || !yout || npts < 0 ||
        (sign != 1 && sign != -1))
        return 1;
    int64_t N = 1;
    for (int a = 0; a < ndim; ++a) {
        if (shape[a] < 1) return 1;
        N *= shape[a];
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    for (int64_t pt = 0; pt < npts; ++pt) {
        if (kflat[pt] < 0 || kflat[pt] >= N) return 1;
        int64_t kk[32];
        unravel(kflat[pt], ndim, shape, kk);
        /* per-axis weights w_a[j_a] = omega_{n_a}^{j_a k_a} */
        long double *wre[32], *wim[32];
        int oom = 0;
        for (int a = 0; a < ndim; ++a) {
            wre[a] = (long double *)malloc(sizeof(long double) * (size_t)shape[a]);
            wim[a] = (long double *)malloc(sizeof(long double) * (size_t)shape[a]);
            if (!wre[a] || !wim[a]) oom = 1;
            for (int64_t j = 0; !oom && j < shape[a]; ++j) {
                int64_t e = (j * kk[a]) % shape[a];
                long double ang = 2.0L * 3.14159265358979323846264338327950288L * (long double)e /
                                  (long double)shape[a];
                wre[a][j] = cosl(ang);
                wim[a][j] = sinl(ang) * (long double)sign;
            }
        }
        long double sr = 0.0L, si = 0.0L;
        if (!oom) {
#pragma omp parallel for schedule(static) reduction(+ : sr, si)
            for (int64_t j = 0; j < N; ++j) {
                int64_t f = j;
                long double cr = 1.0L, ci = 0.0L;
                for (int a = ndim - 1; a >= 0; --a) {
                    int64_t ja = f % shape[a];
                    f /= shape[a];
                    long double nr = cr * wre[a][ja] - ci * wim[a][ja];
                    long double ni = cr * wim[a][ja] + ci * wre[a][ja];
                    cr = nr;
                    ci = ni;
                }
                long double xr = xin[2 * j], xi = xin[2 * j + 1];
                sr += xr * cr - xi * ci;
                si += xr * ci + xi * cr;
            }
        }
        for (int a = 0; a < ndim; ++a) {
            free(wre[a]);
            free(wim[a]);
        }
        if (oom) return 3;
        yout[2 * pt] = (double)sr;
        yout[2 * pt + 1] = (double)si;
    }
    return 0;
}
