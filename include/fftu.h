/*
 * fftu.h -- C ABI of the MI355X (gfx950) implementation of the cyclic-to-cyclic
 * multidimensional FFT with a single all-to-all of Koopman & Bisseling,
 * "Minimizing communication in the multidimensional FFT" (arXiv 2203.11795).
 *
 * What is computed (Section 2.2, Algorithm 2.3 and Theorem 2.1): the
 * d-dimensional DFT of eq. (1.2),
 *     Y[k] = sum_j X[j] prod_l omega_{n_l}^{j_l k_l},  omega_n = exp(-2 pi i / n),
 * of an n_1 x ... x n_d complex array X that is held in the d-dimensional cyclic
 * distribution over a virtual p_1 x ... x p_d processor grid (Section 1.1,
 * phi(s, k) = s + k p elementwise), and the result Y is returned in the same
 * distribution. The P = p_1...p_d virtual processors live in one GPU's HBM; the
 * one all-to-all of Superstep 1 is a permutation inside that memory.
 *
 * Buffer layout (both input and output): N = n_1...n_d complex elements,
 * interleaved (re, im), stored processor by processor:
 *     buf[rank(s) * M + lin(k)] = X[s_1 + k_1 p_1, ..., s_d + k_d p_d]
 * with M = N / P, rank(s) row-major over s (s_d fastest) and lin(k) row-major
 * over the local index k in [n_1/p_1] x ... x [n_d/p_d] (the paper's local
 * arrays are row-major, Section 3). With p = (1, ..., 1) this is the ordinary
 * row-major array.
 *
 * Requirements on a plan (Algorithm 2.3, Input): p_l^2 divides n_l for every l;
 * the transform then has one communication superstep. Grids beyond that
 * (Section 2.3, after eq. (2.13): p_l | n_l but not p_l^2 | n_l for some l) take
 * several supersteps through the group-cyclic distribution: per dimension, with
 * m_l = n_l / p_l, level i handles sub-transforms of n_i points on groups of p_i
 * processors (n_0 = n_l, p_0 = p_l; n_{i+1} = p_i, p_{i+1} = p_i / m_l, which
 * needs m_l | p_i) until a level h has p_h^2 | n_h; the transform takes
 * max_l (h_l + 1) supersteps. A grid whose chain fails (e.g. n_l = p_l > 1)
 * gives FFTU_ERROR_NOT_DIVISIBLE. Such grids run on the mixed-radix kernels and
 * have its limits (below), with lines of m_l and p_h points.
 * This implementation also requires 1 <= d <= FFTU_MAX_DIMS and either
 *   - every n_l and p_l a power of two, N < 2^40, n_l/p_l and p_l <= 2048
 *     (complex128) or 4096 (complex64); or
 *   - every n_l with no prime factor other than 2, 3, 5, 7 (the mixed-radix
 *     path), N < 2^31, n_l/p_l and p_l <= 1024 (complex128) or 2048
 *     (complex64), lcm(n_1, ..., n_d) <= 2^24.
 *
 * Directions: FFTU_FORWARD uses omega_n = exp(-2 pi i / n) and is unnormalised;
 * FFTU_INVERSE conjugates every weight and multiplies by 1/N (Section 1.3,
 * last paragraph), so that inverse(forward(x)) = x.
 *
 * Ownership: the caller owns the input and output buffers (device memory,
 * aligned to the element size: 8 bytes for complex64, 16 for complex128). A
 * plan owns its twiddle table and a workspace of N elements in device memory,
 * allocated on the device that is current when the plan is created, and freed
 * by fftu_destroy. Execution calls never allocate and never synchronise.
 *
 * Errors: each call returns (or records, for calls returning a handle) a status;
 * fftu_last_error() returns the status of the last failing or succeeding call
 * on the calling thread. Argument errors are reported by fftu_plan/fftu_check;
 * execution calls report only FFTU_ERROR_INVALID_VALUE (NULL plan or buffer,
 * a buffer not aligned to the element size, or a forbidden aliasing) and
 * FFTU_ERROR_DEVICE (a HIP launch error).
 *
 * Concurrency: a plan may be executed by one stream at a time (the workspace is
 * shared by its calls). Different plans are independent. Planning may run on
 * several threads; the tuning knobs (fftu_set_tuning) are process-wide.
 */
#ifndef FFTU_H
#define FFTU_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FFTU_MAX_DIMS 8

typedef struct fftu_plan_s *fftu_plan_t;

/* Element types: interleaved complex. */
typedef enum {
    FFTU_C64 = 1,  /* float re, float im  (8 bytes)  */
    FFTU_C128 = 2  /* double re, double im (16 bytes) */
} fftu_dtype;

typedef enum {
    FFTU_FORWARD = -1, /* omega_n = exp(-2 pi i / n), unnormalised */
    FFTU_INVERSE = 1   /* conjugated weights, times 1/N */
} fftu_direction;

typedef enum {
    FFTU_SUCCESS = 0,
    FFTU_ERROR_INVALID_VALUE = 1, /* bad argument: d, n_l, p_l < 1, NULL pointer, bad enum, aliasing */
    FFTU_ERROR_NOT_DIVISIBLE = 2, /* p_l^2 does not divide n_l (Algorithm 2.3 precondition) */
    FFTU_ERROR_UNSUPPORTED = 3,   /* valid for the paper's method but outside this build: non-power-of-two
                                     sizes, d > FFTU_MAX_DIMS, local length above the limit */
    FFTU_ERROR_OUT_OF_MEMORY = 4, /* device allocation failed */
    FFTU_ERROR_DEVICE = 5         /* HIP runtime or launch error */
} fftu_status;

/*
 * Planner tuning knobs (process-wide, read when a plan is created; plans that
 * exist keep their choices). A value of -1 restores the planner's default.
 * Used by the autotuner; every setting gives the same results up to rounding.
 */
typedef enum {
    FFTU_TUNE_LINE_STRIDED_LOGW = 0, /* log2 columns per workgroup, strided single-dimension passes (2..6) */
    FFTU_TUNE_LINE_CONTIG_LOGW = 1,  /* log2 lines per workgroup, contiguous single-dimension passes (0..8) */
    FFTU_TUNE_LINE_PAD = 2,          /* LDS padding (elements) per row of a strided pass tile (0..4) */
    FFTU_TUNE_MAX_LDS_KB = 3,        /* LDS budget per workgroup of a pass, KiB (16..160; default 64) */
    FFTU_TUNE_FUSE_LAST = 4,         /* 0: never fuse the innermost dimension's lines into the exchange; 1 / -1: when possible */
    FFTU_TUNE_PAIR = 5,              /* 0: one pass per strided dimension; 1 / -1: two adjacent dimensions of 8..32-point lines share a pass */
    FFTU_TUNE_MIXED_RADIX = 6,       /* largest power-of-two radix of a mixed-radix line (2, 4, 8; default 8). Unlike
                                        the other knobs this changes the arithmetic: results move within rounding */
    FFTU_TUNE_MIXED_TILE_LOG = 7,    /* log2 elements per mixed-radix pass tile (9..12; default 10 for complex128,
                                        11 for complex64) */
    FFTU_TUNE_COUNT = 8
} fftu_tune_param;

/* Set a tuning knob; FFTU_ERROR_INVALID_VALUE for an unknown knob or a value out of range. */
fftu_status fftu_set_tuning(fftu_tune_param param, int value);

/* Current value of a knob (-1: planner default). */
int fftu_get_tuning(fftu_tune_param param);

/* Static description of how a plan executes (host-side; see fftu_describe). */
typedef struct {
    int32_t d;
    int64_t N;                /* total elements */
    int64_t P;                /* virtual processors p_1...p_d */
    int64_t M;                /* local elements per processor, N / P */
    int32_t s0_kernels;       /* separate kernel launches of Superstep 0 (local FFTs) */
    int32_t exchange_fused;   /* 1: twiddle, permutation, length-p FFTs and scaling run as one kernel;
                                 2: so do the innermost dimension's local FFTs (s0_kernels excludes them) */
    int32_t s2_kernels;       /* extra launches for Supersteps 1-2 when not fused: twiddle and permutation (one
                                 tiled transpose where every q_l = 1), then the F_p passes */
    int32_t launches;         /* kernel launches of one fftu_execute */
    uint64_t workspace_bytes; /* device workspace owned by the plan */
    uint64_t table_bytes;     /* device twiddle table owned by the plan */
    int32_t supersteps;       /* communication supersteps: 1 when every p_l^2 | n_l, more on group-cyclic grids */
} fftu_plan_info;

/* Library version string ("fftu <major>.<minor>"). */
const char *fftu_version(void);

/* Human-readable name of a status code. Never NULL. */
const char *fftu_status_string(fftu_status s);

/* Status of the most recent fftu_* call on the calling thread. */
fftu_status fftu_last_error(void);

/*
 * Validate a plan request on the host without touching any device.
 * Returns FFTU_SUCCESS iff fftu_plan with the same arguments would succeed
 * (device memory permitting). Arguments as for fftu_plan.
 */
fftu_status fftu_check(int d, const int64_t n[], const int64_t p[], fftu_dtype dtype, fftu_direction direction);

/*
 * Host-only dry run of the planner: fills *info for a valid request without
 * touching any device. Returns the same status as fftu_check.
 */
fftu_status fftu_describe(int d, const int64_t n[], const int64_t p[], fftu_dtype dtype,
                          fftu_direction direction, fftu_plan_info *info);

/*
 * Create a plan for the d-dimensional transform of an n[0] x ... x n[d-1]
 * array over the p[0] x ... x p[d-1] virtual grid (Algorithm 2.3).
 * n and p are host arrays of d entries, read during the call only.
 * Allocates the twiddle table (omega_L^j, j in [L], L = max n_l, generated in
 * FP64 on the host; the complex64 table is the FP64 table rounded once) and
 * an N-element workspace on the current device.
 * Returns NULL on failure; fftu_last_error() gives the reason.
 */
fftu_plan_t fftu_plan(int d, const int64_t n[], const int64_t p[], fftu_dtype dtype, fftu_direction direction);

/* Fill *info for an existing plan. */
fftu_status fftu_get_plan_info(fftu_plan_t plan, fftu_plan_info *info);

/*
 * Name of the kernel that fftu_execute launches at position i (0-based, i <
 * launches), as the profiler reports it, e.g. "fftu::k_line<double, 7, 1>".
 * The string is owned by the plan. NULL for a bad plan or index.
 */
const char *fftu_launch_name(fftu_plan_t plan, int i);

/* Device bytes owned by the plan (table + workspace), for memory admission. */
size_t fftu_plan_device_bytes(fftu_plan_t plan);

/*
 * The whole transform (Algorithm 2.3: Superstep 0 local FFTs and twiddle,
 * Superstep 1 permutation, Superstep 2 length-p FFTs): out = F(in), both in the
 * cyclic buffer layout above. in and out are device pointers to N elements of
 * the plan's dtype, on the plan's device; in == out is allowed (in-place);
 * otherwise the buffers must not overlap and in is left unchanged. Enqueued on
 * `stream` (0 = the null stream); returns without waiting. A batch plan
 * (fftu_plan_batch) is refused with FFTU_ERROR_INVALID_VALUE here and in
 * fftu_execute_ws and the fftu_stage_* calls: it runs only through
 * fftu_execute_batch.
 */
fftu_status fftu_execute(fftu_plan_t plan, const void *in, void *out, hipStream_t stream);

/*
 * The transform of a real array (Section 6 names the real-to-complex FFT as the
 * method's next transform). X is real, n_1 x ... x n_d with n_d even; its
 * spectrum Y (eq. (1.2)) satisfies Y[-k] = conj Y[k], so the half k_d <= n_d/2
 * holds all of it. Layouts (h = n_d / 2, n' = (n_1, ..., n_{d-1}, h)):
 *   real side: the N reals of X as its packed complex view
 *     z[j', j] = X[j', 2j] + i X[j', 2j + 1] (shape n'), in the cyclic buffer
 *     layout above over the grid p, each element read as (re, im): N reals of the
 *     plan's precision (double for FFTU_C128, float for FFTU_C64). With
 *     p = (1, ..., 1) this is the row-major real array.
 *   complex side: the half spectrum Y[k', k], k < h (shape n', cyclic over p: the
 *     real side's layout), then the Nyquist plane Y[k', h] (shape n_1 x ... x
 *     n_{d-1}, cyclic over p_1 x ... x p_{d-1}; one element for d = 1):
 *     N/2 + N/n_d complex elements.
 * fftu_plan_real(d, n, p, dtype, FFTU_FORWARD) maps the real side to the complex
 * side (unnormalised); FFTU_INVERSE maps a complex side whose half spectrum
 * belongs to a real array back to the real side, times 1/N. Requirements: n_d
 * even, p_d | n_d/2 (else NOT_DIVISIBLE), and every requirement of fftu_plan for
 * the complex array n' over p (the transform runs the complex path on z, then one
 * pass that separates the even and odd halves of the last dimension; the inverse
 * runs that pass first). Execute with fftu_execute; in == out is allowed (the
 * buffer must hold the larger side), otherwise the buffers must not overlap.
 * fftu_execute_ws, fftu_execute_noalloc and the stage calls refuse real plans.
 */
fftu_plan_t fftu_plan_real(int d, const int64_t n[], const int64_t p[], fftu_dtype dtype, fftu_direction direction);

/*
 * The discrete cosine and sine transforms (Section 6 names the DCT and the DST as
 * the method's next transforms, built from 1-D algorithms dimension by dimension,
 * with the zig-zag cyclic distribution to exploit their symmetry). Per dimension of
 * length n (applied along every dimension):
 *   FFTU_DCT, FFTU_FORWARD (DCT-II):  y[k] = 2 sum_j x[j] cos(pi k (2j + 1) / (2n))
 *   FFTU_DST, FFTU_FORWARD (DST-II):  y[k] = 2 sum_j x[j] sin(pi (k + 1) (2j + 1) / (2n))
 *   FFTU_INVERSE: the exact inverse of the forward transform (DCT-III / DST-III
 *   times 1/n per dimension), so that inverse(forward(x)) = x.
 * Layouts (N reals of the plan's precision on each side, double for FFTU_C128 and
 * float for FFTU_C64):
 *   signal side (x): the zig-zag order v[m(j)] = x[j] along every dimension,
 *     m(j) = j/2 for even j and n - 1 - (j-1)/2 for odd j (even samples ascending,
 *     then odd samples descending), in the real side layout of fftu_plan_real over
 *     p. The DCT-II of x follows from the DFT of v alone, so this dealing of x
 *     (its zig-zag cyclic distribution) makes the reordering free.
 *   coefficient side (y): the cyclic buffer layout above over p.
 * FFTU_FORWARD maps the signal side to the coefficient side, FFTU_INVERSE back.
 * The transform runs fftu_plan_real's forward transform of v and one pass that
 * combines each index with its mirror images n_l - k_l; the inverse runs the
 * combining pass first. The DST is the DCT of the signal with the samples of odd
 * j negated (one more pass), stored at n_l - 1 - k_l.
 * Requirements: 1 <= d <= 4 and lcm(4 n_l) < 2^26 (the table of the combining pass;
 * else UNSUPPORTED), every n_l even (else INVALID_VALUE), and every requirement of
 * fftu_plan_real for v. Execute with
 * fftu_execute (in == out allowed; otherwise the buffers must not overlap);
 * fftu_execute_ws, fftu_execute_noalloc and the stage calls refuse these plans.
 * The plan owns a spectrum workspace of N/2 + N/n_d complex elements.
 */
typedef enum { FFTU_DCT = 0, FFTU_DST = 1 } fftu_r2r_kind;
fftu_plan_t fftu_plan_r2r(int d, const int64_t n[], const int64_t p[], fftu_dtype dtype, fftu_r2r_kind kind,
                          fftu_direction direction);

/*
 * Plans that own no device memory, for callers that manage HBM themselves (a
 * serving loop with its own arena). fftu_plan_external takes the same arguments
 * and applies the same checks as fftu_plan, but allocates nothing for the plan:
 * it uses a twiddle table shared by all external plans of the device and
 * precision (omega_{2^K}^j for the largest K needed so far, at least 2^12; the
 * first call, or one that needs a larger K, allocates and uploads that table,
 * which then stays until the process ends). Results are bitwise those of a
 * plan made by fftu_plan. fftu_plan_device_bytes of such a plan is 0.
 *
 * fftu_execute_ws runs the transform of any plan with the caller's workspace:
 * `workspace` is a device buffer of at least N elements of the plan's dtype
 * (workspace_bytes in fftu_plan_info), overlapping neither in nor out; it is
 * free again once the enqueued work has finished. fftu_execute on an external
 * plan returns FFTU_ERROR_INVALID_VALUE. Errors as for fftu_execute.
 */
fftu_plan_t fftu_plan_external(int d, const int64_t n[], const int64_t p[], fftu_dtype dtype,
                               fftu_direction direction);
fftu_status fftu_execute_ws(fftu_plan_t plan, const void *in, void *out, void *workspace, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under stream capture,
 * serving loops and harnesses that forbid hipMalloc): fftu_execute_ws with the
 * library's own fixed workspace, a device array of FFTU_NOALLOC_MAX_BYTES that
 * every device the library runs on holds from the time the library's code is
 * loaded there until the process ends. The call allocates nothing (the plan's
 * own workspace, if it has one, is not used); the caller passes the input and
 * output as for fftu_execute. Results are bitwise those of fftu_execute_ws.
 *
 * Requirements: the plan's device is the current device (else
 * FFTU_ERROR_INVALID_VALUE); N b <= FFTU_NOALLOC_MAX_BYTES, i.e. at most 4 Mi
 * complex128 or 8 Mi complex64 elements (else FFTU_ERROR_OUT_OF_MEMORY, before
 * anything is enqueued); not a batch plan (FFTU_ERROR_INVALID_VALUE). Buffer
 * rules and the other errors as for fftu_execute_ws.
 *
 * Concurrency: every call on one device uses that device's one array, which
 * keeps the last call's contents (nothing in it needs to start at zero). Calls
 * whose work overlaps on one device race and give wrong results: enqueue them
 * on one stream, or order them with events.
 */
#define FFTU_NOALLOC_MAX_BYTES (64u << 20)
fftu_status fftu_execute_noalloc(fftu_plan_t plan, const void *in, void *out, hipStream_t stream);

/*
 * The supersteps one at a time, for checking each against its definition.
 * All use the plan's direction for every weight and none applies 1/N.
 * Same buffer rules as fftu_execute, except fftu_stage_exchange, which needs
 * in != out.
 *
 *  local_fft:     Y^(s) = (F_{n_1/p_1} x ... x F_{n_d/p_d}) X^(s) for every s   (Superstep 0, first line)
 *  twiddle:       Z^(s)[k] = prod_l omega_{n_l}^{k_l s_l} Y^(s)[k]                (Superstep 0, loop)
 *  exchange:      W^(r)[s q + t] = Z^(s)[r + t p], q = n/p^2                     (Superstep 1, the Put)
 *  remaining_fft: V^(r)(t : q : n/p) = (F_{p_1} x ... x F_{p_d}) W^(r)(t : q : n/p)  (Superstep 2)
 */
fftu_status fftu_stage_local_fft(fftu_plan_t plan, const void *in, void *out, hipStream_t stream);
fftu_status fftu_stage_twiddle(fftu_plan_t plan, const void *in, void *out, hipStream_t stream);
fftu_status fftu_stage_exchange(fftu_plan_t plan, const void *in, void *out, hipStream_t stream);
fftu_status fftu_stage_remaining_fft(fftu_plan_t plan, const void *in, void *out, hipStream_t stream);

/*
 * The same for any plan, one step of one superstep at a time (the four calls
 * above refuse plans with several supersteps). With H = supersteps:
 *   part 0, phase c in [0, H]:  computation phase c's local FFTs (phase 0: every
 *            local F_{m_l}; later phases: the next level's F_{m_l} of dimensions
 *            with levels left, and the length-p_h FFTs of dimensions whose last
 *            Put was superstep c - 1, along the local index s' (n_h/p_h^2) + t)
 *   part 1, phase c in [0, H):  superstep c's twiddle omega_{n_i}^{u k} of each
 *            dimension's level c (u: member of the group, k: local index), in place
 *            of each element
 *   part 2, phase c in [0, H):  superstep c's Put (data movement only; in != out)
 * For H = 1 these are local_fft, twiddle, exchange and remaining_fft. Weights
 * follow the plan's direction; none applies 1/N. INVALID_VALUE for a phase or
 * part out of range, otherwise errors as for fftu_execute.
 */
fftu_status fftu_stage_superstep(fftu_plan_t plan, int phase, int part, const void *in, void *out, hipStream_t stream);

/*
 * Per-kernel timing on the execution stream. After fftu_timing_begin(plan, K),
 * each of the next K calls of fftu_execute on this plan records a HIP event
 * before its first kernel and after each kernel it launches (on the call's
 * stream). fftu_timing_end waits for those events, writes the mean duration in
 * milliseconds of each launch position (launch i of every recorded call) to
 * avg_ms[0 .. min(capacity, launches) - 1], sets *nkernels to the launches per
 * call and *ncalls to the calls recorded, and releases the events. The event
 * pool is created by fftu_timing_begin (host allocation and hipEventCreate);
 * calls beyond K are not recorded. Returns FFTU_ERROR_INVALID_VALUE without a
 * preceding fftu_timing_begin.
 */
fftu_status fftu_timing_begin(fftu_plan_t plan, int max_calls);
fftu_status fftu_timing_end(fftu_plan_t plan, float *avg_ms, int capacity, int *nkernels, int *ncalls);

/*
 * Batches (many independent transforms, uneven shapes, one persistent launch).
 *
 * fftu_plan_batch plans `count` transforms; transform i has d[i] dimensions,
 * sizes n[i][0..d[i]-1] and grid p[i][0..d[i]-1], each a separate instance of
 * Algorithm 2.3 with the buffer layout described above. All share dtype and
 * direction. Supported members: every local length n_l/p_l <= 256 with local
 * size M >= 2, and a grid whose length-p transforms fit one thread's registers
 * (at most 16 complex128 / 32 complex64 points, equal sides); others give
 * FFTU_ERROR_UNSUPPORTED. The plan owns one twiddle table, a workspace of
 * sum_i N_i elements and the work list in device memory.
 *
 * fftu_execute_batch runs every transform: out[i] = F(in[i]); in and out are
 * host arrays of `count` device pointers, each aligned to the element size.
 * in[i] == out[i] is allowed; otherwise in[i] and out[i] must not overlap, and
 * no out[i] may overlap another transform's input or output
 * (FFTU_ERROR_INVALID_VALUE, checked on the host before anything is enqueued).
 * The pointers are read by the persistent kernel from a small device array of
 * the plan. When they differ from the previous call's, the call first enqueues
 * one small kernel per 96 transforms on `stream` that writes the new pointers
 * there (the pointers travel as kernel arguments), so the call never waits for
 * the host or the device and never allocates. It then enqueues a counter reset
 * and the persistent kernel, and returns. As for every plan, one stream at a
 * time may execute it.
 *
 * fftu_batch_error reports (after waiting for the device) whether the last
 * batch on this plan hit its bounded dependency wait (1) or not (0).
 */
fftu_plan_t fftu_plan_batch(int count, const int d[], const int64_t *const n[], const int64_t *const p[],
                            fftu_dtype dtype, fftu_direction direction);
fftu_status fftu_execute_batch(fftu_plan_t plan, const void *const in[], void *const out[], hipStream_t stream);
fftu_status fftu_batch_error(fftu_plan_t plan, int *flag);

/*
 * Batches that own no device memory, for callers that manage HBM themselves (a
 * serving loop that coalesces waiting requests into one launch, with its own
 * arena). fftu_plan_batch_external takes the arguments of fftu_plan_batch and
 * applies its checks, builds the work list on the host only and uses the twiddle
 * table shared with fftu_plan_external plans (allocated on first use, as there).
 * Its results are bitwise those of fftu_plan_batch for the same members.
 *
 * fftu_batch_workspace_bytes: device bytes one execution needs (the members'
 * workspaces, the work list, its counters and buffer array).
 * fftu_batch_staging_bytes: host bytes of the work-list image a call writes.
 *
 * fftu_execute_batch_ws runs every transform as fftu_execute_batch does, with
 * `workspace` (device, 256-byte aligned, at least fftu_batch_workspace_bytes,
 * overlapping no buffer) and `host_staging` (page-locked host memory from
 * hipHostMalloc, at least fftu_batch_staging_bytes). The call writes the work
 * list for these buffers into host_staging, enqueues its copy into the workspace,
 * the counter reset and the persistent kernel on `stream`, and returns without
 * waiting. The caller must leave host_staging unchanged until the enqueued copy
 * has run (an event recorded after the call marks it), and the workspace until
 * the batch has finished. fftu_execute_batch and fftu_graph_capture refuse such
 * plans (INVALID_VALUE); fftu_batch_error reads the flag of the last call's
 * workspace. Errors as for fftu_execute_batch.
 */
fftu_plan_t fftu_plan_batch_external(int count, const int d[], const int64_t *const n[], const int64_t *const p[],
                                     fftu_dtype dtype, fftu_direction direction);
size_t fftu_batch_workspace_bytes(fftu_plan_t plan);
size_t fftu_batch_staging_bytes(fftu_plan_t plan);
fftu_status fftu_execute_batch_ws(fftu_plan_t plan, const void *const in[], void *const out[], void *workspace,
                                  void *host_staging, hipStream_t stream);

/*
 * HIP graphs: fftu_graph_capture records the launches of one fftu_execute
 * (count = 0, in/out point at one device pointer each) or one
 * fftu_execute_batch (count = the batch size, in/out arrays of count device
 * pointers) on a private stream and instantiates them. fftu_graph_launch
 * replays the graph on `stream`; the buffers are the ones given at capture,
 * whatever the plan ran on in between (a batch graph rewrites the plan's
 * pointer array as its first step). A graph replay counts as an execution of
 * its plan: one stream at a time. The graph refers to the plan, which must
 * outlive it. Buffer checks as for the execution it records. NULL on failure.
 */
typedef struct fftu_graph_s *fftu_graph_t;
fftu_graph_t fftu_graph_capture(fftu_plan_t plan, int count, const void *const in[], void *const out[]);
fftu_status fftu_graph_launch(fftu_graph_t graph, hipStream_t stream);
void fftu_graph_destroy(fftu_graph_t graph);

/*
 * Circular convolution in the cyclic layout (the transform starts and ends in
 * the same distribution, so a product of spectra needs no reordering):
 *   out = F^{-1}( F(in) . filter_hat ),
 * i.e. out[j] = sum_k in[k] h[(j - k) mod n] per dimension when filter_hat =
 * F(h) (unnormalised forward transform, as fftu_execute of this plan computes).
 *
 * fftu_plan_convolution makes a forward plan of the given shape (it owns the
 * table and an N-element workspace and may be passed to fftu_execute, e.g. to
 * transform the filter once) together with an inverse plan that shares the
 * workspace. fftu_execute_convolution enqueues the forward transform of `in`
 * with the product by `filter_hat` fused into its exchange (when the exchange is
 * fused; otherwise one pointwise pass follows), then the inverse transform, in
 * place on `out`. in == out allowed; filter_hat (N elements, cyclic layout, the
 * plan's dtype) must not overlap out. Errors as for fftu_execute, and
 * INVALID_VALUE for a plan not made by fftu_plan_convolution.
 *
 * fftu_pointwise_mul: out[i] = a[i] b[i] scale for i < count, complex elements
 * of `dtype`; out may alias a or b. Asynchronous on `stream`.
 */
fftu_plan_t fftu_plan_convolution(int d, const int64_t n[], const int64_t p[], fftu_dtype dtype);
fftu_status fftu_execute_convolution(fftu_plan_t plan, const void *in, const void *filter_hat, void *out,
                                     hipStream_t stream);
fftu_status fftu_pointwise_mul(const void *a, const void *b, void *out, int64_t count, fftu_dtype dtype, double scale,
                               hipStream_t stream);

/*
 * Seeded device input (used by the serving layer to generate request data next
 * to the transform instead of copying it over PCIe).
 *
 * fftu_fill_uniform writes `count` complex elements of `dtype` to the device
 * buffer `out` (interleaved re, im; the caller owns it): element e is
 * Philox4x32-10 (Salmon et al., SC'11: 10 rounds, multipliers 0xD2511F53 and
 * 0xCD9E8D57, key increments 0x9E3779B9 and 0xBB67AE85) of the counter
 * (c mod 2^32, c div 2^32, 0, 0), c = counter_base + e, under the key
 * (key0, key1), with the output words x0..x3 mapped exactly into [-1, 1):
 *   FFTU_C64:  re = (x0 >> 8) 2^-23 - 1,  im = (x1 >> 8) 2^-23 - 1
 *   FFTU_C128: re = (x0 2^21 + (x1 >> 11)) 2^-52 - 1,
 *              im = (x2 2^21 + (x3 >> 11)) 2^-52 - 1
 * so a host implementation of the same definition reproduces it bit for bit.
 * Asynchronous on `stream`. count == 0 does nothing. Errors: INVALID_VALUE
 * (NULL out with count > 0, count < 0, bad dtype), DEVICE.
 */
fftu_status fftu_fill_uniform(void *out, int64_t count, fftu_dtype dtype, uint32_t key0, uint32_t key1,
                              uint64_t counter_base, hipStream_t stream);

/* Release a plan and its device memory. NULL is ignored. The caller must make
 * sure no enqueued work still uses the plan. */
void fftu_destroy(fftu_plan_t plan);

#ifdef __cplusplus
}
#endif

#endif /* FFTU_H */
