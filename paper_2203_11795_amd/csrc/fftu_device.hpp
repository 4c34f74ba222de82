// Device helpers shared by the kernels: interleaved complex type, complex
// arithmetic, exact constant roots of unity up to order 32, and in-register DFTs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

#include "fftu_internal.hpp"

namespace fftu {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> conj_if(cx<T> a, int c) { return c ? cx<T>{a.x, -a.y} : a; }

// cos(2 pi j / 32) for j = 0..8; every 32nd root of unity follows by symmetry.
__host__ __device__ constexpr double cos32_octant(int j)
{
    return j == 0 ? 1.0
         : j == 1 ? 0.98078528040323044912618223613424
         : j == 2 ? 0.92387953251128675612818318939679
         : j == 3 ? 0.83146961230254523707878837761791
         : j == 4 ? 0.70710678118654752440084436210485
         : j == 5 ? 0.55557023301960222474283081394853
         : j == 6 ? 0.38268343236508977172845998403040
         : j == 7 ? 0.19509032201612826784828486847702
                  : 0.0;
}
__host__ __device__ constexpr double cos32(int j)
{
    j = ((j % 32) + 32) % 32;
    return j <= 8 ? cos32_octant(j) : j <= 16 ? -cos32_octant(16 - j) : j <= 24 ? -cos32_octant(j - 16)
                                                                          : cos32_octant(32 - j);
}
__host__ __device__ constexpr double sin32(int j) { return cos32(j - 8); }

// a * omega_R^K with omega_R = exp(-2 pi i / R), R | 32; the quarter turns are exact.
template <typename T, int R, int K>
__device__ __forceinline__ cx<T> mul_root(cx<T> a)
{
    constexpr int k = ((K % R) + R) % R;
    if constexpr (k == 0) {
        return a;
    } else if constexpr (4 * k == R) {
        return {a.y, -a.x};
    } else if constexpr (2 * k == R) {
        return {-a.x, -a.y};
    } else if constexpr (4 * k == 3 * R) {
        return {-a.y, a.x};
    } else {
        constexpr int j = k * (32 / R);
        constexpr T c = static_cast<T>(cos32(j));
        constexpr T s = static_cast<T>(-sin32(j));
        return cmul(a, cx<T>{c, s});
    }
}

// In-register DFT of length R (power of two <= 32), natural order in and out:
// radix-2 decimation in time, recursively.
template <typename T, int R>
struct Dft {
    template <int... K>
    static __device__ __forceinline__ void combine(cx<T> *v, const cx<T> *e, const cx<T> *o,
                                                   std::integer_sequence<int, K...>)
    {
        ((v[K] = e[K] + mul_root<T, R, K>(o[K]), v[K + R / 2] = e[K] - mul_root<T, R, K>(o[K])), ...);
    }
    static __device__ __forceinline__ void run(cx<T> *v)
    {
        cx<T> e[R / 2], o[R / 2];
#pragma unroll
        for (int k = 0; k < R / 2; ++k) {
            e[k] = v[2 * k];
            o[k] = v[2 * k + 1];
        }
        Dft<T, R / 2>::run(e);
        Dft<T, R / 2>::run(o);
        combine(v, e, o, std::make_integer_sequence<int, R / 2>{});
    }
};
template <typename T>
struct Dft<T, 2> {
    static __device__ __forceinline__ void run(cx<T> *v)
    {
        cx<T> a = v[0], b = v[1];
        v[0] = a + b;
        v[1] = a - b;
    }
};
template <typename T>
struct Dft<T, 1> {
    static __device__ __forceinline__ void run(cx<T> *) {}
};

// Compile-time radix plan of a line of 2^LOGL split over TPL = L / E threads with
// E = 2^LOGE_ elements each (by default k_line's, see line_stages_of / line_loge in
// fftu_internal.hpp; k_lastx may hold more). Register m of thread j holds line
// position j + TPL m before the first and after the last stage. Stage s has radix
// 2^lr(s) (the last one may be smaller) and follows Ns = 2^lns(s) points.
template <int LOGL, int LOGE_ = line_loge(LOGL)>
struct LinePlan {
    static constexpr int NS = LOGE_ == line_loge(LOGL) ? line_stages_of(LOGL) : (LOGL + LOGE_ - 1) / LOGE_;
    static constexpr int LOGE = LOGE_;
    static constexpr int E = 1 << LOGE;
    static constexpr int LOGTPL = LOGL - LOGE;
    static constexpr int TPL = 1 << LOGTPL;
    static constexpr int L = 1 << LOGL;
    static constexpr int lr(int s) { return s < NS - 1 ? LOGE : LOGL - (NS - 1) * LOGE; }
    static constexpr int lns(int s) { return s * LOGE; }
};

// Radix stage S on the thread's registers (register m <-> position j + TPL m).
template <typename T, int LOGL, int S, int LOGE = line_loge(LOGL)>
__device__ __forceinline__ void line_compute(cx<T> (&v)[1 << LOGE], int j, const cx<T> *tw)
{
    using PL = LinePlan<LOGL, LOGE>;
    constexpr int LR = PL::lr(S), R = 1 << LR, LNS = PL::lns(S), NB = PL::E / R;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        cx<T> x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = v[c + r * NB];
        if constexpr (S > 0) {
            const int jm = (j + c * PL::TPL) & ((1 << LNS) - 1);
#pragma unroll
            for (int r = 1; r < R; ++r) x[r] = cmul(x[r], tw[(r * jm) << (LOGL - LNS - LR)]);
        }
        Dft<T, R>::run(x);
#pragma unroll
        for (int r = 0; r < R; ++r) v[c + r * NB] = x[r];
    }
}

// Load of one element of a pass's input. Each pass streams its array through
// once, so the load is non-temporal (the caches need not keep the line); this
// measured several per cent faster per pass than plain loads. CO: a plain load
// (the persistent batch kernel reads what other workgroups wrote).
template <bool CO = false, typename T>
__device__ __forceinline__ cx<T> get(const cx<T> *p)
{
    if constexpr (CO) {
        return *p;
    } else {
        typedef T v2 __attribute__((ext_vector_type(2)));
        const v2 r = __builtin_nontemporal_load(reinterpret_cast<const v2 *>(p));
        return cx<T>{r.x, r.y};
    }
}

// Workgroup barrier that orders LDS only: this wave's LDS accesses complete before
// the barrier and later ones start after it, while global loads stay in flight
// (__syncthreads() also waits for every outstanding global access).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Store of one element: non-temporal, as get(). With CO (device-coherent), the
// store is a device-scope relaxed atomic instead: it is written through to the
// level that every workgroup of the device reads from, so that once the storing
// thread has waited for its stores to complete, other workgroups (on any XCD)
// can read the value after an acquire, with no write-back of the storing XCD's
// L2. complex128 goes as two 8-byte halves.
template <bool CO, typename T>
__device__ __forceinline__ void put(cx<T> *p, const cx<T> &v)
{
    if constexpr (!CO) {
        typedef T v2 __attribute__((ext_vector_type(2)));
        const v2 val = {v.x, v.y};
        __builtin_nontemporal_store(val, reinterpret_cast<v2 *>(p));
    } else if constexpr (sizeof(T) == 4) {
        uint64_t u;
        __builtin_memcpy(&u, &v, 8);
        __hip_atomic_store(reinterpret_cast<uint64_t *>(p), u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        uint64_t u0, u1;
        __builtin_memcpy(&u0, &v.x, 8);
        __builtin_memcpy(&u1, &v.y, 8);
        uint64_t *q = reinterpret_cast<uint64_t *>(p);
        __hip_atomic_store(q, u0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(q + 1, u1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace fftu
