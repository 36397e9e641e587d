// Device-side building blocks shared by the QDS kernels: complex arithmetic,
// plane addressing, the mode convolution C_m and the counter-based noise.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define QDS_MAX_MODES 8

namespace qds {

template <typename T>
struct cx {
    T re, im;
};

template <typename T> __device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T> __device__ __forceinline__ cx<T> zero() { return cx<T>{T(0), T(0)}; }
template <typename T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a) { return {-a.re, -a.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
// i * s * a  (multiplication by an imaginary number i s)
template <typename T> __device__ __forceinline__ cx<T> imul(T s, cx<T> a) { return {-s * a.im, s * a.re}; }
// a * conj(b)
template <typename T> __device__ __forceinline__ cx<T> mulc(cx<T> a, cx<T> b) {
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// conj(a) * b
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}

// Vector load/store of one complex element (16 B for double, 8 B for float).
// Every state plane lives in device (global) memory: the accesses go through
// the global address space, so that pointers read from argument tables in
// memory still give global (not flat) instructions.
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const v2d g_cv2d;
typedef __attribute__((address_space(1))) v2d g_v2d;
typedef __attribute__((address_space(1))) const v2f g_cv2f;
typedef __attribute__((address_space(1))) v2f g_v2f;

__device__ __forceinline__ cx<double> ld(const cx<double>* p) {
    const v2d v = *(g_cv2d*)(p);
    return {v.x, v.y};
}
__device__ __forceinline__ cx<float> ld(const cx<float>* p) {
    const v2f v = *(g_cv2f*)(p);
    return {v.x, v.y};
}
__device__ __forceinline__ void st(cx<double>* p, cx<double> a) {
    v2d v;
    v.x = a.re;
    v.y = a.im;
    *(g_v2d*)(p) = v;
}
__device__ __forceinline__ void st(cx<float>* p, cx<float> a) {
    v2f v;
    v.x = a.re;
    v.y = a.im;
    *(g_v2f*)(p) = v;
}
// Streaming store (the non-temporal hint of a vector store): the line is not
// kept in the caches for reuse.
__device__ __forceinline__ void st_nt(cx<double>* p, cx<double> a) {
    v2d v;
    v.x = a.re;
    v.y = a.im;
    __builtin_nontemporal_store(v, (g_v2d*)(p));
}
__device__ __forceinline__ void st_nt(cx<float>* p, cx<float> a) {
    v2f v;
    v.x = a.re;
    v.y = a.im;
    __builtin_nontemporal_store(v, (g_v2f*)(p));
}

// Value held by the next lane of the wavefront (DPP wave shift; lane 63
// receives zero).  Call it with every lane active: a lane masked off by a
// branch supplies zero.
__device__ __forceinline__ double next_lane(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float next_lane(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}
template <typename T>
__device__ __forceinline__ cx<T> next_lane(cx<T> v) {
    return cx<T>{next_lane(v.re), next_lane(v.im)};
}

// Mode convolution C_m{A, B} (the azimuthal projection of a product of two
// real fields, Eqs. source_mode_zero / source_mode_m): with a_k = A^(k) for
// k = 0 and A^(k)/2, conj(A^(k))/2 for +-k, the mode-m coefficient of AB is
// P^(0) = sum_k a_k b_-k and P^(m) = 2 sum_{k+l=m} a_k b_l.  Written out:
//   m = 0: A0 B0 + 1/2 sum_{k>0} Re(A_k conj(B_k))
//   m > 0: 1/2 [ sum_{k+l=m} A_k B_l + sum_{k-l=m} A_k conj(B_l) + sum_{l-k=m} conj(A_k) B_l ]
template <typename T, int M>
__device__ __forceinline__ void conv_acc(const cx<T>* A, const cx<T>* B, T sign, cx<T>* out) {
    {
        cx<T> s = A[0] * B[0];
        T re = T(0);
#pragma unroll
        for (int k = 1; k < M; ++k) re += A[k].re * B[k].re + A[k].im * B[k].im;
        s.re += T(0.5) * re;
        out[0] = out[0] + sign * s;
    }
#pragma unroll
    for (int m = 1; m < M; ++m) {
        cx<T> acc = zero<T>();
#pragma unroll
        for (int k = 0; k <= m; ++k) acc = acc + A[k] * B[m - k];
#pragma unroll
        for (int l = 0; l + m < M; ++l) acc = acc + mulc(A[l + m], B[l]);
#pragma unroll
        for (int k = 0; k + m < M; ++k) acc = acc + cmul(A[k], B[k + m]);
        out[m] = out[m] + (sign * T(0.5)) * acc;
    }
}

template <typename T, int M>
__device__ __forceinline__ void conv_one(const cx<T>* A, const cx<T>* B, int m, cx<T>& out, T sign) {
    // C_m{A, B} for the single output mode m (see conv_acc).  m is a run-time
    // value (the mode of the calling wave): every array index below is a
    // compile-time constant so that A and B stay in registers.
    cx<T> acc = zero<T>();
    if (m == 0) {
        acc = A[0] * B[0];
        T re = T(0);
#pragma unroll
        for (int k = 1; k < M; ++k) re += A[k].re * B[k].re + A[k].im * B[k].im;
        acc.re += T(0.5) * re;
        out = out + sign * acc;
        return;
    }
#pragma unroll
    for (int k = 0; k < M; ++k) {
#pragma unroll
        for (int l = 0; l < M; ++l) {
            if (k + l == m) acc = acc + A[k] * B[l];
            if (k - l == m) acc = acc + mulc(A[k], B[l]);
            if (l - k == m) acc = acc + cmul(A[k], B[l]);
        }
    }
    out = out + (sign * T(0.5)) * acc;
}

// The same C_m{A, B} with the factors of every mode held elsewhere (LDS):
// fa(k), fb(k) return mode k of the two factors.  Each A_k is loaded once and
// its partners B_{m-k}, B_{k-m}, B_{k+m} as they are needed, so many modes do
// not keep both arrays in registers.
template <typename T, int M, typename FA, typename FB>
__device__ __forceinline__ void conv_stream(FA fa, FB fb, int m, cx<T>& out, T sign) {
    cx<T> acc = zero<T>();
    if (m == 0) {
        acc = fa(0) * fb(0);
        T re = T(0);
#pragma unroll
        for (int k = 1; k < M; ++k) {
            const cx<T> a = fa(k), b = fb(k);
            re += a.re * b.re + a.im * b.im;
        }
        acc.re += T(0.5) * re;
        out = out + sign * acc;
        return;
    }
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const cx<T> a = fa(k);
        if (m - k >= 0) acc = acc + a * fb(m - k);
        if (k - m >= 0) acc = acc + mulc(a, fb(k - m));
        if (k + m < M) acc = acc + cmul(a, fb(k + m));
    }
    out = out + (sign * T(0.5)) * acc;
}

// out += sign C_m{F_fa, F_fb} for factors read through get(f, k) (factor f of
// mode k at this lane): register arrays up to four modes, streamed above that.
template <typename T, int M, typename G>
__device__ __forceinline__ void conv_pair(G get, int fa, int fb, int m, cx<T>& out, T sign) {
    if constexpr (M <= 4) {
        cx<T> A[M], B[M];
#pragma unroll
        for (int k = 0; k < M; ++k) {
            A[k] = get(fa, k);
            B[k] = get(fb, k);
        }
        conv_one<T, M>(A, B, m, out, sign);
    } else {
        conv_stream<T, M>([&](int k) { return get(fa, k); }, [&](int k) { return get(fb, k); }, m, out, sign);
    }
}

// SplitMix64 (Steele, Lea & Flood 2014): output k >= 1 of the stream seeded
// with ``seed`` is mix(seed + k * 0x9E3779B97F4A7C15).  Box-Muller normal from
// outputs 2c+1, 2c+2 of counter c = (step << 32) | (lab column << 12) | row.
__device__ __forceinline__ uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ double normal_ctr(uint64_t seed, uint64_t c) {
    const uint64_t g = 0x9E3779B97F4A7C15ull;
    uint64_t z1 = sm64_mix(seed + (2 * c + 1) * g);
    uint64_t z2 = sm64_mix(seed + (2 * c + 2) * g);
    double u1 = (double((z1 >> 11)) + 1.0) * 0x1.0p-53;
    double u2 = double(z2 >> 11) * 0x1.0p-53;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

}  // namespace qds
