// Device helpers shared by the factor and solve kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include "../tasks.hpp"

namespace d3m {

template <typename T> struct C2T;
template <> struct C2T<double> { using type = double2; };
template <> struct C2T<float> { using type = float2; };
template <typename T2> struct T2S;
template <> struct T2S<double2> { using type = double; };
template <> struct T2S<float2> { using type = float; };

__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2(v.x, v.y); }
template <typename T2> __device__ __forceinline__ T2 from_d2(double2 v);
template <> __device__ __forceinline__ double2 from_d2<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ float2 from_d2<float2>(double2 v) { return make_float2((float)v.x, (float)v.y); }

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a - b*c
__device__ __forceinline__ double2 cfms(double2 a, double2 b, double2 c) {
    return make_double2(a.x - (b.x * c.x - b.y * c.y), a.y - (b.x * c.y + b.y * c.x));
}
// a - b*c with fused multiply-adds
__device__ __forceinline__ double2 cfma_neg(double2 a, double2 b, double2 c) {
    return make_double2(fma(-b.x, c.x, fma(b.y, c.y, a.x)), fma(-b.x, c.y, fma(-b.y, c.x, a.y)));
}
// 1/z from the definition conj(z)/|z|^2.  z is first scaled by a power of
// two that brings its larger component near 1 (exact, no overflow in |z|^2);
// 1/|z|^2 is the hardware reciprocal estimate refined by two Newton-Raphson
// steps r <- r + r (1 - d r) (each roughly doubles the correct bits).  A zero
// or non-finite z gives a non-finite result, as the division would.
__device__ __forceinline__ double2 crecip(double2 z) {
    const double m = fmax(fabs(z.x), fabs(z.y));
    const int e = m > 0.0 && m <= 1.7e308 ? __builtin_amdgcn_frexp_exp(m) : 0;
    const double xr = ldexp(z.x, -e), xi = ldexp(z.y, -e);
    const double d = fma(xr, xr, xi * xi);
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    if (!(m > 0.0)) r = 1.0 / d;  // keeps the non-finite result of a zero pivot
    return make_double2(ldexp(xr * r, -e), -ldexp(xi * r, -e));
}
__device__ __forceinline__ double cabs1(double2 z) { return fabs(z.x) + fabs(z.y); }


// Real MFMA products used by the complex tile kernels (three real products
// per complex one in the factor kernels and the FP64 solve: P1 = Re a Re b,
// P2 = Im a Im b, P3 = (Re a + Im a)(Re b + Im b), Re = P1 - P2,
// Im = P3 - P1 - P2; four in the FP32 solve).
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// Operand layout of the 16x16x4 products: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16].  Accumulator layout (lane l, register r holds
// D[row][l % 16]): f64 row = l/16 + 4r, f32 row = 4(l/16) + r.
template <> struct Mfma<double> {
    using acc = d4_t;
    __device__ __forceinline__ static int out_row(int lk, int r) { return lk + 4 * r; }
    __device__ __forceinline__ static acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<float> {
    using acc = f4_t;
    __device__ __forceinline__ static int out_row(int lk, int r) { return 4 * lk + r; }
    __device__ __forceinline__ static acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

// Work-groups are dealt to the 8 XCDs round-robin (group g runs on XCD g % 8),
// each with its own L2.  Task lists are ordered so that neighbouring tasks
// share operand tiles (same subdomain and block column), so XCD x is given
// the contiguous range of tasks [x * per, (x + 1) * per): g -> (g % 8) * per
// + g / 8.  The grid is 8 * per groups; the few beyond ntask exit at once.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_task(int64_t ntask) {
    const int64_t per = (ntask + kXcds - 1) / kXcds;
    return (int64_t)(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
}

template <typename T2> __device__ __forceinline__ T2 *enc_ptr(const Bases &b, int64_t e) {
    return reinterpret_cast<T2 *>(b.p[e >> ENC_SHIFT]) + (e & ENC_MASK);
}

}  // namespace d3m
