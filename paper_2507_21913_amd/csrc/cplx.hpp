// Minimal complex float64 arithmetic usable from host and device code.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace fmmhp {

struct cplx {
    double re, im;
};

__host__ __device__ __forceinline__ cplx mk(double r, double i) { return cplx{r, i}; }
__host__ __device__ __forceinline__ cplx operator+(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__host__ __device__ __forceinline__ cplx operator-(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__host__ __device__ __forceinline__ cplx operator-(cplx a) { return {-a.re, -a.im}; }
// Products of two terms are written with one explicit fused multiply-add each: left to the
// compiler, which of the two products gets fused can differ between copies of the same code (a loop
// unrolled for one charge vector, rolled for eight), and with it the rounding.
__host__ __device__ __forceinline__ cplx operator*(cplx a, cplx b) {
    return {fma(a.re, b.re, -(a.im * b.im)), fma(a.re, b.im, a.im * b.re)};
}
__host__ __device__ __forceinline__ cplx operator*(double s, cplx a) { return {s * a.re, s * a.im}; }
__host__ __device__ __forceinline__ cplx operator*(cplx a, double s) { return {s * a.re, s * a.im}; }
__host__ __device__ __forceinline__ cplx& operator+=(cplx& a, cplx b) { a.re += b.re; a.im += b.im; return a; }
__host__ __device__ __forceinline__ cplx& operator-=(cplx& a, cplx b) { a.re -= b.re; a.im -= b.im; return a; }
__host__ __device__ __forceinline__ cplx conj(cplx a) { return {a.re, -a.im}; }
__host__ __device__ __forceinline__ double abs2(cplx a) { return fma(a.re, a.re, a.im * a.im); }
__host__ __device__ __forceinline__ double cabs(cplx a) { return hypot(a.re, a.im); }
__host__ __device__ __forceinline__ cplx inv(cplx a) {
    // 1/a with scaling to avoid overflow/underflow of |a|^2
    double s = fmax(fabs(a.re), fabs(a.im));
    double r = a.re / s, i = a.im / s;
    double d = s * fma(r, r, i * i);
    return {r / d, -i / d};
}
__host__ __device__ __forceinline__ cplx operator/(cplx a, cplx b) { return a * inv(b); }
__host__ __device__ __forceinline__ cplx cexp_(cplx a) {
    double e = exp(a.re);
    double s, c;
    sincos(a.im, &s, &c);
    return {e * c, e * s};
}
__host__ __device__ __forceinline__ cplx clog_(cplx a) { return {log(cabs(a)), atan2(a.im, a.re)}; }
// acc += a * b with four fused multiply-adds
__host__ __device__ __forceinline__ void cfma(cplx &acc, cplx a, cplx b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
}
// multiply by i^k
__host__ __device__ __forceinline__ cplx mul_ipow(cplx a, int k) {
    switch (k & 3) {
        case 0: return a;
        case 1: return {-a.im, a.re};
        case 2: return {-a.re, -a.im};
        default: return {a.im, -a.re};
    }
}

}  // namespace fmmhp
