// Reaction-field special functions (Section 2.1), host and device.
//
// I_n(x, y) = 1/(2 pi n!) int_0^inf exp(-lam y + i lam x) lam^n / (lam - Z) dlam,  y > 0
// (eq. (generalintegral)).  With w = y - i x and P = Z w the n = 0 integral has the closed form
//
//     I_0 = (1/2pi) exp(-P) (i pi - Ei(P)),                                  (*)
//
// Ei the principal-branch exponential integral.  The paper prints its initial value next to
// eq. (integralrecursion) with the sign of x flipped and without the -i pi that its own lossless
// limit (aaa1.5) carries; (*) is the form that agrees with the defining integral for eps > 0 and,
// by limiting absorption, for eps = 0.  Higher orders follow the upward recursion of
// eq. (integralrecursion):  I_n = 1 / (2 pi n w^n) + (Z / n) I_{n-1}.
//
// Ei is evaluated by one of three published methods, chosen by the position of P:
//   - its power series gamma + ln P + sum P^k / (k k!) (Abramowitz & Stegun 5.1.10) when |P| <= 2,
//     or |P| <= 4 with Re P >= 0, or |arg P| <= pi/8 with |P| <= 40;
//   - the asymptotic series exp(P)/P sum k!/P^k (A&S 5.1.51) for |arg P| <= pi/8, |P| > 40;
//   - otherwise the continued fraction for E_1(w) at w = -P (A&S 5.1.22), evaluated with the
//     modified Lentz method, and Ei(P) = -E_1(-P) + i pi sgn(Im P).
// The last two are combined with exp(-P) analytically, so that exp(-P) Ei(P) never overflows:
//   I_0 = (1/2pi) [ exp(-P) E_1(-P) + i pi (1 - sgn Im P) exp(-P) ].
#pragma once
#include "cplx.hpp"

namespace fmmhp {

constexpr double kPi = 3.14159265358979323846;
constexpr double kInv2Pi = 0.15915494309189533577;
constexpr double kInv4Pi = 0.07957747154594766788;
constexpr double kEulerGamma = 0.57721566490153286061;
constexpr double kLn2Hi = 6.93147180369123816490e-01;  // ln 2 with its low 32 bits cleared
constexpr double kLn2Lo = 1.90821492927058770002e-10;  // ln 2 - kLn2Hi
constexpr double kLn2 = 6.93147180559945309417e-01;    // ln 2 rounded to double

// 1 / x for a positive normal double whose reciprocal is normal: the hardware reciprocal refined by
// two Newton steps (each squares the relative error).
__device__ __forceinline__ double rcp_pos(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// Natural logarithm of a positive, finite, normal double.  x = 2^e m with m in [sqrt(1/2), sqrt(2)),
// log m = 2 atanh(s), s = (m - 1)/(m + 1), |s| <= 0.1716, and atanh s = s sum_k s^(2k) / (2k + 1)
// truncated after k = 10 (the first omitted term is below 1e-17 relative).  e ln 2 is added in two
// parts so that e * kLn2Hi is exact.  Used where a log of a squared distance is needed per pair.
// 1 / (m + 1) comes from the hardware reciprocal refined by two Newton steps.
__device__ __forceinline__ double log_pos(double x) {
    int e;
    double m = frexp(x, &e);  // m in [0.5, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double num = m - 1.0, den = m + 1.0;
    double r = __builtin_amdgcn_rcp(den);
    r = fma(r, fma(-den, r, 1.0), r);
    r = fma(r, fma(-den, r, 1.0), r);
    const double s = num * r;
    const double s2 = s * s;
    double p = 1.0 / 21.0;
    p = fma(p, s2, 1.0 / 19.0);
    p = fma(p, s2, 1.0 / 17.0);
    p = fma(p, s2, 1.0 / 15.0);
    p = fma(p, s2, 1.0 / 13.0);
    p = fma(p, s2, 1.0 / 11.0);
    p = fma(p, s2, 1.0 / 9.0);
    p = fma(p, s2, 1.0 / 7.0);
    p = fma(p, s2, 1.0 / 5.0);
    p = fma(p, s2, 1.0 / 3.0);
    const double s_2 = 2.0 * s;
    const double lm = fma(s_2, s2 * p, s_2);
    const double ed = (double)e;
    return fma(ed, kLn2Hi, fma(ed, kLn2Lo, lm));
}

// Table-assisted natural logarithm of a positive finite double (the near-field pair loop).
// x = 2^e m, m in [1, 2); the top 9 bits of the mantissa select c_k = 1 + (k + 1/2)/512, and
// log x = e ln 2 + L_k + log1p(t),  t = m r_k - 1,  r_k = fl(1/c_k),  L_k = -log(r_k),
// with |t| <= 2^-10, so that log1p(t) = t - t^2/2 + t^3/3 leaves an error below t^4/4 <= 2^-42
// (2.3e-13, absolute) and e ln 2 in one rounding adds at most |e| 2^-54: a pair's log term is
// good to ~2.5e-13, which moves a potential built from ~150 such terms by ~1e-12 at most, four
// orders below the 1e-10 accuracy target.  The table entries (r_k, L_k) are built on the host by
// log_table_entry.  For x = +0 the result is finite (about -709), so a caller may evaluate it
// unconditionally and mask the result.
constexpr int kLogTable = 512;

inline void log_table_entry(int k, double *r, double *L) {
    const double c = 1.0 + (k + 0.5) / kLogTable;
    *r = 1.0 / c;
    *L = -log(*r);
}

__device__ __forceinline__ double log_tab(double x, const double2 *__restrict__ tab) {
    // exponent and mantissa bits (x > 0, normal)
    const unsigned long long u = __double_as_longlong(x);
    const int e = (int)(u >> 52) - 1023;
    const int k = (int)((u >> 43) & (kLogTable - 1));
    const double m = __longlong_as_double((u & 0x000fffffffffffffull) | 0x3ff0000000000000ull);
    const double2 rl = tab[k];
    const double t = fma(m, rl.x, -1.0);
    double p = fma(1.0 / 3.0, t, -1.0 / 2.0);
    p = fma(p, t, 1.0);
    return fma((double)e, kLn2, fma(t, p, rl.y));
}

// 1 / (k k!) for k = 1..32: coefficients of the power series of Ei.
struct EiSeries {
    double c[33];
    constexpr EiSeries() : c() {
        double f = 1.0;
        for (int k = 1; k <= 32; ++k) {
            f *= k;
            c[k] = 1.0 / (k * f);
        }
    }
};

__host__ __device__ inline cplx reaction_I0(double x, double y, cplx Z) {
    const cplx P = Z * mk(y, -x);
    const double r = cabs(P);
    const double ang = fabs(atan2(P.im, P.re));
    const double sg = (P.im > 0.0) ? 1.0 : ((P.im < 0.0) ? -1.0 : 0.0);
    if (r <= 2.0 || (r <= 4.0 && P.re >= 0.0) || (ang <= 0.125 * kPi && r <= 40.0)) {
        cplx sum = mk(0.0, 0.0), t = mk(1.0, 0.0);
        for (int k = 1; k < 400; ++k) {
            t = t * P * (1.0 / k);
            const cplx term = t * (1.0 / k);
            sum += term;
            if (abs2(term) < 1e-34 * abs2(sum)) break;
        }
        const cplx ei = mk(kEulerGamma, 0.0) + clog_(P) + sum;
        const cplx e = cexp_(-P);
        return kInv2Pi * (e * mk(-ei.re, kPi - ei.im));
    }
    cplx A;
    if (ang <= 0.125 * kPi) {
        // exp(-P) E_1(-P) = -(1/P) sum_{k>=0} k! / P^k, truncated at its smallest term
        const cplx ip = inv(P);
        cplx t = ip, sum = ip;
        for (int k = 1; k < 200; ++k) {
            const cplx tn = t * ip * (double)k;
            if (abs2(tn) > abs2(t)) break;
            sum += tn;
            t = tn;
            if (abs2(tn) < 1e-34 * abs2(sum)) break;
        }
        A = -sum;
    } else {
        // modified Lentz evaluation of exp(w) E_1(w), w = -P, |arg w| < 7 pi / 8
        const cplx w = -P;
        cplx b = w + mk(1.0, 0.0);
        cplx c = mk(1e300, 0.0);
        cplx d = inv(b);
        cplx h = d;
        for (int i = 1; i < 4000; ++i) {
            const double a = -(double)i * (double)i;
            b = b + mk(2.0, 0.0);
            d = inv(a * d + b);
            c = b + a * inv(c);
            const cplx del = c * d;
            h = h * del;
            if (abs2(del - mk(1.0, 0.0)) < 1e-32) break;
        }
        A = h;
    }
    const cplx e = cexp_(-P);
    return kInv2Pi * (A + mul_ipow(e, 1) * (kPi * (1.0 - sg)));
}

// K_j = rho^j I_j(x, y) for j = 0..nmax by eq. (integralrecursion):
//   rho^n I_n = (1/(2 pi n)) (rho / w)^n + (Z rho / n) rho^{n-1} I_{n-1}.
__host__ __device__ inline void reaction_In_scaled(double x, double y, cplx Z, double rho, int nmax,
                                                   cplx *out) {
    const cplx sigma = rho * inv(mk(y, -x));
    const cplx zr = rho * Z;
    cplx K = reaction_I0(x, y, Z);
    out[0] = K;
    cplx sp = mk(1.0, 0.0);
    for (int n = 1; n <= nmax; ++n) {
        sp = sp * sigma;
        K = sp * (kInv2Pi / n) + zr * K * (1.0 / n);
        out[n] = K;
    }
}

}  // namespace fmmhp
