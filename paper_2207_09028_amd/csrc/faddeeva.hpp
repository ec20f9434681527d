// Faddeeva function w(z) = exp(-z^2) erfc(-iz) for Im z >= 0, in FP64.
//
// Method: J. A. C. Weideman, "Computation of the complex error function",
// SIAM J. Numer. Anal. 31 (1994) 1497-1518.  With L = (N / sqrt 2)^(1/2) and the
// Moebius variable Z = (L + iz) / (L - iz),
//
//   w(z) = 2 p(Z) / (L - iz)^2 + 1 / (sqrt(pi) (L - iz)),   p(Z) = sum_{n<N} a_{n+1} Z^n,
//
// where a_n are the Fourier coefficients of f(theta) = exp(-t^2) (L^2 + t^2),
// t = L tan(theta / 2), sampled at 4N points on (-pi, pi].  The coefficients are
// generated here at compile time from that definition.  N = 40 gives a relative
// error near 1e-14 over the region the truncated long-range kernel uses.
#pragma once

#include "common.hpp"

namespace occrik {
namespace fad {

constexpr int kN = 40;
constexpr double kPi = 3.14159265358979323846264338327950288;

// compile-time elementary functions (Taylor series after range reduction)
constexpr double ct_sin(double x) {      // |x| <= pi
    double term = x, sum = x;
    for (int n = 1; n < 30; ++n) {
        term *= -x * x / double((2 * n) * (2 * n + 1));
        sum += term;
    }
    return sum;
}
constexpr double ct_cos(double x) {      // |x| <= pi
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 30; ++n) {
        term *= -x * x / double((2 * n - 1) * (2 * n));
        sum += term;
    }
    return sum;
}
constexpr double ct_exp_neg(double y) {   // exp(-y), y >= 0
    if (y > 745.0) return 0.0;
    // exp(-y) = exp(-y / 2^k)^(2^k) with y / 2^k <= 1/2
    int k = 0;
    double r = y;
    while (r > 0.5) {
        r *= 0.5;
        ++k;
    }
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 25; ++n) {
        term *= -r / double(n);
        sum += term;
    }
    for (int i = 0; i < k; ++i) sum *= sum;
    return sum;
}
constexpr double ct_sqrt(double x) {
    if (x <= 0.0) return 0.0;
    double g = x > 1.0 ? x : 1.0;
    for (int i = 0; i < 100; ++i) g = 0.5 * (g + x / g);
    return g;
}

struct Coefficients {
    double L;
    double a[kN];                         // a_1 .. a_N
    constexpr Coefficients() : L(0.0), a() {
        constexpr int M = 2 * kN;         // samples theta_j = j pi / M, j = -M+1 .. M-1, plus theta = -pi
        L = ct_sqrt(double(kN) / ct_sqrt(2.0));
        double f[2 * M] = {};
        for (int j = -M + 1; j <= M - 1; ++j) {
            const double half = 0.5 * j * kPi / M;            // theta / 2 in (-pi/2, pi/2)
            const double t = L * ct_sin(half) / ct_cos(half);
            f[j + M] = ct_exp_neg(t * t) * (L * L + t * t);
        }
        f[0] = 0.0;                                           // theta = -pi: t infinite, f = 0
        // f is even in theta: a_n = (1 / 2M) sum_j f_j cos(n theta_j)
        for (int n = 1; n <= kN; ++n) {
            double s = 0.0;
            for (int j = -M + 1; j <= M - 1; ++j) {
                // n j pi / M reduced to (-pi, pi]
                long e = (long(n) * j) % (2 * M);
                if (e > M) e -= 2 * M;
                if (e <= -M) e += 2 * M;
                s += f[j + M] * ct_cos(double(e) * kPi / M);
            }
            a[n - 1] = s / (2.0 * M);
        }
    }
};

// w(x + i y), y >= 0
__host__ __device__ inline void faddeeva(double x, double y, double& wr, double& wi) {
    constexpr Coefficients C{};
    const double L = C.L;
    // L - iz = (L + y) - i x ;  L + iz = (L - y) + i x
    const double dr = L + y, di = -x;
    const double nr = L - y, ni = x;
    const double den = dr * dr + di * di;
    const double Zr = (nr * dr + ni * di) / den, Zi = (ni * dr - nr * di) / den;
    double pr = 0.0, pi = 0.0;
    for (int n = kN - 1; n >= 0; --n) {      // Horner: p = p Z + a_{n+1}
        const double tr = pr * Zr - pi * Zi + C.a[n];
        pi = pr * Zi + pi * Zr;
        pr = tr;
    }
    // 1 / (L - iz) and its square
    const double ir = dr / den, ii = -di / den;
    const double sr = ir * ir - ii * ii, si = 2.0 * ir * ii;
    constexpr double inv_sqrt_pi = 0.56418958354775628694807945156077259;
    wr = 2.0 * (pr * sr - pi * si) + inv_sqrt_pi * ir;
    wi = 2.0 * (pr * si + pi * sr) + inv_sqrt_pi * ii;
}

}  // namespace fad
}  // namespace occrik
