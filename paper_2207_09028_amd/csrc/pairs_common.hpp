// Device helpers shared by the pair-pass kernels (LDS Stockham and register forms).
#pragma once

#include "faddeeva.hpp"
#include "fft.hpp"
#include "internal.hpp"

namespace occrik {
namespace pairs {

template <typename T>
__device__ inline void load_twiddles(cplx<T>* dst, const cplx<T>* src) {
    for (int t = threadIdx.x; t < 3 * kMaxN; t += blockDim.x) dst[t] = src[t];
}

__device__ inline int freq(int t, int n) { return (t < (n + 1) / 2) ? t : t - n; }

__device__ inline void kfrac_of(int idx, int M1, int M2, int M3, double* f) {
    const int k3 = idx % M3;
    const int k2 = (idx / M3) % M2;
    const int k1 = idx / (M2 * M3);
    f[0] = double(k1) / M1;
    f[1] = double(k2) / M2;
    f[2] = double(k3) / M3;
}

// f(x) at x^2 = x2 (paper eq. recipcoul) with this build's x = 0 rule.
template <typename T>
__device__ inline T kernel_f(T x2, int kind, T omega) {
    if (kind == OCCRIK_KERNEL_COULOMB) {
        return x2 == T(0) ? T(0) : T(12.566370614359172953850573533118) / x2;
    } else if (kind == OCCRIK_KERNEL_ERF_LR) {
        return x2 == T(0) ? T(0) : T(12.566370614359172953850573533118) / x2 * exp(-x2 / (T(4) * omega * omega));
    } else {
        return x2 == T(0) ? T(3.1415926535897932384626433832795) / (omega * omega)
                          : T(12.566370614359172953850573533118) / x2 * (-expm1(-x2 / (T(4) * omega * omega)));
    }
}

template <typename T>
__device__ inline T kernel_dfdw(T x2, int kind, T omega) {
    const T w3 = omega * omega * omega;
    if (kind == OCCRIK_KERNEL_ERF_LR) {
        return x2 == T(0) ? T(0) : T(6.283185307179586476925286766559) / w3 * exp(-x2 / (T(4) * omega * omega));
    } else if (kind == OCCRIK_KERNEL_ERFC_SR) {
        return x2 == T(0) ? -T(6.283185307179586476925286766559) / w3
                          : -T(6.283185307179586476925286766559) / w3 * exp(-x2 / (T(4) * omega * omega));
    }
    return T(0);
}

template <typename T>
struct Recip {
    T b[9];
};

// truncated Coulomb, 4 pi / x^2 (1 - cos(x R_c)) as 8 pi sin^2(x R_c / 2) / x^2, in FP64:
// x R_c reaches a few hundred radians on fine grids, beyond what FP32 phases resolve
__device__ inline double trunc_coulomb(double x2, double rcut) {
    if (x2 == 0.0) return 6.283185307179586476925286766559 * rcut * rcut;
    const double sn = sin(0.5 * sqrt(x2) * rcut);
    return 25.132741228718345907701147066236 * sn * sn / x2;
}

template <typename T>
__device__ inline T momentum_sq(const Recip<T>& rc, double q0, double q1, double q2, int m1, int m2, int m3) {
    const T a = T(m1 + q0), b = T(m2 + q1), c = T(m3 + q2);
    const T gx = a * rc.b[0] + b * rc.b[3] + c * rc.b[6];
    const T gy = a * rc.b[1] + b * rc.b[4] + c * rc.b[7];
    const T gz = a * rc.b[2] + b * rc.b[5] + c * rc.b[8];
    return gx * gx + gy * gy + gz * gz;
}

// truncated long range (erf(w r)/r cut off at R_c), and its omega derivative, in FP64:
//   f   = 4 pi / x^2 [e^{-x^2/4w^2} - erf(w R) cos(x R) - e^{-w^2 R^2} Re(e^{-ixR} w(z))]
//   df  = -(8 sqrt(pi) / x) I'(x),  I = sqrt(pi)/(2w) [e^{-x^2/4w^2} - e^{-w^2 R^2} Re(e^{-ixR} w(z))]
// with z = -x/(2w) + i w R and w(z) the Faddeeva function (w' = -2 z w + 2i/sqrt(pi))
__device__ inline double trunc_erf_lr(double x2, double om, double rcut, bool deriv) {
    constexpr double kPi = 3.14159265358979323846264338327950288;
    constexpr double kSqrtPi = 1.77245385090551602729816748334114518;
    const double wr2 = om * om * rcut * rcut;
    if (x2 == 0.0) {
        if (deriv)
            return 8.0 * kSqrtPi * (kSqrtPi * erf(om * rcut) / (4.0 * om * om * om) -
                                    rcut * exp(-wr2) / (2.0 * om * om));
        return 4.0 * kPi * ((0.5 * rcut * rcut - 0.25 / (om * om)) * erf(om * rcut) +
                            rcut * exp(-wr2) / (2.0 * om * kSqrtPi));
    }
    const double x = sqrt(x2);
    const double zr = -x / (2.0 * om), zi = om * rcut;
    double fr, fi;
    fad::faddeeva(zr, zi, fr, fi);
    double sn, cs;
    sincos(x * rcut, &sn, &cs);                 // e^{-ixR} = cs - i sn
    const double g = exp(-x2 / (4.0 * om * om));
    const double ew = exp(-wr2);
    if (!deriv) {
        const double re = cs * fr + sn * fi;    // Re(e^{-ixR} w)
        return 4.0 * kPi / x2 * (g - erf(om * rcut) * cs - ew * re);
    }
    // d/dx [e^{-ixR} w(z)] = e^{-ixR} (-iR w + w'(z) (-1 / 2w))
    const double dwr = -2.0 * (zr * fr - zi * fi), dwi = -2.0 * (zr * fi + zi * fr) + 2.0 / kSqrtPi;
    const double ur = rcut * fi - dwr / (2.0 * om);          // -iR w - w'/(2w), real part
    const double ui = -rcut * fr - dwi / (2.0 * om);         //                   imaginary part
    const double dre = cs * ur + sn * ui;                    // Re(e^{-ixR} u)
    const double dI = kSqrtPi / (2.0 * om) * (-(x / (2.0 * om * om)) * g - ew * dre);
    return -8.0 * kSqrtPi / x * dI;
}

// f (or df/domega when deriv) at G_m + q, m = (m1, m2, m3) as signed frequencies
template <typename T>
__device__ inline T kernel_at(const PairBatch& B, const Recip<T>& rc, double q0, double q1, double q2, int m1, int m2,
                              int m3, bool deriv, T om) {
    if (B.kernel == OCCRIK_KERNEL_TRUNC_COULOMB || B.kernel == OCCRIK_KERNEL_TRUNC_ERF_LR) {
        if (deriv && B.kernel == OCCRIK_KERNEL_TRUNC_COULOMB) return T(0);
        const double a = m1 + q0, b = m2 + q1, c = m3 + q2;
        const double gx = a * B.recip[0] + b * B.recip[3] + c * B.recip[6];
        const double gy = a * B.recip[1] + b * B.recip[4] + c * B.recip[7];
        const double gz = a * B.recip[2] + b * B.recip[5] + c * B.recip[8];
        const double x2 = gx * gx + gy * gy + gz * gz;
        if (B.kernel == OCCRIK_KERNEL_TRUNC_COULOMB) return T(trunc_coulomb(x2, B.rcut));
        return T(trunc_erf_lr(x2, B.omega, B.rcut, deriv));
    }
    const T x2 = momentum_sq<T>(rc, q0, q1, q2, m1, m2, m3);
    if (x2 == T(0) && B.madelung &&
        (B.kernel == OCCRIK_KERNEL_COULOMB || B.kernel == OCCRIK_KERNEL_ERF_LR)) {
        // Madelung mode at G + q = 0 (q = 0 exactly when k_b = k_a)
        constexpr double kPi = 3.14159265358979323846264338327950288;
        const double w = B.omega;
        if (B.kernel == OCCRIK_KERNEL_COULOMB) return deriv ? T(0) : T(B.g0);
        return deriv ? T(2.0 * kPi / (w * w * w)) : T(B.g0 - kPi / (w * w));
    }
    return deriv ? kernel_dfdw<T>(x2, B.kernel, om) : kernel_f<T>(x2, B.kernel, om);
}

// Table block of summed k-point b in the batch's kernel values: (b - b0) for a
// per-batch table, or with the plan's cache the index of the difference k_a - k_b
// (each component in [-(M - 1), M - 1], row-major over the three directions).
__device__ inline int kv_block(const PairBatch& B, int b) {
    if (!B.kcache) return b - B.b0;
    const int a3 = B.a % B.M3, a2 = (B.a / B.M3) % B.M2, a1 = B.a / (B.M2 * B.M3);
    const int b3 = b % B.M3, b2 = (b / B.M3) % B.M2, b1 = b / (B.M2 * B.M3);
    return ((a1 - b1 + B.M1 - 1) * (2 * B.M2 - 1) + (a2 - b2 + B.M2 - 1)) * (2 * B.M3 - 1) + (a3 - b3 + B.M3 - 1);
}

// f (or df/domega) at grid index (i1, i2, i3) for momentum q (fractional), with the
// Nyquist-plane mean of the symmetric mode
template <typename T>
__device__ inline T kernel_value(const PairBatch& B, const Recip<T>& rc, double q0, double q1, double q2, int i1,
                                 int i2, int i3, bool deriv, T om) {
    const int N1 = B.N1, N2 = B.N2, N3 = B.N3;
    const int m1 = freq(i1, N1), m2 = freq(i2, N2), m3 = freq(i3, N3);
    T f = kernel_at<T>(B, rc, q0, q1, q2, m1, m2, m3, deriv, om);
    if (B.nyquist == OCCRIK_NYQUIST_SYMMETRIC && ((2 * m1 == -N1) || (2 * m2 == -N2) || (2 * m3 == -N3))) {
        const int mm1 = (2 * m1 == -N1) ? -m1 : m1;
        const int mm2 = (2 * m2 == -N2) ? -m2 : m2;
        const int mm3 = (2 * m3 == -N3) ? -m3 : m3;
        f = T(0.5) * (f + kernel_at<T>(B, rc, q0, q1, q2, mm1, mm2, mm3, deriv, om));
    }
    return f;
}

// Sizes: compile-time when NN > 0 (cubic NN^3 grid), else taken from the batch.
template <int NN>
struct Dims {
    int n1, n2, n3;
    __device__ explicit Dims(const PairBatch& B)
        : n1(NN ? NN : B.N1), n2(NN ? NN : B.N2), n3(NN ? NN : B.N3) {}
};

template <typename T, int NN, int DIR>
__device__ __forceinline__ void lines(int n, cplx<T>* buf, int count, int es, int ls, const cplx<T>* tw) {
    if constexpr (NN > 0) fft_lines<T, NN, DIR, NN>(buf, count, es, ls, tw);
    else fft_lines_n<T, DIR>(n, buf, count, es, ls, tw);
}

// index of the stored pair (i, j), i <= j, of a diagonal block: rows of the upper triangle
__device__ inline int tri_index(int i, int j, int nocc) { return i * nocc - (i * (i - 1)) / 2 + (j - i); }

// Stored pair slot -> (b, i, j).
__device__ inline void decode_slot(const PairBatch& B, int slot, int& b, int& i, int& j) {
    const int nn = B.nocc * B.nout;
    if (B.diag && slot < B.ntri) {
        int r = 0;
        while (r + 1 < B.nocc && tri_index(r + 1, r + 1, B.nocc) <= slot) ++r;
        b = B.a;
        i = r;
        j = r + (slot - tri_index(r, r, B.nocc));
        return;
    }
    const int s = slot - (B.diag ? B.ntri : 0);
    const int blk = s / nn;
    const int rem = s - blk * nn;
    b = B.b0 + (B.diag ? 1 : 0) + blk;
    i = rem / B.nout;
    j = rem - i * B.nout;
}


}  // namespace pairs
}  // namespace occrik
