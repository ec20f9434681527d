// Register-resident line FFTs: two lanes per line, one lane exchange per transform.
//
// A line of N = 2H points is held by a lane pair (s = lane & 1), H points each.
//
//   forward_dit  in:  lane s holds x[2a + s], a < H                (interleaved)
//                out: lane s holds X[s H/2 + m] in slot m and
//                     X[H + s H/2 + m] in slot H/2 + m, m < H/2   (blocked)
//   inverse_dif  in:  blocked (as above), out: interleaved
//
// (any direction of either form is available through DIR).  Decimation in time:
// y_s = DFT_H(x_s), y_1 *= w_N^k, then X[k] = y_0[k] + y_1[k] and
// X[k + H] = y_0[k] - y_1[k] with lane 0 keeping k < H/2 and lane 1 the rest,
// which needs H/2 values from the partner lane.  Decimation in frequency is the
// mirror image: u_c[a] = (x[a] + (-1)^c x[a + H]) w_N^{ac} formed locally, lane
// c gathers u_c for every a (H/2 values from the partner) and X[2k + c] =
// DFT_H(u_c)[k].  H must be even.  The H-point DFTs are mixed-radix
// Cooley-Tukey in registers with twiddles fixed at compile time (FP64
// constants rounded once to the working precision).
#pragma once

#include "common.hpp"

namespace occrik {

// ---------------------------------------------------------------------------
// compile-time twiddles
// ---------------------------------------------------------------------------
constexpr double kPiD = 3.14159265358979323846264338327950288;

constexpr double ct_sin_reduced(double x) {      // |x| <= pi
    double term = x, sum = x;
    const double x2 = x * x;
    for (int n = 1; n < 30; ++n) {
        term *= -x2 / double((2 * n) * (2 * n + 1));
        sum += term;
    }
    return sum;
}
constexpr double ct_cos_reduced(double x) {      // |x| <= pi
    double term = 1.0, sum = 1.0;
    const double x2 = x * x;
    for (int n = 1; n < 30; ++n) {
        term *= -x2 / double((2 * n - 1) * (2 * n));
        sum += term;
    }
    return sum;
}

// w_N^e = exp(DIR 2 pi i e / N), returned as (re, im)
struct TwPair {
    double re, im;
};
constexpr TwPair ct_twiddle(int e, int n, int dir) {
    int t = e % n;
    if (t < 0) t += n;
    // exact values on the axes and diagonals keep trivial factors exact
    if (t == 0) return {1.0, 0.0};
    if (4 * t == n) return {0.0, double(dir)};
    if (2 * t == n) return {-1.0, 0.0};
    if (4 * t == 3 * n) return {0.0, -double(dir)};
    double ang = 2.0 * kPiD * double(t) / double(n);
    if (ang > kPiD) ang -= 2.0 * kPiD;
    return {ct_cos_reduced(ang), double(dir) * ct_sin_reduced(ang)};
}

template <int N, int DIR>
struct TwTable {
    TwPair v[N > 0 ? N : 1];
    constexpr TwTable() : v() {
        for (int e = 0; e < N; ++e) v[e] = ct_twiddle(e, N, DIR);
    }
};

// a * (wr + i wi) for a compile-time twiddle; the trivial ones (+-1, +-i) cost
// no multiplies (without fast-math the compiler cannot drop x * 0 by itself)
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cmul_c(cplx<T> a, double wr, double wi) {
    cplx<T> o;
    if (wi == 0.0 && wr == 1.0) return a;
    if (wi == 0.0 && wr == -1.0) {
        o.x = -a.x; o.y = -a.y;
        return o;
    }
    if (wr == 0.0 && wi == 1.0) {
        o.x = -a.y; o.y = a.x;
        return o;
    }
    if (wr == 0.0 && wi == -1.0) {
        o.x = a.y; o.y = -a.x;
        return o;
    }
    const T r = T(wr), i = T(wi);
    o.x = a.x * r - a.y * i;
    o.y = a.x * i + a.y * r;
    return o;
}

// ---------------------------------------------------------------------------
// host/device leaf DFTs
// ---------------------------------------------------------------------------
template <typename T, int R, int DIR>
__host__ __device__ __forceinline__ void leaf_dft(cplx<T>* v) {
    if constexpr (R == 2) {
        const cplx<T> a = v[0], b = v[1];
        v[0].x = a.x + b.x; v[0].y = a.y + b.y;
        v[1].x = a.x - b.x; v[1].y = a.y - b.y;
    } else if constexpr (R == 4) {
        const T ax = v[0].x + v[2].x, ay = v[0].y + v[2].y;
        const T bx = v[0].x - v[2].x, by = v[0].y - v[2].y;
        const T cx = v[1].x + v[3].x, cy = v[1].y + v[3].y;
        T dx = v[1].x - v[3].x, dy = v[1].y - v[3].y;
        // d *= DIR i
        const T tx = DIR < 0 ? dy : -dy, ty = DIR < 0 ? -dx : dx;
        dx = tx; dy = ty;
        v[0].x = ax + cx; v[0].y = ay + cy;
        v[2].x = ax - cx; v[2].y = ay - cy;
        v[1].x = bx + dx; v[1].y = by + dy;
        v[3].x = bx - dx; v[3].y = by - dy;
    } else if constexpr (R == 3) {
        // X0 = x0 + t1, X1,2 = (x0 - t1/2) +- i DIR sin(2 pi/3) (x1 - x2), t1 = x1 + x2
        constexpr double c = 0.86602540378443864676372317075293618 * DIR;
        const T t1x = v[1].x + v[2].x, t1y = v[1].y + v[2].y;
        const T t2x = v[1].x - v[2].x, t2y = v[1].y - v[2].y;
        const T mx = v[0].x - T(0.5) * t1x, my = v[0].y - T(0.5) * t1y;
        v[0].x = v[0].x + t1x; v[0].y = v[0].y + t1y;
        v[1].x = mx - T(c) * t2y; v[1].y = my + T(c) * t2x;
        v[2].x = mx + T(c) * t2y; v[2].y = my - T(c) * t2x;
    } else {
        static_assert(R == 5, "leaf radices are 2, 3, 4 and 5");
        // pairs (1, 4) and (2, 3): cosines on the sums, DIR i sines on the differences
        constexpr double c1 = 0.30901699437494742410229341718281906;    // cos(2 pi/5)
        constexpr double c2 = -0.80901699437494742410229341718281906;   // cos(4 pi/5)
        constexpr double s1 = 0.95105651629515357211643933337938214 * DIR;   // sin(2 pi/5)
        constexpr double s2 = 0.58778525229247312916870595463907277 * DIR;   // sin(4 pi/5)
        const T t1x = v[1].x + v[4].x, t1y = v[1].y + v[4].y;
        const T t2x = v[2].x + v[3].x, t2y = v[2].y + v[3].y;
        const T t3x = v[1].x - v[4].x, t3y = v[1].y - v[4].y;
        const T t4x = v[2].x - v[3].x, t4y = v[2].y - v[3].y;
        const T a1x = v[0].x + T(c1) * t1x + T(c2) * t2x, a1y = v[0].y + T(c1) * t1y + T(c2) * t2y;
        const T a2x = v[0].x + T(c2) * t1x + T(c1) * t2x, a2y = v[0].y + T(c2) * t1y + T(c1) * t2y;
        const T b1x = T(s1) * t3x + T(s2) * t4x, b1y = T(s1) * t3y + T(s2) * t4y;
        const T b2x = T(s2) * t3x - T(s1) * t4x, b2y = T(s2) * t3y - T(s1) * t4y;
        v[0].x = v[0].x + t1x + t2x; v[0].y = v[0].y + t1y + t2y;
        v[1].x = a1x - b1y; v[1].y = a1y + b1x;      // a1 + i b1
        v[4].x = a1x + b1y; v[4].y = a1y - b1x;      // a1 - i b1
        v[2].x = a2x - b2y; v[2].y = a2y + b2x;
        v[3].x = a2x + b2y; v[3].y = a2y - b2x;
    }
}

template <int H> struct RegSplit;   // H = P * Q, first radix P (a leaf), Q handled recursively
#define OCCRIK_REGSPLIT(H_, P_) \
    template <> struct RegSplit<H_> { static constexpr int P = P_; };
OCCRIK_REGSPLIT(2, 2)
OCCRIK_REGSPLIT(3, 3)
OCCRIK_REGSPLIT(4, 4)
OCCRIK_REGSPLIT(5, 5)
OCCRIK_REGSPLIT(6, 3)
OCCRIK_REGSPLIT(8, 4)
OCCRIK_REGSPLIT(9, 3)
OCCRIK_REGSPLIT(10, 5)
OCCRIK_REGSPLIT(12, 4)
OCCRIK_REGSPLIT(15, 5)
OCCRIK_REGSPLIT(16, 4)
OCCRIK_REGSPLIT(18, 3)
OCCRIK_REGSPLIT(20, 4)
OCCRIK_REGSPLIT(24, 4)
OCCRIK_REGSPLIT(25, 5)
OCCRIK_REGSPLIT(27, 3)
OCCRIK_REGSPLIT(30, 5)
OCCRIK_REGSPLIT(32, 4)
#undef OCCRIK_REGSPLIT

// In-place H-point DFT of x[0..H) in natural order:
// X[k1 + P k2] = sum_{n2 < Q} w_H^{n2 k1} [sum_{n1 < P} x[Q n1 + n2] w_P^{n1 k1}] w_Q^{n2 k2}
template <typename T, int H, int DIR>
__host__ __device__ __forceinline__ void reg_dft(cplx<T>* x) {
    constexpr int P = RegSplit<H>::P;
    if constexpr (P == H) {
        leaf_dft<T, H, DIR>(x);
    } else {
        constexpr int Q = H / P;
        constexpr TwTable<H, DIR> tw{};
        cplx<T> t[Q][P];
#pragma unroll
        for (int n2 = 0; n2 < Q; ++n2) {
            cplx<T> g[P];
#pragma unroll
            for (int n1 = 0; n1 < P; ++n1) g[n1] = x[Q * n1 + n2];
            leaf_dft<T, P, DIR>(g);
#pragma unroll
            for (int k1 = 0; k1 < P; ++k1) {
                const int e = n2 * k1;
                t[n2][k1] = e == 0 ? g[k1] : cmul_c<T>(g[k1], tw.v[e % H].re, tw.v[e % H].im);
            }
        }
#pragma unroll
        for (int k1 = 0; k1 < P; ++k1) {
            cplx<T> h[Q];
#pragma unroll
            for (int n2 = 0; n2 < Q; ++n2) h[n2] = t[n2][k1];
            reg_dft<T, Q, DIR>(h);
#pragma unroll
            for (int k2 = 0; k2 < Q; ++k2) x[k1 + P * k2] = h[k2];
        }
    }
}

// ---------------------------------------------------------------------------
// two-lane line transforms, split into local steps around the lane exchange so
// that the host can run both lanes of a pair to check the arithmetic
// ---------------------------------------------------------------------------
// DIT, local part: x holds x[2a + s]; afterwards x holds the H/2 values to keep
// (first half of the slots) and the H/2 values to send (second half).
template <typename T, int N, int DIR>
__host__ __device__ __forceinline__ void dit_local(cplx<T>* x, int s) {
    constexpr int H = N / 2;
    constexpr TwTable<N, DIR> tw{};
    reg_dft<T, H, DIR>(x);
    if (s) {
#pragma unroll
        for (int k = 1; k < H; ++k) x[k] = cmul_c<T>(x[k], tw.v[k].re, tw.v[k].im);
        // lane 1 keeps k >= H/2 and sends k < H/2: swap the halves
#pragma unroll
        for (int m = 0; m < H / 2; ++m) {
            const cplx<T> a = x[m];
            x[m] = x[H / 2 + m];
            x[H / 2 + m] = a;
        }
    }
}
// DIT, combine: keep[m] = own y_s, recv[m] = partner's y_{1-s} at the same k.
template <typename T, int N>
__host__ __device__ __forceinline__ void dit_combine(cplx<T>* x, const cplx<T>* recv, int s) {
    constexpr int H = N / 2;
#pragma unroll
    for (int m = 0; m < H / 2; ++m) {
        const cplx<T> own = x[m];
        const cplx<T> y0 = s ? recv[m] : own, y1 = s ? own : recv[m];
        x[m].x = y0.x + y1.x; x[m].y = y0.y + y1.y;
        x[H / 2 + m].x = y0.x - y1.x; x[H / 2 + m].y = y0.y - y1.y;
    }
}
// DIF, local part: x holds the blocked values of lane s (slot m: index
// s H/2 + m, slot H/2 + m: index H + s H/2 + m).  Forms u_0, u_1 at the lane's
// H/2 indices a; afterwards slots [0, H/2) hold u_s (kept) and [H/2, H) hold
// u_{1-s} (sent).
template <typename T, int N, int DIR>
__host__ __device__ __forceinline__ void dif_local(cplx<T>* x, int s) {
    constexpr int H = N / 2;
    constexpr TwTable<N, DIR> tw{};
#pragma unroll
    for (int m = 0; m < H / 2; ++m) {
        const cplx<T> lo = x[m], hi = x[H / 2 + m];
        cplx<T> u0, u1;
        u0.x = lo.x + hi.x; u0.y = lo.y + hi.y;
        u1.x = lo.x - hi.x; u1.y = lo.y - hi.y;
        const int a = s * (H / 2) + m;
        if (a != 0) u1 = cmul_c<T>(u1, tw.v[a].re, tw.v[a].im);
        x[m] = s ? u1 : u0;
        x[H / 2 + m] = s ? u0 : u1;
    }
}
// DIF, combine: own u_s at indices of this lane, recv u_s at the partner's
// indices; assemble u_s over all a (lane 0 owns a < H/2) and transform.
template <typename T, int N, int DIR>
__host__ __device__ __forceinline__ void dif_combine(cplx<T>* x, const cplx<T>* recv, int s) {
    constexpr int H = N / 2;
    cplx<T> u[H];
#pragma unroll
    for (int m = 0; m < H / 2; ++m) {
        u[m] = s ? recv[m] : x[m];
        u[H / 2 + m] = s ? x[m] : recv[m];
    }
    reg_dft<T, H, DIR>(u);
#pragma unroll
    for (int k = 0; k < H; ++k) x[k] = u[k];
}

// interleaved -> blocked, and blocked -> interleaved, for the lane pair that
// holds the line (device only: the lane exchange is a DPP move)
template <typename T, int N, int DIR>
__device__ void line_dit(cplx<T>* x, int s);
template <typename T, int N, int DIR>
__device__ void line_dif(cplx<T>* x, int s);

#if defined(__HIP_DEVICE_COMPILE__)
// exchange with lane ^ 1 (DPP quad permutation [1, 0, 3, 2])
__device__ __forceinline__ float lane_swap(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double lane_swap(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0xB1, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename T, int N>
__device__ __forceinline__ void exchange_half(cplx<T>* x, cplx<T>* recv) {
    constexpr int H = N / 2;
#pragma unroll
    for (int m = 0; m < H / 2; ++m) {
        recv[m].x = lane_swap(x[H / 2 + m].x);
        recv[m].y = lane_swap(x[H / 2 + m].y);
    }
}

template <typename T, int N, int DIR>
__device__ __forceinline__ void line_dit(cplx<T>* x, int s) {
    constexpr int H = N / 2;
    cplx<T> recv[H / 2];
    dit_local<T, N, DIR>(x, s);
    exchange_half<T, N>(x, recv);
    dit_combine<T, N>(x, recv, s);
}
template <typename T, int N, int DIR>
__device__ __forceinline__ void line_dif(cplx<T>* x, int s) {
    constexpr int H = N / 2;
    cplx<T> recv[H / 2];
    dif_local<T, N, DIR>(x, s);
    exchange_half<T, N>(x, recv);
    dif_combine<T, N, DIR>(x, recv, s);
}
#endif

// index along the line of slot m of lane s in the blocked layout
__host__ __device__ constexpr int blocked_index(int m, int s, int h) {
    return m < h / 2 ? s * (h / 2) + m : h + s * (h / 2) + (m - h / 2);
}

}  // namespace occrik
