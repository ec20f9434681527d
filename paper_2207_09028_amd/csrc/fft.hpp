// Batched 1D FFTs of a 2D tile held in LDS (self-sorting mixed-radix Stockham).
//
// A tile of `lines` lines of length N sits in LDS; element e of line l is at
// buf[l * ls + e * es].  Every stage reads each point once into registers,
// synchronises the workgroup, applies twiddles and a radix-R DFT in registers
// and writes each point once, so one LDS buffer suffices.  The transform is
// unnormalised: DIR = -1 computes X_m = sum_n x_n e^{-2 pi i m n / N}, DIR = +1
// the same with e^{+...}.  Output is in natural order.
//
// Twiddles come from an LDS table tw[t] = e^{-2 pi i t / N}, t in [0, N),
// computed in FP64 on the host and rounded once to the working precision.
#pragma once

#include "common.hpp"

namespace occrik {

// ---------------------------------------------------------------------------
// in-register DFTs of size R (R in {2, 3, 4, 5, 6, 8})
// ---------------------------------------------------------------------------
template <typename T, int R, int DIR> struct Dft;

template <typename T, int DIR> struct Dft<T, 2, DIR> {
    static __device__ __forceinline__ void run(cplx<T>* v) {
        cplx<T> a = v[0], b = v[1];
        v[0] = cadd<T>(a, b);
        v[1] = csub<T>(a, b);
    }
};

template <typename T, int DIR> struct Dft<T, 3, DIR> {
    static __device__ __forceinline__ void run(cplx<T>* v) {
        const T c = T(-0.5);
        const T s = T(0.86602540378443864676372317075294);
        cplx<T> t = cadd<T>(v[1], v[2]);
        cplx<T> u = csub<T>(v[1], v[2]);
        cplx<T> x0 = v[0];
        cplx<T> m = mk<T>(x0.x + c * t.x, x0.y + c * t.y);
        cplx<T> su = mul_i<T, DIR>(cscale<T>(u, s));     // DIR * i * s * u
        v[0] = cadd<T>(x0, t);
        v[1] = cadd<T>(m, su);
        v[2] = csub<T>(m, su);
    }
};

template <typename T, int DIR> struct Dft<T, 4, DIR> {
    static __device__ __forceinline__ void run(cplx<T>* v) {
        cplx<T> a = cadd<T>(v[0], v[2]);
        cplx<T> b = csub<T>(v[0], v[2]);
        cplx<T> c = cadd<T>(v[1], v[3]);
        cplx<T> d = mul_i<T, DIR>(csub<T>(v[1], v[3]));
        v[0] = cadd<T>(a, c);
        v[2] = csub<T>(a, c);
        v[1] = cadd<T>(b, d);
        v[3] = csub<T>(b, d);
    }
};

template <typename T, int DIR> struct Dft<T, 5, DIR> {
    static __device__ __forceinline__ void run(cplx<T>* v) {
        const T c1 = T(0.30901699437494742410229341718282);    // cos(2 pi / 5)
        const T c2 = T(-0.80901699437494742410229341718282);   // cos(4 pi / 5)
        const T s1 = T(0.95105651629515357211643933337938);    // sin(2 pi / 5)
        const T s2 = T(0.58778525229247312916870595463907);    // sin(4 pi / 5)
        cplx<T> x0 = v[0];
        cplx<T> t1 = cadd<T>(v[1], v[4]), u1 = csub<T>(v[1], v[4]);
        cplx<T> t2 = cadd<T>(v[2], v[3]), u2 = csub<T>(v[2], v[3]);
        cplx<T> a1 = mk<T>(x0.x + c1 * t1.x + c2 * t2.x, x0.y + c1 * t1.y + c2 * t2.y);
        cplx<T> a2 = mk<T>(x0.x + c2 * t1.x + c1 * t2.x, x0.y + c2 * t1.y + c1 * t2.y);
        cplx<T> b1 = mul_i<T, DIR>(mk<T>(s1 * u1.x + s2 * u2.x, s1 * u1.y + s2 * u2.y));
        cplx<T> b2 = mul_i<T, DIR>(mk<T>(s2 * u1.x - s1 * u2.x, s2 * u1.y - s1 * u2.y));
        v[0] = mk<T>(x0.x + t1.x + t2.x, x0.y + t1.y + t2.y);
        v[1] = cadd<T>(a1, b1);
        v[4] = csub<T>(a1, b1);
        v[2] = cadd<T>(a2, b2);
        v[3] = csub<T>(a2, b2);
    }
};

// 6 = 2 x 3 with coprime factors (Good-Thomas prime-factor mapping, no twiddles):
// input n = (3 n1 + 2 n2) mod 6, so w6^{n k} = w2^{n1 k} w3^{n2 k}; 2-point DFTs over
// n1 for each n2, then 3-point DFTs over n2 for each k1 = k mod 2, and X_k is the
// result at (k mod 2, k mod 3).
template <typename T, int DIR> struct Dft<T, 6, DIR> {
    static __device__ __forceinline__ void run(cplx<T>* v) {
        // n2 = 0, 1, 2 take the input pairs (n1 = 0, 1) = (0, 3), (2, 5), (4, 1)
        cplx<T> e[3] = {cadd<T>(v[0], v[3]), cadd<T>(v[2], v[5]), cadd<T>(v[4], v[1])};   // k1 = 0
        cplx<T> o[3] = {csub<T>(v[0], v[3]), csub<T>(v[2], v[5]), csub<T>(v[4], v[1])};   // k1 = 1
        Dft<T, 3, DIR>::run(e);
        Dft<T, 3, DIR>::run(o);
        // k = 0..5 -> (k mod 2, k mod 3)
        v[0] = e[0];
        v[1] = o[1];
        v[2] = e[2];
        v[3] = o[0];
        v[4] = e[1];
        v[5] = o[2];
    }
};

// 8 = 2 x 4: inner 2-point DFTs over (x[n2], x[n2 + 4]), twiddle w8^{n2 k1}, outer 4-point.
template <typename T, int DIR> struct Dft<T, 8, DIR> {
    static __device__ __forceinline__ void run(cplx<T>* v) {
        cplx<T> y0[4], y1[4];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
            y0[n2] = cadd<T>(v[n2], v[n2 + 4]);
            y1[n2] = csub<T>(v[n2], v[n2 + 4]);
        }
        const T r = T(0.70710678118654752440084436210485);
        // w8^1 = r(1, DIR), w8^2 = DIR i, w8^3 = r(-1, DIR)
        y1[1] = mk<T>(r * (y1[1].x - T(DIR) * y1[1].y), r * (y1[1].y + T(DIR) * y1[1].x));
        y1[2] = mul_i<T, DIR>(y1[2]);
        y1[3] = mk<T>(r * (-y1[3].x - T(DIR) * y1[3].y), r * (-y1[3].y + T(DIR) * y1[3].x));
        Dft<T, 4, DIR>::run(y0);
        Dft<T, 4, DIR>::run(y1);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) {
            v[2 * k2] = y0[k2];
            v[2 * k2 + 1] = y1[k2];
        }
    }
};

// ---------------------------------------------------------------------------
// radix schedules of the supported lengths
// ---------------------------------------------------------------------------
template <int N> struct Sched;
#define OCCRIK_SCHED(N_, a_, b_, c_)                                   \
    template <> struct Sched<N_> {                                     \
        static constexpr int r0 = a_, r1 = b_, r2 = c_;                \
    };
OCCRIK_SCHED(2, 2, 0, 0)
OCCRIK_SCHED(3, 3, 0, 0)
OCCRIK_SCHED(4, 4, 0, 0)
OCCRIK_SCHED(5, 5, 0, 0)
OCCRIK_SCHED(6, 6, 0, 0)
OCCRIK_SCHED(8, 8, 0, 0)
OCCRIK_SCHED(9, 3, 3, 0)
OCCRIK_SCHED(10, 5, 2, 0)
OCCRIK_SCHED(12, 4, 3, 0)
OCCRIK_SCHED(15, 5, 3, 0)
OCCRIK_SCHED(16, 4, 4, 0)
OCCRIK_SCHED(18, 6, 3, 0)
OCCRIK_SCHED(20, 5, 4, 0)
OCCRIK_SCHED(24, 8, 3, 0)
OCCRIK_SCHED(25, 5, 5, 0)
OCCRIK_SCHED(27, 3, 3, 3)
OCCRIK_SCHED(30, 6, 5, 0)
OCCRIK_SCHED(32, 8, 4, 0)
OCCRIK_SCHED(36, 6, 6, 0)
OCCRIK_SCHED(40, 8, 5, 0)
OCCRIK_SCHED(45, 5, 3, 3)
OCCRIK_SCHED(48, 8, 6, 0)
OCCRIK_SCHED(50, 5, 5, 2)
OCCRIK_SCHED(54, 6, 3, 3)
OCCRIK_SCHED(60, 6, 5, 2)
OCCRIK_SCHED(64, 8, 8, 0)
#undef OCCRIK_SCHED

// The supported lengths, for host-side validation (1 means "no transform").
inline bool grid_size_supported(int n) {
    switch (n) {
        case 1: case 2: case 3: case 4: case 5: case 6: case 8: case 9: case 10: case 12:
        case 15: case 16: case 18: case 20: case 24: case 25: case 27: case 30: case 32:
        case 36: case 40: case 45: case 48: case 50: case 54: case 60: case 64:
            return true;
        default:
            return false;
    }
}

// One Stockham stage of radix R after sub-transforms of length NS, run by NT
// threads.  With the line count fixed at compile time (LINES > 0) work items
// are numbered line-fastest, so the lanes of a wave touch consecutive lines:
// consecutive LDS addresses when lines are adjacent (ls = 1) and a fixed
// odd-padded stride when elements are adjacent (es = 1), both free of bank
// conflicts.  With a run-time line count (LINES = 0, at most kMaxN lines) they
// are numbered element-fastest, which needs no run-time division.
template <typename T, int N, int R, int NS, int DIR, int LINES, int NT>
__device__ __forceinline__ void stockham_stage(cplx<T>* buf, int lines, int es, int ls, const cplx<T>* tw) {
    constexpr int NB = N / R;                                   // butterflies per line
    constexpr int MAXL = LINES > 0 ? LINES : kMaxN;
    constexpr int ITEMS = (MAXL * NB + NT - 1) / NT;
    constexpr int TWS = N / (NS * R);                           // twiddle index step
    if constexpr (LINES > 0) lines = LINES;
    cplx<T> v[ITEMS][R];
    const int total = lines * NB;
    auto split = [&](int it, int& line, int& j) {
        if constexpr (LINES > 0) {
            j = it / LINES;
            line = it - j * LINES;
        } else {
            line = it / NB;
            j = it - line * NB;
        }
    };
#pragma unroll
    for (int t = 0; t < ITEMS; ++t) {
        const int it = threadIdx.x + t * NT;
        if (it < total) {
            int line, j;
            split(it, line, j);
            const cplx<T>* p = buf + line * ls;
#pragma unroll
            for (int r = 0; r < R; ++r) v[t][r] = p[(j + r * NB) * es];
        }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < ITEMS; ++t) {
        const int it = threadIdx.x + t * NT;
        if (it < total) {
            int line, j;
            split(it, line, j);
            const int jm = j % NS;
            if (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    cplx<T> w = tw[jm * r * TWS];
                    if (DIR > 0) w.y = -w.y;
                    v[t][r] = cmul<T>(v[t][r], w);
                }
            }
            Dft<T, R, DIR>::run(v[t]);
            const int base = (j / NS) * NS * R + jm;
            cplx<T>* p = buf + line * ls;
#pragma unroll
            for (int r = 0; r < R; ++r) p[(base + r * NS) * es] = v[t][r];
        }
    }
    __syncthreads();
}

// Full transform of length N along every line of the tile.  The caller must
// have synchronised after writing the tile; the tile is ready on return.
template <typename T, int N, int DIR, int LINES = 0, int NT = kFftThreads>
__device__ __forceinline__ void fft_lines(cplx<T>* buf, int lines, int es, int ls, const cplx<T>* tw) {
    using S = Sched<N>;
    stockham_stage<T, N, S::r0, 1, DIR, LINES, NT>(buf, lines, es, ls, tw);
    if constexpr (S::r1 != 0) stockham_stage<T, N, S::r1, S::r0, DIR, LINES, NT>(buf, lines, es, ls, tw);
    if constexpr (S::r2 != 0) stockham_stage<T, N, S::r2, S::r0 * S::r1, DIR, LINES, NT>(buf, lines, es, ls, tw);
}

// ---------------------------------------------------------------------------
// Two-stage lengths N = R0 R1 with the stages exposed, for kernels that feed the
// first stage from registers, keep the second stage's outputs in registers, or
// alternate two LDS buffers.  Stage A (radix R0, no twiddles): item (line, j),
// j < R1, inputs at elements j + r R1 (r < R0), outputs at j R0 + r.  Stage B
// (radix R1, twiddles w_N^{j r}): item (line, j), j < R0, inputs and outputs at
// the same elements j + r R0 (r < R1), so stage B runs in place.  A then B is
// the Stockham transform of fft_lines; output in natural order.
// ---------------------------------------------------------------------------
template <int N>
struct Split2 {
    static constexpr int R0 = Sched<N>::r0;
    static constexpr int R1 = Sched<N>::r1;
    static_assert(Sched<N>::r2 == 0 && Sched<N>::r1 > 0, "two-stage lengths only");
};

// stage A on v[R0] (inputs in v), outputs stored at elements j R0 + r of a line
template <typename T, int N, int DIR>
__device__ __forceinline__ void stage_a_store(cplx<T>* v, cplx<T>* line, int j, int es) {
    constexpr int R0 = Split2<N>::R0;
    Dft<T, R0, DIR>::run(v);
#pragma unroll
    for (int r = 0; r < R0; ++r) line[(j * R0 + r) * es] = v[r];
}

template <typename T, int N>
__device__ __forceinline__ void stage_a_load(cplx<T>* v, const cplx<T>* line, int j, int es) {
    constexpr int R0 = Split2<N>::R0, R1 = Split2<N>::R1;
#pragma unroll
    for (int r = 0; r < R0; ++r) v[r] = line[(j + r * R1) * es];
}

// stage B twiddles of item j for the forward table tw[t] = e^{-2 pi i t / N}
template <typename T, int N>
__device__ __forceinline__ void stage_b_twiddles(cplx<T>* w, const cplx<T>* tw, int j) {
    constexpr int R1 = Split2<N>::R1;
#pragma unroll
    for (int r = 1; r < R1; ++r) w[r - 1] = tw[j * r];
}

template <typename T, int N>
__device__ __forceinline__ void stage_b_load(cplx<T>* v, const cplx<T>* line, int j, int es) {
    constexpr int R0 = Split2<N>::R0, R1 = Split2<N>::R1;
#pragma unroll
    for (int r = 0; r < R1; ++r) v[r] = line[(j + r * R0) * es];
}

// stage B on v[R1] with the item's forward twiddles w (conjugated for DIR = +1)
template <typename T, int N, int DIR>
__device__ __forceinline__ void stage_b(cplx<T>* v, const cplx<T>* w) {
    constexpr int R1 = Split2<N>::R1;
#pragma unroll
    for (int r = 1; r < R1; ++r) v[r] = DIR < 0 ? cmul<T>(v[r], w[r - 1]) : cjmul<T>(w[r - 1], v[r]);
    Dft<T, R1, DIR>::run(v);
}

template <typename T, int N>
__device__ __forceinline__ void stage_b_store(const cplx<T>* v, cplx<T>* line, int j, int es) {
    constexpr int R0 = Split2<N>::R0, R1 = Split2<N>::R1;
#pragma unroll
    for (int r = 0; r < R1; ++r) line[(j + r * R0) * es] = v[r];
}

// Run-time length dispatch for grids without a compile-time specialisation.
// Each length is a separate out-of-line function so that the caller does not
// carry the register footprint of every length at once.
template <typename T, int N, int DIR>
__device__ __noinline__ void fft_lines_out_of_line(cplx<T>* buf, int lines, int es, int ls, const cplx<T>* tw) {
    fft_lines<T, N, DIR>(buf, lines, es, ls, tw);
}

template <typename T, int DIR>
__device__ inline void fft_lines_n(int n, cplx<T>* buf, int lines, int es, int ls, const cplx<T>* tw) {
#define OCCRIK_CASE(N_) \
    case N_: fft_lines_out_of_line<T, N_, DIR>(buf, lines, es, ls, tw); break;
    switch (n) {
        OCCRIK_CASE(2) OCCRIK_CASE(3) OCCRIK_CASE(4) OCCRIK_CASE(5) OCCRIK_CASE(6) OCCRIK_CASE(8)
        OCCRIK_CASE(9) OCCRIK_CASE(10) OCCRIK_CASE(12) OCCRIK_CASE(15) OCCRIK_CASE(16) OCCRIK_CASE(18)
        OCCRIK_CASE(20) OCCRIK_CASE(24) OCCRIK_CASE(25) OCCRIK_CASE(27) OCCRIK_CASE(30) OCCRIK_CASE(32)
        OCCRIK_CASE(36) OCCRIK_CASE(40) OCCRIK_CASE(45) OCCRIK_CASE(48) OCCRIK_CASE(50) OCCRIK_CASE(54)
        OCCRIK_CASE(60) OCCRIK_CASE(64)
        default: break;                                   // n == 1: identity
    }
#undef OCCRIK_CASE
}

}  // namespace occrik
