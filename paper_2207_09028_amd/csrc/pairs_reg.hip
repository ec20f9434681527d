// Pair round trips with register-resident line FFTs (cubic grids whose edge
// N is even with N/2 even: 24, 32, 36, 40, 48).
//
// Same three passes and the same batch/slot conventions as the LDS Stockham
// kernels in pairs.hip (paper Alg. 3 inner loops; eqs. aodf, Vrao, VGao,
// occrikinterm), but every 1D transform runs in registers on a lane pair
// (regfft.hpp) and LDS only carries the transposes between directions:
//
//   pass 1  planes n1: coalesced load of conj(psi~_{i b}) psi~_{j a} into LDS,
//           rows -> FFT along n3 (in place in the row), columns -> FFT along n2,
//           store X[slot][n1][m2][m3] straight from registers
//   pass 2  slab m2 of a group of pairs sharing k_b: columns m3 loaded straight
//           from X, FFT along n1 (DIT, blocked output), multiply by the kernel
//           f(|G+q|)/N_g from the batch's table, inverse along m1
//           (DIF, interleaved output), LDS transpose, inverse along m3, LDS
//           staging for a coalesced in-place store
//   pass 3  128-byte column blocks of x-planes: inverse along m2 of the potentials
//           of every output orbital at once, a-side accumulation in registers,
//           b-side (conjugate-pair reuse) summed over the orbitals through LDS
#include <algorithm>

#include "fft.hpp"
#include "internal.hpp"
#include "pairs_common.hpp"
#include "regfft.hpp"

namespace occrik {

using namespace pairs;

namespace {

template <int NN>
struct RegCfg {
    static constexpr int H = NN / 2;
    static constexpr int TPP = 2 * NN;                         // threads per plane or slab
    static constexpr int PL = (256 / TPP) > 0 ? 256 / TPP : 1;  // planes per workgroup
    static constexpr int NT = PL * TPP;                        // workgroup size
    static constexpr int S = NN + 1;                           // LDS row stride
    static constexpr int PLANE = NN * NN;
};

constexpr int colblock_r(int n, int elem) {
    int w = 128 / elem;
    while (w > 1 && n % w != 0) --w;
    return w;
}

// ---------------------------------------------------------------------------
// pass 1
// ---------------------------------------------------------------------------
template <typename T, int NN>
__global__ void __launch_bounds__(RegCfg<NN>::NT) pass1r_kernel(PairBatch B, const cplx<T>* __restrict__ psi,
                                                                cplx<T>* __restrict__ X) {
    using C = RegCfg<NN>;
    constexpr int H = C::H, S = C::S, PLANE = C::PLANE, PL = C::PL, NT = C::NT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* L = reinterpret_cast<cplx<T>*>(smem_raw);          // [PL][NN][S]
    constexpr int GPS = (NN + PL - 1) / PL;                      // plane groups per slot
    const int slot = blockIdx.x / GPS;
    const int n1base = (blockIdx.x - slot * GPS) * PL;
    int b, i, j;
    decode_slot(B, slot, b, i, j);
    const cplx<T>* pj = psi + ((size_t)B.a * B.nocc + j) * B.ng;
    const cplx<T>* pi = psi + ((size_t)b * B.nocc + i) * B.ng;
    // every load of the plane group issued before the first product is formed
    constexpr int TOT = PL * PLANE;
    constexpr int IT = (TOT + NT - 1) / NT;
    const int nvalid = (NN - n1base < PL ? NN - n1base : PL) * PLANE;
    const size_t g0 = (size_t)n1base * PLANE;
    cplx<T> ui[IT], uj[IT];
    static_assert(TOT % NT == 0, "a plane group is a whole number of workgroup sweeps");
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int e = threadIdx.x + it * NT;
        // planes past the grid edge (only when PL does not divide N) read plane n1base
        // again and are zeroed below, so every load stays in bounds without a branch
        const int ee = (NN % PL == 0 || e < nvalid) ? e : e % PLANE;
        ui[it] = pi[g0 + ee];
        uj[it] = pj[g0 + ee];
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int e = threadIdx.x + it * NT;
        const int p = e / PLANE, r = e - p * PLANE, n2 = r / NN, n3 = r - n2 * NN;
        cplx<T> u = cjmul<T>(ui[it], uj[it]);
        if (NN % PL != 0 && e >= nvalid) u = mk<T>(T(0), T(0));
        L[(p * NN + n2) * S + n3] = u;
    }
    __syncthreads();
    const int p = threadIdx.x / C::TPP, t = threadIdx.x - p * C::TPP, line = t >> 1, s = t & 1;
    cplx<T>* Lp = L + p * NN * S;
    cplx<T> x[H];
    // along n3: this lane pair owns row n2 = line (reads and writes stay in the row)
#pragma unroll
    for (int a = 0; a < H; ++a) x[a] = Lp[line * S + 2 * a + s];
    line_dit<T, NN, -1>(x, s);
#pragma unroll
    for (int m = 0; m < H; ++m) Lp[line * S + blocked_index(m, s, H)] = x[m];
    __syncthreads();
    // along n2: column m3 = line
#pragma unroll
    for (int a = 0; a < H; ++a) x[a] = Lp[(2 * a + s) * S + line];
    line_dit<T, NN, -1>(x, s);
    const int n1 = n1base + p;
    if (n1 < NN) {
        cplx<T>* out = X + (size_t)slot * B.ng + (size_t)n1 * PLANE + line;
#pragma unroll
        for (int m = 0; m < H; ++m) out[(size_t)blocked_index(m, s, H) * NN] = x[m];
    }
}

// ---------------------------------------------------------------------------
// pass 2
// ---------------------------------------------------------------------------
template <int NN>
__global__ void __launch_bounds__(RegCfg<NN>::NT) pass2r_kernel(PairBatch B, cplx<float>* __restrict__ X,
                                                                double* __restrict__ parts, int deriv_only) {
    using T = float;
    using C = RegCfg<NN>;
    constexpr int H = C::H, S = C::S, PLANE = C::PLANE, PL = C::PL, NT = C::NT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* L = reinterpret_cast<cplx<T>*>(smem_raw);          // [PL][NN][S]
    double* red = reinterpret_cast<double*>(L + PL * NN * S);     // [NT]
    const int m2i = blockIdx.x % NN;
    const int grp = blockIdx.x / NN;
    const int P = B.group;
    const int nn = B.nocc * B.nocc;
    const int gd = B.diag ? (B.ntri + P - 1) / P : 0;
    const int go = (nn + P - 1) / P;
    int s0, s1, b;
    if (grp < gd) {
        s0 = grp * P;
        s1 = min(B.ntri, s0 + P);
        b = B.a;
    } else {
        const int g = grp - gd;
        const int blk = g / go;
        const int base = (B.diag ? B.ntri : 0) + blk * nn;
        s0 = base + (g - blk * go) * P;
        s1 = min(base + nn, s0 + P);
        b = B.b0 + (B.diag ? 1 : 0) + blk;
    }
    const int p = threadIdx.x / C::TPP, t = threadIdx.x - p * C::TPP, line = t >> 1, s = t & 1;

    // kernel values at this lane's (m1, m2, m3 = line) points, shared by the whole group;
    // re-read per pair (cache hits) rather than held, which keeps the kernel at 3 waves/SIMD
    const float* kv = static_cast<const float*>(B.kvals) + ((size_t)kv_block(B, b) * NN + m2i) * PLANE + line;
    const T scale = T(B.inv_ng);
    cplx<T>* Lp = L + p * NN * S;
    double acc = 0.0;
    for (int sb = s0; sb < s1; sb += PL) {
        const int slot = sb + p;
        const bool active = slot < s1;
        double wgt = 1.0;
        if (B.reuse) {
            if (b != B.a) wgt = 2.0;
            else if (active) {
                int bb, ii, jj;
                decode_slot(B, slot, bb, ii, jj);
                wgt = ii == jj ? 1.0 : 2.0;
            }
        }
        cplx<T>* base = X + (size_t)(active ? slot : s0) * B.ng + (size_t)m2i * NN + line;
        cplx<T> x[H];
        // column m3 = line along n1, straight from device memory
#pragma unroll
        for (int a = 0; a < H; ++a) x[a] = active ? base[(size_t)(2 * a + s) * PLANE] : mk<T>(T(0), T(0));
        T v[H];
#pragma unroll
        for (int m = 0; m < H; ++m) v[m] = kv[blocked_index(m, s, H) * NN];
        line_dit<T, NN, -1>(x, s);
        if (deriv_only || B.parseval) {
            double pacc = 0.0;
#pragma unroll
            for (int m = 0; m < H; ++m)
                pacc += double(v[m]) * (double(x[m].x) * double(x[m].x) + double(x[m].y) * double(x[m].y));
            if (active) acc += wgt * pacc;
            if (deriv_only) continue;
        }
#pragma unroll
        for (int m = 0; m < H; ++m) x[m] = cscale<T>(x[m], v[m] * scale);
        line_dif<T, NN, +1>(x, s);                              // back along m1: n1 = 2k + s
        __syncthreads();                                        // LDS free from the last pair
#pragma unroll
        for (int k = 0; k < H; ++k) Lp[(2 * k + s) * S + line] = x[k];
        __syncthreads();
        // rows n1 = line along m3, inverse; this lane pair owns the row
#pragma unroll
        for (int a = 0; a < H; ++a) x[a] = Lp[line * S + 2 * a + s];
        line_dit<T, NN, +1>(x, s);
#pragma unroll
        for (int m = 0; m < H; ++m) Lp[line * S + blocked_index(m, s, H)] = x[m];
        __syncthreads();
        // coalesced in-place store of the slab [n1][n3]
        for (int e = threadIdx.x; e < PL * PLANE; e += NT) {
            const int pp = e / PLANE, r = e - pp * PLANE, n1 = r / NN, n3 = r - n1 * NN;
            if (sb + pp < s1)
                X[(size_t)(sb + pp) * B.ng + ((size_t)n1 * NN + m2i) * NN + n3] = L[(pp * NN + n1) * S + n3];
        }
    }
    if (B.parseval || deriv_only) {
        __syncthreads();
        red[threadIdx.x] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double tot = 0.0;
            for (int q = 0; q < NT; ++q) tot += red[q];
            parts[blockIdx.x] = tot;
        }
    }
}

// ---------------------------------------------------------------------------
// pass 3
// ---------------------------------------------------------------------------
template <typename T, int NN, int JC>
struct P3Cfg {
    static constexpr int H = NN / 2;
    static constexpr int WB = colblock_r(NN, (int)sizeof(cplx<T>));
    static constexpr int NCB = NN / WB;
    static constexpr int LN = JC * WB;     // lines (orbital, column)
    static constexpr int NT = 2 * LN;
};

template <typename T, int NN, int JC>
__global__ void __launch_bounds__((P3Cfg<T, NN, JC>::NT)) pass3r_kernel(PairBatch B, const cplx<T>* __restrict__ X,
                                                                       const cplx<T>* __restrict__ psi,
                                                                       cplx<T>* __restrict__ Wpart,
                                                                       cplx<T>* __restrict__ W) {
    using C = P3Cfg<T, NN, JC>;
    constexpr int H = C::H, WB = C::WB, NCB = C::NCB, LN = C::LN, NT = C::NT;
    constexpr int PLANE = NN * NN;
    constexpr int RW = (NN * WB + NT - 1) / NT;                 // b-side block points per thread
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* red = reinterpret_cast<cplx<T>*>(smem_raw);         // [NN][LN] b-side products
    const int n1 = blockIdx.x % NN;
    const int cb = (blockIdx.x / NN) % NCB;
    const int sp = blockIdx.x / (NN * NCB);
    const int c0 = cb * WB;
    const int nocc = B.nocc;
    const int nn = nocc * nocc;
    const int total = B.nb * nocc;
    const int chunk = (total + B.splits - 1) / B.splits;
    const int q0 = sp * chunk;
    const int q1 = min(total, q0 + chunk);
    const int first_full = B.b0 + (B.diag ? 1 : 0);
    const int full_base = B.diag ? B.ntri : 0;
    const int line = threadIdx.x >> 1, s = threadIdx.x & 1;
    const int jl = line / WB, w = line - jl * WB;
    const bool active = jl < nocc;
    const size_t col = (size_t)n1 * PLANE + c0 + w;
    // stored slot of (b, i; jl, a) for summed pair q = (b - b0) nocc + i, and whether it
    // holds the conjugate (lower triangle of the diagonal block)
    auto slot_of = [&](int q, bool& cj) {
        const int bb = B.b0 + q / nocc, i = q - (q / nocc) * nocc;
        cj = false;
        if (B.diag && bb == B.a) {
            cj = jl < i;
            return cj ? tri_index(jl, i, nocc) : tri_index(i, jl, nocc);
        }
        return full_base + (bb - first_full) * nn + i * nocc + jl;
    };
    auto load_line = [&](int q, cplx<T>* dst) {
        bool cj;
        const int slot = active ? slot_of(q, cj) : 0;
        const cplx<T>* src = X + (size_t)slot * B.ng + col;
#pragma unroll
        for (int a = 0; a < H; ++a) dst[a] = active ? src[(size_t)(2 * a + s) * NN] : mk<T>(T(0), T(0));
    };
    cplx<T> acc[H];
#pragma unroll
    for (int m = 0; m < H; ++m) acc[m] = mk<T>(T(0), T(0));
    for (int q = q0; q < q1; ++q) {
        const int bb = B.b0 + q / nocc, i = q - (q / nocc) * nocc;
        const bool bside = B.reuse && !(B.diag && bb == B.a);
        bool cj;
        (void)slot_of(q, cj);
        cplx<T> x[H];
        load_line(q, x);
        // this pair's b-side target block, read ahead of the reduction below
        cplx<T>* wout = W + ((size_t)bb * nocc + i) * B.ng + (size_t)n1 * PLANE + c0;
        cplx<T> wpre[RW];
        if (bside) {
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const int e = threadIdx.x + r * NT;
                const int n2 = e / WB, ww = e - n2 * WB;
                wpre[r] = (RW * NT == NN * WB || e < NN * WB) ? wout[(size_t)n2 * NN + ww] : mk<T>(T(0), T(0));
            }
        }
        line_dit<T, NN, +1>(x, s);                              // along m2: n2 blocked
        const cplx<T>* pi = psi + ((size_t)bb * nocc + i) * B.ng + col;
        const cplx<T>* pa = psi + ((size_t)B.a * nocc + (active ? jl : 0)) * B.ng + col;
        if (bside) __syncthreads();                             // red free from the last pair
#pragma unroll
        for (int m = 0; m < H; ++m) {
            const int n2 = blocked_index(m, s, H);
            cplx<T> v = x[m];
            if (cj) v.y = -v.y;
            if (active) {
                const cplx<T> u = pi[(size_t)n2 * NN];
                acc[m] = mk<T>(acc[m].x + u.x * v.x - u.y * v.y, acc[m].y + u.x * v.y + u.y * v.x);
                if (bside) {
                    const cplx<T> o = pa[(size_t)n2 * NN];
                    red[n2 * LN + line] = mk<T>(o.x * v.x + o.y * v.y, o.y * v.x - o.x * v.y);   // o conj(v)
                }
            }
        }
        if (bside) {
            __syncthreads();
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const int e = threadIdx.x + r * NT;
                if (RW * NT == NN * WB || e < NN * WB) {
                    const int n2 = e / WB, ww = e - n2 * WB;
                    cplx<T> sum = wpre[r];
                    for (int jj = 0; jj < nocc; ++jj) sum = cadd<T>(sum, red[n2 * LN + jj * WB + ww]);
                    wout[(size_t)n2 * NN + ww] = sum;
                }
            }
        }
    }
    if (active) {
        cplx<T>* out = Wpart + ((size_t)sp * nocc + jl) * B.ng + col;
#pragma unroll
        for (int m = 0; m < H; ++m) out[(size_t)blocked_index(m, s, H) * NN] = acc[m];
    }
}

}  // namespace

bool reg_fft_size(int n1, int n2, int n3) {
    if (n1 != n2 || n2 != n3) return false;
    switch (n1) {
        case 24: case 32: case 36: case 40: case 48: return true;
        default: return false;
    }
}

#define OCCRIK_RDISPATCH(NNV, ...)                              \
    switch (NNV) {                                              \
        case 24: { constexpr int NN = 24; __VA_ARGS__; } break; \
        case 32: { constexpr int NN = 32; __VA_ARGS__; } break; \
        case 36: { constexpr int NN = 36; __VA_ARGS__; } break; \
        case 40: { constexpr int NN = 40; __VA_ARGS__; } break; \
        case 48: { constexpr int NN = 48; __VA_ARGS__; } break; \
        default: return hipErrorInvalidValue;                   \
    }

hipError_t launch_pass1_reg(const PairBatch& B, const cplx<float>* psi, cplx<float>* X, hipStream_t s) {
    using T = float;
    OCCRIK_RDISPATCH(B.N1, {
        using C = RegCfg<NN>;
        const unsigned grid = (unsigned)((size_t)B.nslots * ((NN + C::PL - 1) / C::PL));
        const size_t lds = sizeof(cplx<T>) * (size_t)C::PL * NN * C::S;
        hipLaunchKernelGGL((pass1r_kernel<T, NN>), dim3(grid), dim3(C::NT), lds, s, B, psi, X);
    });
    return hipGetLastError();
}

hipError_t launch_pass2_reg(const PairBatch& B, cplx<float>* X, double* parts, int deriv_only, hipStream_t s) {
    using T = float;
    if (!B.kvals) return hipErrorInvalidValue;
    OCCRIK_RDISPATCH(B.N1, {
        using C = RegCfg<NN>;
        const unsigned grid = (unsigned)((size_t)NN * pair_groups(B));
        const size_t lds = sizeof(cplx<T>) * (size_t)C::PL * NN * C::S + sizeof(double) * C::NT;
        hipLaunchKernelGGL((pass2r_kernel<NN>), dim3(grid), dim3(C::NT), lds, s, B, X, parts, deriv_only);
    });
    return hipGetLastError();
}

hipError_t launch_pass3_reg(const PairBatch& B, const cplx<float>* X, const cplx<float>* psi, cplx<float>* Wpart,
                            cplx<float>* W, hipStream_t s) {
    using T = float;
    if (B.nocc > 8) return hipErrorInvalidValue;
    OCCRIK_RDISPATCH(B.N1, {
        using C = P3Cfg<T, NN, 8>;
        const unsigned grid = (unsigned)((size_t)NN * C::NCB * B.splits);
        const size_t lds = sizeof(cplx<T>) * (size_t)NN * C::LN;
        hipLaunchKernelGGL((pass3r_kernel<T, NN, 8>), dim3(grid), dim3(C::NT), lds, s, B, X, psi, Wpart, W);
    });
    return hipGetLastError();
}

}  // namespace occrik
