// The two grid contractions of the build, on the matrix cores.
//
//   orbitals   psi~_{j k}(r) = sum_mu C_{mu j}(k) chi~_{mu k}(r)           (paper eq. occmo)
//   contract   K_{mu j}(k)   = -(dV/N_k) sum_r conj(chi~_{mu k}(r)) W~_{j k}(r)
//                                                      (the contraction of Alg. 3)
//
// Both are written as real GEMMs over interleaved (re, im) data:
//   orbitals   D[2j + c][n]  = sum_{2mu + c'} A[2j + c][2mu + c'] chi_{c'}(mu, n),
//              A = [[Re C, -Im C], [Im C, Re C]] per (j, mu)
//   contract   D[mu][2j + c'] = sum_{2n + c} chi_c(mu, n) B[2n + c][2j + c'],
//              B = [[Re W, Im W], [Im W, -Re W]] per (n, j)
// and run as 16 x 16 MFMA tiles:
//   MODE 0  FP64 data, v_mfma_f64_16x16x4_f64 (the contraction: 8 points per step)
//   MODE 1  FP32 data, v_mfma_f32_16x16x4_f32
//   MODE 2  FP32 data split into three bf16 terms x = h + m + l per operand,
//           v_mfma_f32_16x16x32_bf16 on the six products hh, hm, mh, hl, lh, mm
//           with FP32 accumulation (the 3-term splitting of Henry, Tang and
//           Heinecke, ARITH 2019).
// Lane layouts (16x16xK): A[i][k] in lane i%16 + 16 * (k / KL), B[k][j] in lane
// j + 16 * (k / KL), where KL is the number of k values a lane holds (1 for x4,
// 8 for x32).  D[i][j] sits in lane j + 16 * (i / 4), register i % 4 for the
// FP32-output forms, and in lane j + 16 * (i % 4), register i / 4 for the FP64
// form (both checked on the device with one-hot operands).
//
// The contraction splits the grid sum into chunks; each chunk is accumulated
// in the working precision and the chunk partials are added in FP64 in a fixed
// order.  Its FP32 forms consume 16 grid points per step, each lane loading 4
// consecutive points of its AO row and of W as 16-byte vectors; MODE 1 issues
// eight 16x16x4 products for them, MODE 2 the six split-bf16 16x16x32 products.  Both kernels stream the Bloch AOs once and are bandwidth-bound for
// the few occupied columns involved.
#include <type_traits>

#include "internal.hpp"

namespace occrik {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

template <int MODE> struct Acc { typedef f4 type; };
template <> struct Acc<0> { typedef d4 type; };

// row of D held by lane l in accumulator register r
template <int MODE>
__device__ __forceinline__ int out_row(int l, int r) {
    return MODE == 0 ? 4 * r + (l >> 4) : 4 * (l >> 4) + r;
}

// three-term bf16 splitting of an FP32 value
__device__ __forceinline__ void split3(float x, __bf16& h, __bf16& m, __bf16& l) {
    h = (__bf16)x;
    const float r1 = x - (float)h;
    m = (__bf16)r1;
    l = (__bf16)(r1 - (float)m);
}

template <int MODE>
__device__ __forceinline__ typename Acc<MODE>::type mfma4(double a, double b, typename Acc<MODE>::type c);
template <>
__device__ __forceinline__ d4 mfma4<0>(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ f4 mfma4<1>(double a, double b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32((float)a, (float)b, c, 0, 0, 0);
}

// six-product split-bf16 step over 8 k values per lane
// 32 real k values as eight FP32 16x16x4 products: lane group g supplies its value s as
// the k index g of product s (the same assignment for both operands, so the sum over k
// is only reordered)
__device__ __forceinline__ f4 mfma_x8(const float* a, const float* b, f4 c) {
#pragma unroll
    for (int v = 0; v < 8; ++v) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[v], b[v], c, 0, 0, 0);
    return c;
}

__device__ __forceinline__ f4 mfma_split(const float* a, const float* b, f4 c) {
    bf8 ah, am, al, bh, bm, bl;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        __bf16 h, m, l;
        split3(a[v], h, m, l);
        ah[v] = h; am[v] = m; al[v] = l;
        split3(b[v], h, m, l);
        bh[v] = h; bm[v] = m; bl[v] = l;
    }
    // small terms first
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
    return c;
}

constexpr int kMaxRowTiles = 2;   // 2 nocc <= 32
constexpr int kOrbChunk = 32;     // AOs per LDS chunk of the A operand
constexpr int kOrbTiles = 4;      // 16-point tiles per wave (one tile when a launch is small)
constexpr int kFlush = 32;        // FP32 MFMA steps (x4 forms) between FP64 flushes in the contraction

// ---------------------------------------------------------------------------
// orbitals: one workgroup = 4 waves x TILES tiles x 16 points of one k
// ---------------------------------------------------------------------------
template <typename T, int MODE, int TILES>
__global__ void __launch_bounds__(256) orbitals_mfma(const cplx<T>* __restrict__ chi, size_t ldc,
                                                     const double2* __restrict__ C, cplx<T>* __restrict__ psi,
                                                     int nao, int nocc, int ng, int n0, int cnt) {
    typedef typename Acc<MODE>::type acc_t;
    constexpr int KCH = 2 * kOrbChunk;                  // real k values per chunk
    __shared__ T alds[kMaxRowTiles][16][KCH];
    const int k = blockIdx.y;
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int nbase = (blockIdx.x * 4 + wave) * TILES * 16;    // point of the chunk
    const int rt_n = (2 * nocc + 15) / 16;
    const T* chir = reinterpret_cast<const T*>(chi) + (size_t)2 * k * nao * ldc;
    const double2* Ck = C + (size_t)k * nao * nocc;
    acc_t acc[kMaxRowTiles][TILES];
#pragma unroll
    for (int rt = 0; rt < kMaxRowTiles; ++rt)
#pragma unroll
        for (int t = 0; t < TILES; ++t) acc[rt][t] = acc_t{};
    for (int m0 = 0; m0 < nao; m0 += kOrbChunk) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < kMaxRowTiles * 16 * KCH; idx += 256) {
            const int rt = idx / (16 * KCH), rem = idx - rt * 16 * KCH, row = rem / KCH, kk = rem - row * KCH;
            const int j = (rt * 16 + row) >> 1, c = row & 1, mu = m0 + (kk >> 1), cc = kk & 1;
            T a = T(0);
            if (j < nocc && mu < nao) {
                const double2 cv = Ck[(size_t)mu * nocc + j];
                a = T(c == 0 ? (cc == 0 ? cv.x : -cv.y) : (cc == 0 ? cv.y : cv.x));
            }
            alds[rt][row][kk] = a;
        }
        __syncthreads();
        if constexpr (MODE < 2) {
#pragma unroll 4
            for (int s = 0; s < KCH / 4; ++s) {
                const int kk = 4 * s + (l >> 4);
                const int mu = m0 + (kk >> 1), cc = kk & 1;
                T bv[TILES];
#pragma unroll
                for (int t = 0; t < TILES; ++t) {
                    const int n = nbase + 16 * t + (l & 15);
                    bv[t] = (mu < nao && n < cnt) ? chir[2 * ((size_t)mu * ldc + n) + cc] : T(0);
                }
#pragma unroll
                for (int rt = 0; rt < kMaxRowTiles; ++rt) {
                    if (rt < rt_n) {
                        const T a = alds[rt][l & 15][kk];
#pragma unroll
                        for (int t = 0; t < TILES; ++t) acc[rt][t] = mfma4<MODE>(a, bv[t], acc[rt][t]);
                    }
                }
            }
        } else {
#pragma unroll 1
            for (int s = 0; s < KCH / 32; ++s) {
                const int kk0 = 32 * s + 8 * (l >> 4);
                float bv[TILES][8];
#pragma unroll
                for (int t = 0; t < TILES; ++t) {
                    const int n = nbase + 16 * t + (l & 15);
                    // (re, im) of one AO at this point in one 8-byte load (kk0 is even)
#pragma unroll
                    for (int v = 0; v < 8; v += 2) {
                        const int mu = m0 + ((kk0 + v) >> 1);
                        cplx<T> x = mk<T>(T(0), T(0));
                        if (mu < nao && n < cnt) x = *reinterpret_cast<const cplx<T>*>(chir + 2 * ((size_t)mu * ldc + n));
                        bv[t][v] = (float)x.x;
                        bv[t][v + 1] = (float)x.y;
                    }
                }
#pragma unroll
                for (int rt = 0; rt < kMaxRowTiles; ++rt) {
                    if (rt < rt_n) {
                        float av[8];
#pragma unroll
                        for (int v = 0; v < 8; ++v) av[v] = (float)alds[rt][l & 15][kk0 + v];
#pragma unroll
                        for (int t = 0; t < TILES; ++t) acc[rt][t] = mfma_split(av, bv[t], acc[rt][t]);
                    }
                }
            }
        }
    }
    T* psir = reinterpret_cast<T*>(psi) + (size_t)2 * k * nocc * ng;
#pragma unroll
    for (int rt = 0; rt < kMaxRowTiles; ++rt) {
        if (rt >= rt_n) continue;
#pragma unroll
        for (int t = 0; t < TILES; ++t) {
            const int n = nbase + 16 * t + (l & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rt * 16 + out_row<MODE>(l, r), j = row >> 1, c = row & 1;
                if (j < nocc && n < cnt) psir[2 * ((size_t)j * ng + n0 + n) + c] = T(acc[rt][t][r]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// contraction: one wave = 16 AOs x (2 nocc) columns over one chunk of the grid
// ---------------------------------------------------------------------------
template <typename T, int MODE>
__global__ void __launch_bounds__(256) contract_mfma(const cplx<T>* __restrict__ chi, size_t ldc, int chi_n0,
                                                     const cplx<T>* __restrict__ W, double* __restrict__ Kpart,
                                                     int nao, int nocc, int ng, int chunk, int c_first, int nchunks) {
    typedef typename Acc<MODE>::type acc_t;
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int c = c_first + blockIdx.x;
    const int mu0 = (blockIdx.y * 4 + wave) * 16;
    const int k = blockIdx.z;
    const int n0 = c * chunk, n1 = min(ng, n0 + chunk);
    const int ct_n = (2 * nocc + 15) / 16;
    const int mu = mu0 + (l & 15);
    // chi holds grid points chi_n0.. of each (k, mu) row
    const T* chir = reinterpret_cast<const T*>(chi) + (size_t)2 * ((size_t)k * nao + min(mu, nao - 1)) * ldc -
                    (ptrdiff_t)2 * chi_n0;
    const cplx<T>* Wk = W + (size_t)k * nocc * ng;
    acc_t acc[kMaxRowTiles];
    double tot[kMaxRowTiles][4];
#pragma unroll
    for (int rt = 0; rt < kMaxRowTiles; ++rt) {
        acc[rt] = acc_t{};
#pragma unroll
        for (int r = 0; r < 4; ++r) tot[rt][r] = 0.0;
    }
    // FP32 accumulators are flushed into FP64 running sums every kFlush steps
    auto flush = [&]() {
#pragma unroll
        for (int rt = 0; rt < kMaxRowTiles; ++rt) {
#pragma unroll
            for (int r = 0; r < 4; ++r) tot[rt][r] += double(acc[rt][r]);
            acc[rt] = acc_t{};
        }
    };
    if (mu0 < nao) {
        if constexpr (MODE == 0) {
            // 16 real k values per step = 8 grid points: lane group g holds the 2 consecutive
            // points n + 2g, n + 2g + 1 (re, im of each) and supplies its value s as the k
            // index g of the s-th 16x16x4 product
            const bool mu_ok = mu < nao;
            for (int n = n0; n < n1; n += 8) {
                const int nb = n + 2 * (l >> 4);
                double av[4];
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    cplx<T> x = mk<T>(T(0), T(0));
                    if (mu_ok && nb + p < n1) x = *reinterpret_cast<const cplx<T>*>(chir + 2 * (size_t)(nb + p));
                    av[2 * p] = x.x;
                    av[2 * p + 1] = x.y;
                }
#pragma unroll
                for (int rt = 0; rt < kMaxRowTiles; ++rt) {
                    if (rt < ct_n) {
                        const int col = rt * 16 + (l & 15), j = col >> 1, cp = col & 1;
                        double bv[4];
#pragma unroll
                        for (int p = 0; p < 2; ++p) {
                            cplx<T> w = mk<T>(T(0), T(0));
                            if (j < nocc && nb + p < n1) w = Wk[(size_t)j * ng + nb + p];
                            bv[2 * p] = cp == 0 ? w.x : w.y;
                            bv[2 * p + 1] = cp == 0 ? w.y : -w.x;
                        }
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[rt] = mfma4<MODE>(av[v], bv[v], acc[rt]);
                    }
                }
            }
        } else {
            // 32 real k values per step = 16 grid points; this lane holds 4 consecutive points.
            // Whole steps load them as two 16-byte vectors when every row stride and offset is
            // even (then, with steps on multiples of 4 points, each load is 16-byte aligned);
            // otherwise, and for the ragged last step of a chunk, point by point.
            int step = 0;
            const bool mu_ok = mu < nao;
            const bool vec = ((ldc | (size_t)ng | (size_t)chi_n0) & 1) == 0;
            for (int n = n0; n < n1; n += 16) {
                const int nb = n + 4 * (l >> 4);
                const bool whole = vec && n + 16 <= n1;
                float av[8];
                if (whole) {
                    const float4* s4 = reinterpret_cast<const float4*>(chir + 2 * (size_t)nb);
                    const float4 x0 = s4[0], x1 = s4[1];
                    const float z = mu_ok ? 1.f : 0.f;
                    av[0] = z * x0.x; av[1] = z * x0.y; av[2] = z * x0.z; av[3] = z * x0.w;
                    av[4] = z * x1.x; av[5] = z * x1.y; av[6] = z * x1.z; av[7] = z * x1.w;
                } else {
#pragma unroll
                    for (int p = 0; p < 4; ++p) {
                        const bool ok = nb + p < n1 && mu_ok;
                        av[2 * p] = ok ? (float)chir[2 * (size_t)(nb + p)] : 0.f;
                        av[2 * p + 1] = ok ? (float)chir[2 * (size_t)(nb + p) + 1] : 0.f;
                    }
                }
#pragma unroll
                for (int rt = 0; rt < kMaxRowTiles; ++rt) {
                    if (rt < ct_n) {
                        const int col = rt * 16 + (l & 15), j = col >> 1, cp = col & 1;
                        float bv[8];
                        if (whole) {
                            const int jc = j < nocc ? j : nocc - 1;
                            const float4* w4 = reinterpret_cast<const float4*>(Wk + (size_t)jc * ng + nb);
                            const float4 y0 = w4[0], y1 = w4[1];
                            const float z = j < nocc ? 1.f : 0.f;
                            const float wr[4] = {z * y0.x, z * y0.z, z * y1.x, z * y1.z};
                            const float wi[4] = {z * y0.y, z * y0.w, z * y1.y, z * y1.w};
#pragma unroll
                            for (int p = 0; p < 4; ++p) {
                                bv[2 * p] = cp == 0 ? wr[p] : wi[p];
                                bv[2 * p + 1] = cp == 0 ? wi[p] : -wr[p];
                            }
                        } else {
#pragma unroll
                            for (int p = 0; p < 4; ++p) {
                                cplx<T> w = mk<T>(T(0), T(0));
                                if (nb + p < n1 && j < nocc) w = Wk[(size_t)j * ng + nb + p];
                                bv[2 * p] = cp == 0 ? (float)w.x : (float)w.y;
                                bv[2 * p + 1] = cp == 0 ? (float)w.y : -(float)w.x;
                            }
                        }
                        if constexpr (MODE == 2) acc[rt] = mfma_split(av, bv, acc[rt]);
                        else acc[rt] = mfma_x8(av, bv, acc[rt]);
                    }
                }
                if (++step == kFlush / 8) {
                    flush();
                    step = 0;
                }
            }
        }
    }
    flush();
#pragma unroll
    for (int rt = 0; rt < kMaxRowTiles; ++rt) {
        if (rt >= ct_n) continue;
        const int col = rt * 16 + (l & 15), j = col >> 1, cp = col & 1;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = mu0 + out_row<MODE>(l, r);
            if (m < nao && j < nocc) Kpart[2 * ((((size_t)k * nao + m) * nocc + j) * nchunks + c) + cp] = tot[rt][r];
        }
    }
}

__global__ void contract_reduce_kernel(const double2* __restrict__ Kpart, double2* __restrict__ Kmi, size_t n,
                                       int nchunks, double scale) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    double sx = 0.0, sy = 0.0;
    for (int c = 0; c < nchunks; ++c) {
        const double2 v = Kpart[t * nchunks + c];
        sx += v.x;
        sy += v.y;
    }
    double2 r;
    r.x = scale * sx;
    r.y = scale * sy;
    Kmi[t] = r;
}

}  // namespace

template <typename T>
hipError_t launch_orbitals(const cplx<T>* chi, size_t ldc, const double2* C, cplx<T>* psi, int nk, int nao, int nocc,
                           int ng, int n0, int cnt, int mode, hipStream_t s) {
    if (cnt <= 0) return hipSuccess;
    // four 16-point tiles per wave share each A-operand load; a launch that would then
    // hold fewer than 2048 workgroups (a small cell) takes one tile per wave instead, so
    // that more of the chip streams chi~.  Every point's sum runs in the same order
    // either way.
    const bool wide = (size_t)((cnt + 4 * kOrbTiles * 16 - 1) / (4 * kOrbTiles * 16)) * nk >= 2048;
    const int per_wg = 4 * (wide ? kOrbTiles : 1) * 16;
    dim3 grid((unsigned)((cnt + per_wg - 1) / per_wg), (unsigned)nk);
    auto go = [&](auto tiles) {
        constexpr int TL = decltype(tiles)::value;
        if constexpr (sizeof(T) == 8) {
            hipLaunchKernelGGL((orbitals_mfma<T, 0, TL>), grid, dim3(256), 0, s, chi, ldc, C, psi, nao, nocc, ng, n0,
                               cnt);
        } else if (mode == 2) {
            hipLaunchKernelGGL((orbitals_mfma<T, 2, TL>), grid, dim3(256), 0, s, chi, ldc, C, psi, nao, nocc, ng, n0,
                               cnt);
        } else {
            hipLaunchKernelGGL((orbitals_mfma<T, 1, TL>), grid, dim3(256), 0, s, chi, ldc, C, psi, nao, nocc, ng, n0,
                               cnt);
        }
    };
    if (wide) go(std::integral_constant<int, kOrbTiles>{});
    else go(std::integral_constant<int, 1>{});
    return hipGetLastError();
}

int contract_chunk(int ng, int nchunks) {
    const int chunk = (ng + nchunks - 1) / nchunks;
    return (chunk + 15) / 16 * 16;
}

// chunks that hold grid points when nchunks are asked for: rounding the chunk up to
// 16 points can leave trailing chunks empty (12 x 10 x 9 points in 64 chunks of 32
// fill only 34).  contract_chunk(ng, contract_chunk_count(ng, n)) equals
// contract_chunk(ng, n), so the chunk boundaries do not move.
int contract_chunk_count(int ng, int nchunks) {
    const int chunk = contract_chunk(ng, nchunks);
    return (ng + chunk - 1) / chunk;
}

template <typename T>
hipError_t launch_contract_part(const cplx<T>* chi, size_t ldc, int chi_n0, const cplx<T>* W, double2* Kpart, int nk,
                                int nao, int nocc, int ng, int nchunks, int c0, int nc, int mode, hipStream_t s) {
    if (nc <= 0) return hipSuccess;
    const int chunk = contract_chunk(ng, nchunks);
    dim3 grid((unsigned)nc, (unsigned)((nao + 63) / 64), (unsigned)nk);
    double* kp = reinterpret_cast<double*>(Kpart);
    if constexpr (sizeof(T) == 8) {
        hipLaunchKernelGGL((contract_mfma<T, 0>), grid, dim3(256), 0, s, chi, ldc, chi_n0, W, kp, nao, nocc, ng, chunk,
                           c0, nchunks);
    } else {
        if (mode == 2)
            hipLaunchKernelGGL((contract_mfma<T, 2>), grid, dim3(256), 0, s, chi, ldc, chi_n0, W, kp, nao, nocc, ng,
                               chunk, c0, nchunks);
        else
            hipLaunchKernelGGL((contract_mfma<T, 1>), grid, dim3(256), 0, s, chi, ldc, chi_n0, W, kp, nao, nocc, ng,
                               chunk, c0, nchunks);
    }
    return hipGetLastError();
}

hipError_t launch_contract_reduce(const double2* Kpart, double2* Kmi, size_t n, int nchunks, double scale,
                                  hipStream_t s) {
    hipLaunchKernelGGL(contract_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Kpart, Kmi, n,
                       nchunks, scale);
    return hipGetLastError();
}

template hipError_t launch_orbitals<float>(const cplx<float>*, size_t, const double2*, cplx<float>*, int, int, int,
                                           int, int, int, int, hipStream_t);
template hipError_t launch_orbitals<double>(const cplx<double>*, size_t, const double2*, cplx<double>*, int, int, int,
                                            int, int, int, int, hipStream_t);
template hipError_t launch_contract_part<float>(const cplx<float>*, size_t, int, const cplx<float>*, double2*, int, int,
                                                int, int, int, int, int, int, hipStream_t);
template hipError_t launch_contract_part<double>(const cplx<double>*, size_t, int, const cplx<double>*, double2*, int,
                                                 int, int, int, int, int, int, int, hipStream_t);

}  // namespace occrik
