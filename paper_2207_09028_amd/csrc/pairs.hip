// The occ-RI-K pair round trips (paper Alg. 3, inner loops; eqs. aodf, Vrao,
// VGao, occrikinterm) as three fused passes over a batch of pair densities.
//
// A 3D transform of N_1 x N_2 x N_3 points does not fit one CU's LDS, so each
// forward + inverse round trip exchanges the data through device memory twice:
//
//   pass 1  (one x-plane n1 of one stored pair per workgroup)
//           u = conj(psi~_{i b}) psi~_{j a} on the plane, FFT along n3 and n2,
//           store X[slot][n1][m2][m3]
//   pass 2  (one m2-slab of a group of stored pairs of one (a, b) block per
//           workgroup, in place) the kernel f(|G+q|)/N_g is evaluated once per
//           slab and reused for every pair of the group; FFT along n1, multiply,
//           inverse FFT along m1 and m3, store X[slot][n1][m2][n3]
//   pass 3  inverse FFT along m2 of each plane, multiply by the partner orbital
//           and accumulate: W~_{j a} (a-side, split over the (b, i) sum, partial
//           sums reduced in a fixed order) and, with conjugate-pair reuse,
//           W~_{i b} += psi~_{j a} conj(Vt_ij) (b-side, one workgroup per plane)
//
// The potential Vt = IDFT(f DFT(u)) / N_g is the cell-periodic part of V;
// psi~_{i b} Vt is the cell-periodic part of psi_{i b} V, so W~ = e^{-ik_a.r} W.
//
// Conjugate-pair reuse (symmetric Nyquist mode only, where it is exact): the
// density of (k_b, k_a, j, i) is the conjugate of that of (k_a, k_b, i, j) and
// its potential is the conjugate potential.  A batch then covers the blocks
// (a, b) with b >= a; the diagonal block stores the pairs i <= j only.
#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "fft.hpp"
#include "internal.hpp"
#include "pairs_common.hpp"

namespace occrik {

using namespace pairs;

namespace {

// ---------------------------------------------------------------------------
// pass 1
// ---------------------------------------------------------------------------
// streaming load and store of a pair spectrum: the stored spectra of a batch far
// exceed the caches, and each pass touches a stored element once
template <typename T>
__device__ __forceinline__ cplx<T> load_nt(const cplx<T>* p) {
    typedef T nv2 __attribute__((ext_vector_type(2)));
    const nv2 t = __builtin_nontemporal_load(reinterpret_cast<const nv2*>(p));
    return mk<T>(t.x, t.y);
}

template <typename T>
__device__ __forceinline__ void store_nt(cplx<T>* p, cplx<T> v) {
    typedef T nv2 __attribute__((ext_vector_type(2)));
    nv2 t = {v.x, v.y};
    __builtin_nontemporal_store(t, reinterpret_cast<nv2*>(p));
}

template <typename T, int NN>
__global__ void __launch_bounds__(kFftThreads) pass1_kernel(PairBatch B, const cplx<T>* __restrict__ psi,
                                                            cplx<T>* __restrict__ X, const cplx<T>* __restrict__ twg) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* plane = tw + 3 * kMaxN;
    const Dims<NN> D(B);
    const int N2 = D.n2, N3 = D.n3, S = N3 + 1;
    const int plane_sz = N2 * N3;
    const int n1 = blockIdx.x % D.n1;
    const int slot = blockIdx.x / D.n1;
    int b, i, j;
    decode_slot(B, slot, b, i, j);
    load_twiddles<T>(tw, twg);
    const cplx<T>* pj = static_cast<const cplx<T>*>(B.outp) + (size_t)j * B.ng + (size_t)n1 * plane_sz;
    const cplx<T>* pi = psi + ((size_t)b * B.kstride + i) * B.ng + (size_t)n1 * plane_sz;
    constexpr int PTS = ((NN > 0 ? NN * NN : kMaxN * kMaxN) + kFftThreads - 1) / kFftThreads;
#pragma unroll
    for (int t = 0; t < PTS; ++t) {
        const int e = threadIdx.x + t * kFftThreads;
        if (e < plane_sz) {
            const int n2 = e / N3, n3 = e - n2 * N3;
            plane[n2 * S + n3] = cjmul<T>(pi[e], pj[e]);
        }
    }
    __syncthreads();
    lines<T, NN, -1>(N3, plane, N2, 1, S, tw + 2 * kMaxN);
    lines<T, NN, -1>(N2, plane, N3, S, 1, tw + kMaxN);
    cplx<T>* out = X + (size_t)slot * B.ng + (size_t)n1 * plane_sz;
#pragma unroll
    for (int t = 0; t < PTS; ++t) {
        const int e = threadIdx.x + t * kFftThreads;
        if (e < plane_sz) {
            const int m2 = e / N3, m3 = e - m2 * N3;
            out[e] = plane[m2 * S + m3];
        }
    }
}

// Pass 1 for the compiled cubic sizes, one workgroup per x-plane and group of rows
// of stored pairs (a row: one summed orbital i of block b with all its partners j;
// a group: up to four consecutive i of one block on large launches, one on small
// ones, or one row of the diagonal block): the summed
// orbitals psi~_{i b} of the group on the plane are held in
// registers for all their partners, each partner's plane is loaded once for the
// group's densities, and the next partner's plane is loaded while the current pairs
// are transformed.  A workgroup waits for device memory at its start, for the held
// orbitals; with several rows per workgroup that wait is shared by more pairs, and in
// complex64 an extra wave of each grouped workgroup loads a later workgroup's held
// orbitals into L2 ahead of it (pass1g_prefetch).  The
// plane transform runs as two-stage lines: stage A of axis n2 on the pair density in
// registers (lanes along n3), stage B in place, axis n3 from one LDS buffer into a
// second, and its stage B stored straight to memory.  Stage B items are numbered
// element-fastest, so eight consecutive lanes store 64 contiguous bytes of a row.
// 3 barriers and 6 LDS accesses per point per pair.
template <int NN>
struct P1G {
    static constexpr int R0 = Split2<NN>::R0, R1 = Split2<NN>::R1;
    static constexpr int NA = NN * R1, NBI = NN * R0;
    static constexpr int NT = ((NA > NBI ? NA : NBI) + 63) / 64 * 64;
    static constexpr int S = NN + 1;
};

// pass-1 workgroups per x-plane of a batch: the diagonal block's rows one by one, the
// other blocks' rows in groups of `rows`
inline int pass1_groups(const PairBatch& B, int rows) {
    return (B.diag ? B.nocc : 0) + (B.nb - (B.diag ? 1 : 0)) * ((B.nocc + rows - 1) / rows);
}

// rows of a block that one pass-1 workgroup holds: kPass1Rows where the launch keeps at
// least 4096 single-row workgroups (126 VGPRs at 48^3 in complex64, two workgroups per
// CU; 234 in complex128, one); one row otherwise, so that a small cell's launch still
// spreads over the chip
constexpr int kPass1Rows = 4;
inline int pass1_rows(const PairBatch& B, int nn) {
    return (size_t)nn * pass1_groups(B, 1) >= 4096 ? kPass1Rows : 1;
}

// group -> (block b, first summed orbital i, its rows, first slot, first partner j0);
// the diagonal block (if any) comes first, one row per group, and stores the
// partners j >= i of row i; row i + h of a group stores at slot0 + h nout + j
template <int ROWS>
__device__ __forceinline__ void pass1_group(const PairBatch& B, const int grp, int& b, int& i, int& slot0, int& j0,
                                            int& nrows) {
    const int nocc = B.nocc, nout = B.nout;
    if (B.diag && grp < nocc) {
        b = B.a;
        i = grp;
        j0 = i;
        slot0 = tri_index(i, i, nocc);
        nrows = 1;
    } else {
        const int r = grp - (B.diag ? nocc : 0);
        const int per_blk = (nocc + ROWS - 1) / ROWS;
        const int blk = r / per_blk;
        i = ROWS * (r - blk * per_blk);
        nrows = ROWS == 1 ? 1 : (nocc - i < ROWS ? nocc - i : ROWS);
        b = B.b0 + (B.diag ? 1 : 0) + blk;
        j0 = 0;
        slot0 = (B.diag ? B.ntri : 0) + blk * nocc * nout + i * nout;
    }
}

// Workgroups of a grouped pass-1 launch carry one extra wave that touches (one value
// per 128-byte line) the held orbitals of the workgroup pass1_lead places later.
// Workgroups go to the XCDs by blockIdx modulo 8, so with a lead that is a multiple
// of 8 the lines land in the L2 of the XCD that will run it, and that workgroup's
// wait at its start, for its held orbitals, becomes an L2 hit.  The wave must not
// wait for these loads while the other waves still meet at barriers: it passes the
// same number of barriers as they do, and the loaded values feed only a store under
// a condition that never holds (a batch has at least one block), so its one wait
// for them comes after its last barrier.  Leads of 64 to 256 run equally fast; the
// lines of longer leads are more often evicted before use (pass 1 reads 0.84, 0.88,
// 0.99 and 1.20 GB per paper-sized launch at 64, 128, 192 and 256, against 0.80
// without the wave).  Complex64 only: in complex128 the grouped kernel holds one
// workgroup per CU, and the extra wave made pass 1 slower at every lead tried.
template <typename T>
constexpr int pass1_lead() { return sizeof(T) == 4 ? 128 : 0; }

template <typename T, int NN, int ROWS>
__device__ __forceinline__ void pass1g_prefetch(const PairBatch& B, const cplx<T>* __restrict__ psi,
                                                cplx<T>* __restrict__ X, const int bid, const int nbar) {
    constexpr int LINE = 128 / (int)sizeof(T);          // values of T per 128-byte line
    constexpr int PT = 2 * NN * NN;                      // values of T per plane
    constexpr int LPL = (PT + LINE - 1) / LINE;          // lines per plane
    constexpr int PER = (LPL + 63) / 64;                 // lines per lane per plane
    // bid is blockIdx.x of a plain grouped launch (the fused kernels run single rows,
    // without this wave), so the launch's workgroups are 0 .. gridDim.x - 1.
    // Every load is unconditional and in bounds (straight-line code, so that nothing
    // consumes a value before the barriers): past the end of the grid the wave touches
    // its own workgroup's orbitals, and missing rows or lines repeat ones already touched
    constexpr int LEAD = pass1_lead<T>();
    const int tgt = bid + LEAD < (int)gridDim.x ? bid + LEAD : bid;
    int b, i, slot0, j0, nrows;
    pass1_group<ROWS>(B, tgt / NN, b, i, slot0, j0, nrows);
    const T* base = reinterpret_cast<const T*>(psi + ((size_t)b * B.kstride + i) * B.ng + (size_t)(tgt % NN) * NN * NN);
    const int lane = threadIdx.x & 63;
    T v[ROWS * PER];
#pragma unroll
    for (int h = 0; h < ROWS; ++h)
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int l = lane + p * 64 < LPL ? lane + p * 64 : LPL - 1;
            const int e = l * LINE < PT ? l * LINE : PT - 1;
            v[h * PER + p] = base[(size_t)(h < nrows ? h : 0) * 2 * B.ng + e];
        }
    for (int k = 0; k < nbar; ++k) __syncthreads();
    if (B.nb < 1) {
        T sum = T(0);
#pragma unroll
        for (int k = 0; k < ROWS * PER; ++k) sum += v[k];
        X[0].x = sum;
    }
}

template <typename T, int NN, int ROWS>
constexpr int pass1g_threads() { return P1G<NN>::NT + (ROWS > 1 && pass1_lead<T>() > 0 ? 64 : 0); }

template <typename T, int NN, int ROWS>
__device__ __forceinline__ void pass1g_body(const PairBatch& B, const cplx<T>* __restrict__ psi, cplx<T>* __restrict__ X, const cplx<T>* __restrict__ twg, const int bid) {
    using C = P1G<NN>;
    constexpr int R0 = C::R0, R1 = C::R1, S = C::S;
    constexpr int PLANE = NN * NN;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* Pb = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* Qb = Pb + NN * S;
    const int n1 = bid % NN;
    const int nocc = B.nocc, nout = B.nout;
    int b, i, slot0, j0, nrows;
    pass1_group<ROWS>(B, bid / NN, b, i, slot0, j0, nrows);
    const int tid = threadIdx.x;
    if constexpr (ROWS > 1 && pass1_lead<T>() > 0) {
        // the prefetch wave (wave-uniform test, so that each wave takes one path)
        if (__builtin_amdgcn_readfirstlane(tid) >= C::NT) {
            pass1g_prefetch<T, NN, ROWS>(B, psi, X, bid, 3 * nrows * (nout - j0));
            return;
        }
    }
    const bool ha = tid < C::NA, hb = tid < C::NBI;
    const int sj = tid / NN, ln = tid - sj * NN;        // stage A items: line-fastest
    const int bj = tid % R0, bl = tid / R0;             // stage B items: element-fastest
    cplx<T> w[R1 - 1];
    if (hb) stage_b_twiddles<T, NN>(w, twg + kMaxN, bj);
    else {
#pragma unroll
        for (int r = 0; r < R1 - 1; ++r) w[r] = mk<T>(T(0), T(0));
    }
    // this thread's stage A points (n2 = sj + r R1, n3 = ln) of psi~_{i + h, b}, held
    const size_t poff = (size_t)n1 * PLANE + ln;
    const cplx<T>* pi = psi + ((size_t)b * B.kstride + i) * B.ng + poff;
    cplx<T> uh[ROWS][R0], xn[R0];
#pragma unroll
    for (int h = 0; h < ROWS; ++h)
#pragma unroll
        for (int r = 0; r < R0; ++r)
            uh[h][r] = (ha && h < nrows) ? load_nt<T>(pi + (size_t)h * B.ng + (size_t)(sj + r * R1) * NN)
                                         : mk<T>(T(0), T(0));
    auto load_partner = [&](int j) {
        const cplx<T>* pj = static_cast<const cplx<T>*>(B.outp) + (size_t)j * B.ng + poff;
#pragma unroll
        for (int r = 0; r < R0; ++r) xn[r] = ha ? pj[(size_t)(sj + r * R1) * NN] : mk<T>(T(0), T(0));
    };
    load_partner(j0);
    for (int j = j0; j < nout; ++j)
#pragma unroll
    for (int h = 0; h < ROWS; ++h) {
        if (h >= nrows) break;
        const int slot = slot0 + h * nout + (j - j0);
        // axis n2 (lines n3 = ln, elements n2 at stride S): stage A on the pair density
        if (ha) {
            cplx<T> a[R0];
#pragma unroll
            for (int r = 0; r < R0; ++r) a[r] = cjmul<T>(uh[h][r], xn[r]);
            stage_a_store<T, NN, -1>(a, Pb + ln, sj, S);
        }
        // the next partner, once the group's last density of this one is formed
        if (h == nrows - 1 && j + 1 < nout) load_partner(j + 1);
        __syncthreads();
        if (hb) {
            cplx<T> u[R1];
            stage_b_load<T, NN>(u, Pb + bl, bj, S);
            stage_b<T, NN, -1>(u, w);
            stage_b_store<T, NN>(u, Pb + bl, bj, S);
        }
        __syncthreads();
        // axis n3 (lines m2 = ln at stride S, elements adjacent): P -> Q
        if (ha) {
            cplx<T> a[R0];
            stage_a_load<T, NN>(a, Pb + ln * S, sj, 1);
            stage_a_store<T, NN, -1>(a, Qb + ln * S, sj, 1);
        }
        __syncthreads();
        // last stage B straight to memory: eight consecutive lanes store elements
        // m3 = bj + r R0 of row m2 = bl, so a wave writes whole rows over its R1 stores
        if (hb) {
            cplx<T> u[R1];
            stage_b_load<T, NN>(u, Qb + bl * S, bj, 1);
            stage_b<T, NN, -1>(u, w);
            cplx<T>* out = X + (size_t)slot * B.ng + (size_t)n1 * PLANE + (size_t)bl * NN + bj;
#pragma unroll
            for (int r = 0; r < R1; ++r) store_nt<T>(out + r * R0, u[r]);
        }
    }
}

template <typename T, int NN, int ROWS>
__global__ void __launch_bounds__((pass1g_threads<T, NN, ROWS>())) pass1g_kernel(PairBatch B, const cplx<T>* __restrict__ psi, cplx<T>* __restrict__ X, const cplx<T>* __restrict__ twg) {
    pass1g_body<T, NN, ROWS>(B, psi, X, twg, (int)blockIdx.x);
}

// ---------------------------------------------------------------------------
// pass 2
// ---------------------------------------------------------------------------
// kernel values of a batch: f(|G+q|) (or df/domega) for every summed k_b, with the
// Nyquist-plane mean of the symmetric mode, laid out [b - b0][m2][m1][m3] so that
// every form of pass 2 reads them coalesced; evaluated in the working precision
// (the truncated kernels in FP64)
template <typename T>
__global__ void __launch_bounds__(256) kvals_kernel(PairBatch B, T* __restrict__ out, int deriv_only) {
    const int N1 = B.N1, N2 = B.N2, N3 = B.N3;
    const size_t per_b = (size_t)N1 * N2 * N3;
    const size_t total = (size_t)B.nb * per_b;
    Recip<T> rc;
#pragma unroll
    for (int d = 0; d < 9; ++d) rc.b[d] = T(B.recip[d]);
    const T om = T(B.omega);
    double qa[3];
    kfrac_of(B.a, B.M1, B.M2, B.M3, qa);
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
        const int bi = (int)(e / per_b);
        const int r = (int)(e - (size_t)bi * per_b);
        const int i2 = r / (N1 * N3), rem = r - i2 * (N1 * N3), i1 = rem / N3, i3 = rem - i1 * N3;
        double qb[3];
        kfrac_of(B.b0 + bi, B.M1, B.M2, B.M3, qb);
        out[e] = kernel_value<T>(B, rc, qa[0] - qb[0], qa[1] - qb[1], qa[2] - qb[2], i1, i2, i3, deriv_only, om);
    }
}

// the same values for every k-point difference of the mesh, q_d = (kappa_a - kappa_b)_d / M_d,
// laid out [difference index][m2][m1][m3] (kv_block gives the index of a pair of k-points)
template <typename T>
__global__ void __launch_bounds__(256) kcache_kernel(PairBatch B, T* __restrict__ out, int nq) {
    const int N1 = B.N1, N2 = B.N2, N3 = B.N3;
    const size_t per_q = (size_t)N1 * N2 * N3;
    const size_t total = (size_t)nq * per_q;
    const int D2 = 2 * B.M2 - 1, D3 = 2 * B.M3 - 1;
    Recip<T> rc;
#pragma unroll
    for (int d = 0; d < 9; ++d) rc.b[d] = T(B.recip[d]);
    const T om = T(B.omega);
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
        const int qi = (int)(e / per_q);
        const int r = (int)(e - (size_t)qi * per_q);
        const int i2 = r / (N1 * N3), rem = r - i2 * (N1 * N3), i1 = rem / N3, i3 = rem - i1 * N3;
        const int d1 = qi / (D2 * D3) - (B.M1 - 1), d2 = (qi / D3) % D2 - (B.M2 - 1), d3 = qi % D3 - (B.M3 - 1);
        out[e] = kernel_value<T>(B, rc, double(d1) / B.M1, double(d2) / B.M2, double(d3) / B.M3, i1, i2, i3, false, om);
    }
}

template <typename T, int NN>
__global__ void __launch_bounds__(kFftThreads) pass2_kernel(PairBatch B, cplx<T>* __restrict__ X,
                                                            const cplx<T>* __restrict__ twg,
                                                            double* __restrict__ parts, int deriv_only) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
    double* red = reinterpret_cast<double*>(tw + 3 * kMaxN);
    cplx<T>* tile = reinterpret_cast<cplx<T>*>(red + kFftThreads);
    constexpr int ITEMS = (kMaxN * kMaxN + kFftThreads - 1) / kFftThreads;
    constexpr int VI = NN > 0 ? (NN * NN + kFftThreads - 1) / kFftThreads : ITEMS;
    const Dims<NN> D(B);
    const int N1 = D.n1, N2 = D.n2, N3 = D.n3, S = N3 + 1;
    const int m2i = blockIdx.x % N2;
    const int grp = blockIdx.x / N2;
    // group -> (block, first slot, slot count); the diagonal block (if any) comes first
    const int P = B.group;
    const int nn = B.nocc * B.nout;
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
    load_twiddles<T>(tw, twg);

    // kernel values of this slab from the batch's table, shared by every pair of the group
    const int tile_sz = N1 * N3;
    const T* kv = static_cast<const T*>(B.kvals) + ((size_t)kv_block(B, b) * N2 + m2i) * tile_sz;
    T v[VI];
#pragma unroll
    for (int t = 0; t < VI; ++t) {
        const int e = threadIdx.x + t * kFftThreads;
        v[t] = e < tile_sz ? kv[e] : T(0);
    }
    const T scale = T(B.inv_ng);
    const size_t rs = (size_t)N2 * N3;
    double acc = 0.0;
    // the next pair's slab is loaded into registers while this one is transformed
    cplx<T> xn[VI];
    auto load_slab = [&](int sl) {
        const cplx<T>* src = X + (size_t)sl * B.ng + (size_t)m2i * N3;
#pragma unroll
        for (int t = 0; t < VI; ++t) {
            const int e = threadIdx.x + t * kFftThreads;
            const int n1 = e / N3, m3 = e - n1 * N3;
            xn[t] = e < tile_sz ? src[n1 * rs + m3] : mk<T>(T(0), T(0));
        }
    };
    load_slab(s0);
    for (int slot = s0; slot < s1; ++slot) {
        // weight of this stored pair in the full (k, k', i, j) sum
        double wgt = 1.0;
        if (B.reuse) {
            if (b != B.a) wgt = 2.0;
            else {
                int bb, ii, jj;
                decode_slot(B, slot, bb, ii, jj);
                wgt = ii == jj ? 1.0 : 2.0;
            }
        }
        cplx<T>* base = X + (size_t)slot * B.ng + (size_t)m2i * N3;
        __syncthreads();
#pragma unroll
        for (int t = 0; t < VI; ++t) {
            const int e = threadIdx.x + t * kFftThreads;
            if (e < tile_sz) {
                const int n1 = e / N3, m3 = e - n1 * N3;
                tile[n1 * S + m3] = xn[t];
            }
        }
        if (slot + 1 < s1) load_slab(slot + 1);
        __syncthreads();
        lines<T, NN, -1>(N1, tile, N3, S, 1, tw);
        double pacc = 0.0;
#pragma unroll
        for (int t = 0; t < VI; ++t) {
            const int e = threadIdx.x + t * kFftThreads;
            if (e < tile_sz) {
                const int t1 = e / N3, t3 = e - t1 * N3;
                const cplx<T> u = tile[t1 * S + t3];
                if (deriv_only || B.parseval)
                    pacc += double(v[t]) * (double(u.x) * double(u.x) + double(u.y) * double(u.y));
                if (!deriv_only) tile[t1 * S + t3] = cscale<T>(u, v[t] * scale);
            }
        }
        acc += wgt * pacc;
        if (deriv_only) continue;
        __syncthreads();
        lines<T, NN, +1>(N1, tile, N3, S, 1, tw);
        lines<T, NN, +1>(N3, tile, N1, 1, S, tw + 2 * kMaxN);
#pragma unroll
        for (int t = 0; t < VI; ++t) {
            const int e = threadIdx.x + t * kFftThreads;
            if (e < tile_sz) {
                const int n1 = e / N3, n3 = e - n1 * N3;
                base[n1 * rs + n3] = tile[n1 * S + n3];
            }
        }
    }
    if (B.parseval || deriv_only) {
        __syncthreads();
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int w = kFftThreads / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) parts[blockIdx.x] = red[0];
    }
}

// Pass 2 for the compiled cubic sizes (N = R0 R1): the slab transforms run as
// two-stage Stockham lines with stage A fed from the registers the global
// prefetch filled, the kernel multiply applied to the forward stage B outputs
// in registers, and the last inverse stage B stored straight to device memory
// (lanes along n3: coalesced).  Two LDS buffers alternate so that a stage A
// reads one and writes the other; stage B works in place.  Per pair: 5
// barriers and 10 LDS accesses per point (the single-buffer form takes 15 and 16).
template <int NN>
struct P2S {
    static constexpr int R0 = Split2<NN>::R0, R1 = Split2<NN>::R1;
    static constexpr int NA = NN * R1;                  // stage A items of a slab (line-fastest)
    static constexpr int NBI = NN * R0;                 // stage B items
    static constexpr int NT = ((NA > NBI ? NA : NBI) + 63) / 64 * 64;
    static constexpr int S = NN + 1;                    // padded row of the slab in LDS
};

template <typename T, int NN>
__device__ __forceinline__ void pass2s_body(const PairBatch& B, cplx<T>* __restrict__ X, const cplx<T>* __restrict__ twg, double* __restrict__ parts, int deriv_only, const int bid) {
    using C = P2S<NN>;
    constexpr int R0 = C::R0, R1 = C::R1, S = C::S, NT = C::NT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* red = reinterpret_cast<double*>(smem_raw);
    cplx<T>* buf0 = reinterpret_cast<cplx<T>*>(red + NT);
    cplx<T>* buf1 = buf0 + NN * S;
    const int m2i = bid % NN;
    const int grp = bid / NN;
    const int P = B.group;
    const int nn = B.nocc * B.nout;
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
    const int tid = threadIdx.x;
    const bool ha = tid < C::NA, hb = tid < C::NBI;
    const int aj = tid / NN, al = tid - aj * NN;        // stage A item (line al, index aj)
    const int bj = tid / NN, bl = al;                   // stage B item (line bl, index bj)
    constexpr size_t rs = (size_t)NN * NN;              // n1 stride of a pair's spectrum
    // stage B twiddles and this item's kernel values (element (m1, m3) = (bj + r R0, bl))
    cplx<T> w[R1 - 1];
    T v[R1];
    {
        const T* kv = static_cast<const T*>(B.kvals) + ((size_t)kv_block(B, b) * NN + m2i) * rs;
        if (hb) {
            stage_b_twiddles<T, NN>(w, twg, bj);
#pragma unroll
            for (int r = 0; r < R1; ++r) v[r] = kv[(size_t)(bj + r * R0) * NN + bl];
        } else {
#pragma unroll
            for (int r = 0; r < R1; ++r) v[r] = T(0);
#pragma unroll
            for (int r = 0; r < R1 - 1; ++r) w[r] = mk<T>(T(0), T(0));
        }
    }
    const T scale = T(B.inv_ng);
    double acc = 0.0;
    // stage A inputs of the forward n1 transform: elements n1 = aj + r R1 of line m3 = al
    cplx<T> xn[R0];
    auto load_slab = [&](int sl) {
        const cplx<T>* src = X + (size_t)sl * B.ng + (size_t)m2i * NN + al;
#pragma unroll
        for (int r = 0; r < R0; ++r) xn[r] = ha ? load_nt<T>(src + (size_t)(aj + r * R1) * rs) : mk<T>(T(0), T(0));
    };
    load_slab(s0);
    cplx<T>* Pb = buf0;
    cplx<T>* Qb = buf1;
    for (int slot = s0; slot < s1; ++slot) {
        double wgt = 1.0;
        if (B.reuse) {
            if (b != B.a) wgt = 2.0;
            else {
                int bb, ii, jj;
                decode_slot(B, slot, bb, ii, jj);
                wgt = ii == jj ? 1.0 : 2.0;
            }
        }
        // forward along n1 (lines m3, elements n1 at stride S): stage A from registers
        if (ha) {
            cplx<T> a[R0];
#pragma unroll
            for (int r = 0; r < R0; ++r) a[r] = xn[r];
            stage_a_store<T, NN, -1>(a, Pb + al, aj, S);
        }
        if (slot + 1 < s1) load_slab(slot + 1);
        __syncthreads();
        double pacc = 0.0;
        if (hb) {
            cplx<T> u[R1];
            stage_b_load<T, NN>(u, Pb + bl, bj, S);
            stage_b<T, NN, -1>(u, w);
#pragma unroll
            for (int r = 0; r < R1; ++r) {
                if (deriv_only || B.parseval)
                    pacc += double(v[r]) * (double(u[r].x) * double(u[r].x) + double(u[r].y) * double(u[r].y));
                u[r] = cscale<T>(u[r], v[r] * scale);
            }
            if (!deriv_only) stage_b_store<T, NN>(u, Pb + bl, bj, S);
        }
        acc += wgt * pacc;
        if (deriv_only) {
            // the next pair's stage A writes the other buffer while this one is read
            cplx<T>* t = Pb;
            Pb = Qb;
            Qb = t;
            continue;
        }
        __syncthreads();
        // inverse along m3 (lines m1 at stride S, elements m3 adjacent): P -> Q
        if (ha) {
            cplx<T> a[R0];
            stage_a_load<T, NN>(a, Pb + al * S, aj, 1);
            stage_a_store<T, NN, +1>(a, Qb + al * S, aj, 1);
        }
        __syncthreads();
        if (hb) {
            cplx<T> u[R1];
            stage_b_load<T, NN>(u, Qb + bl * S, bj, 1);
            stage_b<T, NN, +1>(u, w);
            stage_b_store<T, NN>(u, Qb + bl * S, bj, 1);
        }
        __syncthreads();
        // inverse along m1 (lines n3, elements m1 at stride S): Q -> P, stage B to memory
        if (ha) {
            cplx<T> a[R0];
            stage_a_load<T, NN>(a, Qb + al, aj, S);
            stage_a_store<T, NN, +1>(a, Pb + al, aj, S);
        }
        __syncthreads();
        if (hb) {
            cplx<T> u[R1];
            stage_b_load<T, NN>(u, Pb + bl, bj, S);
            stage_b<T, NN, +1>(u, w);
            cplx<T>* dst = X + (size_t)slot * B.ng + (size_t)m2i * NN + bl;
#pragma unroll
            for (int r = 0; r < R1; ++r) store_nt<T>(dst + (size_t)(bj + r * R0) * rs, u[r]);
        }
        cplx<T>* t = Pb;
        Pb = Qb;
        Qb = t;
    }
    if (B.parseval || deriv_only) {
        constexpr int P2 = NT & (NT - 1) ? (NT >= 256 ? 256 : 128) : NT;   // power of two <= NT
        static_assert(P2 <= NT && 2 * P2 >= NT, "reduction fold");
        __syncthreads();
        red[tid] = acc;
        __syncthreads();
        if (tid < NT - P2) red[tid] += red[tid + P2];
        __syncthreads();
        for (int h = P2 / 2; h > 0; h >>= 1) {
            if (tid < h) red[tid] += red[tid + h];
            __syncthreads();
        }
        if (tid == 0) parts[bid] = red[0];
    }
}

template <typename T, int NN>
__global__ void __launch_bounds__(P2S<NN>::NT) pass2s_kernel(PairBatch B, cplx<T>* __restrict__ X, const cplx<T>* __restrict__ twg, double* __restrict__ parts, int deriv_only) {
    pass2s_body<T, NN>(B, X, twg, parts, deriv_only, (int)blockIdx.x);
}

// ---------------------------------------------------------------------------
// pass 3
// ---------------------------------------------------------------------------
template <typename T, int NN>
__global__ void __launch_bounds__(kFftThreads) pass3_kernel(PairBatch B, const cplx<T>* __restrict__ X,
                                                            cplx<T>* __restrict__ Wpart, cplx<T>* __restrict__ W,
                                                            const cplx<T>* __restrict__ twg) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* plane = tw + 3 * kMaxN;
    constexpr int ACC0 = (kMaxN * kMaxN + kFftThreads - 1) / kFftThreads;
    constexpr int ACC = NN > 0 ? (NN * NN + kFftThreads - 1) / kFftThreads : ACC0;
    const Dims<NN> D(B);
    const int N2 = D.n2, N3 = D.n3, S = N3 + 1;
    const int plane_sz = N2 * N3;
    const int nA = D.n1 * B.nout * B.splits;
    const int nn = B.nocc * B.nout;
    const int first_full = B.b0 + (B.diag ? 1 : 0);
    const int full_base = B.diag ? B.ntri : 0;
    load_twiddles<T>(tw, twg);
    cplx<T> acc[ACC];
#pragma unroll
    for (int t = 0; t < ACC; ++t) acc[t] = mk<T>(T(0), T(0));

    // one term: acc += partner(plane) * (conj?)(IDFT_m2 X[slot] plane)
    auto term = [&](int slot, bool conj_v, const cplx<T>* partner, int n1) {
        const cplx<T>* src = X + (size_t)slot * B.ng + (size_t)n1 * plane_sz;
    #pragma unroll
    for (int e = threadIdx.x; e < plane_sz; e += kFftThreads) {
            const int m2 = e / N3, n3 = e - m2 * N3;
            plane[m2 * S + n3] = src[e];
        }
        __syncthreads();
        lines<T, NN, +1>(N2, plane, N3, S, 1, tw + kMaxN);
#pragma unroll
        for (int t = 0; t < ACC; ++t) {
            const int e = threadIdx.x + t * kFftThreads;
            if (e < plane_sz) {
                const int n2 = e / N3, n3 = e - n2 * N3;
                cplx<T> v = plane[n2 * S + n3];
                if (conj_v) v.y = -v.y;
                const cplx<T> w = partner[e];
                acc[t] = mk<T>(acc[t].x + w.x * v.x - w.y * v.y, acc[t].y + w.x * v.y + w.y * v.x);
            }
        }
        __syncthreads();
    };

    if ((int)blockIdx.x < nA) {
        // a-side: W~_{j a}(plane n1) partial over a slice of the (b, i) sum
        const int n1 = blockIdx.x % D.n1;
        const int j = (blockIdx.x / D.n1) % B.nout;
        const int s = blockIdx.x / (D.n1 * B.nout);
        const int total = B.nb * B.nocc;
        const int chunk = (total + B.splits - 1) / B.splits;
        const int q0 = s * chunk;
        const int q1 = min(total, q0 + chunk);
        for (int q = q0; q < q1; ++q) {
            const int bb = B.b0 + q / B.nocc, i = q % B.nocc;
            int slot;
            bool cj = false;
            if (B.diag && bb == B.a) {
                if (i <= j) slot = tri_index(i, j, B.nocc);
                else {
                    slot = tri_index(j, i, B.nocc);
                    cj = true;
                }
            } else {
                slot = full_base + (bb - first_full) * nn + i * B.nout + j;
            }
            const cplx<T>* pi = static_cast<const cplx<T>*>(B.accp) + ((size_t)bb * B.kstride + i) * B.ng +
                                (size_t)n1 * plane_sz;
            term(slot, cj, pi, n1);
        }
        cplx<T>* out = Wpart + ((size_t)s * B.nout + j) * B.ng + (size_t)n1 * plane_sz;
#pragma unroll
        for (int t = 0; t < ACC; ++t) {
            const int e = threadIdx.x + t * kFftThreads;
            if (e < plane_sz) out[e] = acc[t];
        }
    } else {
        // b-side (reuse only): W~_{i b}(plane n1) += sum_j psi~_{j a} conj(Vt_ij)
        const int g = blockIdx.x - nA;
        const int n1 = g % D.n1;
        const int i = (g / D.n1) % B.nocc;
        const int blk = g / (D.n1 * B.nocc);
        const int bb = first_full + blk;
        for (int j = 0; j < B.nocc; ++j) {
            const int slot = full_base + blk * nn + i * B.nout + j;
            const cplx<T>* pj = static_cast<const cplx<T>*>(B.outp) + (size_t)j * B.ng + (size_t)n1 * plane_sz;
            term(slot, true, pj, n1);
        }
        cplx<T>* out = W + ((size_t)bb * B.kstride + i) * B.ng + (size_t)n1 * plane_sz;
#pragma unroll
        for (int t = 0; t < ACC; ++t) {
            const int e = threadIdx.x + t * kFftThreads;
            if (e < plane_sz) out[e] = cadd<T>(out[e], acc[t]);
        }
    }
}

// ---------------------------------------------------------------------------
// pass 3, fused form for compile-time cubic grids
// ---------------------------------------------------------------------------
// One workgroup owns an x-plane n1, a block of WB adjacent n3 columns (WB
// complex values = 128 bytes, one cache line per row) and a slice of the
// (b, i) pairs of the batch.  For each (b, i) it loads the column block of the
// potentials of all output orbitals j at once, runs one batched inverse FFT
// along m2 over JC * WB lines, then
//   a-side  acc_j += psi~_{i b} Vt_ij            (registers, all j of the slice)
//   b-side  W~_{i b} += sum_j psi~_{j a} conj(Vt_ij)   (conjugate-pair reuse)
// so every stored potential is read from device memory once and the partner
// orbital psi~_{i b} once per (b, i) rather than once per j.
constexpr int kPass3Threads = 1024;   // fused pass 3: 16 waves, a few rows per thread
constexpr int kReduceThreads = 256;   // W reduction over the pass-3 splits

constexpr int colblock(int n, int elem) {
    int w = 128 / elem;
    while (w > 1 && n % w != 0) --w;
    return w;
}

// s_waitcnt operand that waits until at most n vector-memory operations are in flight
// and leaves the export and LDS/scalar counters alone (gfx9 encoding: vmcnt bits 3:0
// and 15:14, expcnt 6:4, lgkmcnt 11:8)
constexpr int waitcnt_vm(int n) { return (n & 15) | (7 << 4) | (15 << 8) | (((n >> 4) & 3) << 14); }

constexpr int pow2_at_least(int n) {
    int p = 1;
    while (p < n) p *= 2;
    return p;
}

template <typename T, int NN, int JC>
__device__ __forceinline__ void pass3f_body(const PairBatch& B, const cplx<T>* __restrict__ X, cplx<T>* __restrict__ Wpart, cplx<T>* __restrict__ W, const cplx<T>* __restrict__ twg, const int bid) {
    constexpr int WB = colblock(NN, (int)sizeof(cplx<T>));
    constexpr int NCB = NN / WB;
    constexpr int LN = JC * WB;                      // FFT lines of the tile: (j, column)
    constexpr int LNP = pow2_at_least(LN);           // padded line count (divides the thread count)
    static_assert(LNP <= kPass3Threads, "tile lines exceed the workgroup");
    constexpr int RPI = kPass3Threads / LNP;           // rows per sweep of the workgroup
    constexpr int PT = (NN + RPI - 1) / RPI;         // rows per thread
    constexpr int PLANE = NN * NN;
    constexpr int BP = NN * WB;                      // points of one column block
    constexpr int BPT = (BP + kPass3Threads - 1) / kPass3Threads;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* tile = tw + 3 * kMaxN;                  // tile[m2][LNP]
    const int n1 = bid % NN;
    const int cb = (bid / NN) % NCB;
    const int s = bid / (NN * NCB);
    const int c0 = cb * WB;
    const int nocc = B.nocc, nout = B.nout;
    const int nn = nocc * nout;
    const int total = B.nb * nocc;
    const int chunk = (total + B.splits - 1) / B.splits;
    const int q0 = s * chunk;
    const int q1 = min(total, q0 + chunk);
    const int first_full = B.b0 + (B.diag ? 1 : 0);
    const int full_base = B.diag ? B.ntri : 0;
    // this thread's fixed (orbital, column) lane and first row
    const int lane = threadIdx.x % LNP;
    const int r0 = threadIdx.x / LNP;
    const int jl = lane / WB;
    const int w = lane - jl * WB;
    const bool active = lane < LN && jl < nout;
    load_twiddles<T>(tw, twg);
    const size_t plane_off = (size_t)n1 * PLANE + c0 + w;
    // stored slot of (b, i; jl, a) for summed pair q = (b - b0) nocc + i, and whether it
    // holds the conjugate (lower triangle of the diagonal block)
    auto slot_of = [&](int q, bool& cj) {
        const int bb = B.b0 + q / nocc, i = q - (q / nocc) * nocc;
        cj = false;
        if (B.diag && bb == B.a) {
            cj = jl < i;
            return cj ? tri_index(jl, i, nocc) : tri_index(i, jl, nocc);
        }
        return full_base + (bb - first_full) * nn + i * nout + jl;
    };
    auto load_column = [&](int q, cplx<T>* dst) {
        bool cj;
        const cplx<T>* src = X + (size_t)(active ? slot_of(q, cj) : 0) * B.ng + plane_off;
#pragma unroll
        for (int t = 0; t < PT; ++t) {
            const int m2 = r0 + t * RPI;
            dst[t] = (active && m2 < NN) ? src[(size_t)m2 * NN] : mk<T>(T(0), T(0));
        }
    };
    // Register prefetch (8 orbital lanes; 16 lanes double the per-thread rows and would
    // spill): the next pair's column is loaded while this pair is transformed, and the
    // a-side orbital at this thread's points, the same for every summed pair, is held.
    constexpr bool PF = JC <= 8;
    const cplx<T>* pa_src = static_cast<const cplx<T>*>(B.outp) + (size_t)(active ? jl : 0) * B.ng + plane_off;
    cplx<T> pa[PT];
    if constexpr (PF) {
#pragma unroll
        for (int t = 0; t < PT; ++t) {
            const int n2 = r0 + t * RPI;
            pa[t] = (active && n2 < NN) ? pa_src[(size_t)n2 * NN] : mk<T>(T(0), T(0));
        }
    }
    cplx<T> acc[PT], xn[PT];
#pragma unroll
    for (int t = 0; t < PT; ++t) acc[t] = mk<T>(T(0), T(0));
    if (PF && q0 < q1) load_column(q0, xn);

    for (int q = q0; q < q1; ++q) {
        const int bb = B.b0 + q / nocc, i = q - (q / nocc) * nocc;
        const bool bside = B.reuse && !(B.diag && bb == B.a);
        bool cj;
        (void)slot_of(q, cj);
        if constexpr (!PF) load_column(q, xn);
        __syncthreads();
#pragma unroll
        for (int t = 0; t < PT; ++t) {
            const int m2 = r0 + t * RPI;
            if (m2 < NN) tile[m2 * LNP + lane] = xn[t];
        }
        // in flight during this pair's transform: the next pair's column, this pair's
        // b-side orbital values and its W block
        if (PF && q + 1 < q1) load_column(q + 1, xn);
        const cplx<T>* ui_src = static_cast<const cplx<T>*>(B.accp) + ((size_t)bb * B.kstride + i) * B.ng + plane_off;
        cplx<T> ui[PT];
        if constexpr (PF) {
#pragma unroll
            for (int t = 0; t < PT; ++t) {
                const int n2 = r0 + t * RPI;
                ui[t] = (active && n2 < NN) ? ui_src[(size_t)n2 * NN] : mk<T>(T(0), T(0));
            }
        }
        cplx<T>* wout = W + ((size_t)bb * B.kstride + i) * B.ng + (size_t)n1 * PLANE + c0;
        cplx<T> wv[BPT];
        if (PF && bside) {
#pragma unroll
            for (int t = 0; t < BPT; ++t) {
                const int e = threadIdx.x + t * kPass3Threads;
                const int n2 = e / WB, ww = e - n2 * WB;
                wv[t] = e < BP ? wout[(size_t)n2 * NN + ww] : mk<T>(T(0), T(0));
            }
        }
        __syncthreads();
        fft_lines<T, NN, +1, LNP, kPass3Threads>(tile, LNP, LNP, 1, tw + kMaxN);
        if (active) {
#pragma unroll
            for (int t = 0; t < PT; ++t) {
                const int n2 = r0 + t * RPI;
                if (n2 < NN) {
                    cplx<T> v = tile[n2 * LNP + lane];
                    if (cj) v.y = -v.y;
                    const cplx<T> u = PF ? ui[t] : ui_src[(size_t)n2 * NN];
                    acc[t] = mk<T>(acc[t].x + u.x * v.x - u.y * v.y, acc[t].y + u.x * v.y + u.y * v.x);
                    if (bside) {
                        const cplx<T> o = PF ? pa[t] : pa_src[(size_t)n2 * NN];
                        tile[n2 * LNP + lane] = mk<T>(o.x * v.x + o.y * v.y, o.y * v.x - o.x * v.y);  // o conj(v)
                    }
                }
            }
        }
        if (bside) {
            __syncthreads();
#pragma unroll
            for (int t = 0; t < BPT; ++t) {
                const int e = threadIdx.x + t * kPass3Threads;
                if (e < BP) {
                    const int n2 = e / WB, ww = e - n2 * WB;
                    cplx<T> sum = PF ? wv[t] : wout[(size_t)n2 * NN + ww];
                    for (int j = 0; j < nocc; ++j) sum = cadd<T>(sum, tile[n2 * LNP + j * WB + ww]);
                    wout[(size_t)n2 * NN + ww] = sum;
                }
            }
        }
    }
    if (active) {
        cplx<T>* out = Wpart + ((size_t)s * nout + jl) * B.ng + plane_off;
#pragma unroll
        for (int t = 0; t < PT; ++t) {
            const int n2 = r0 + t * RPI;
            if (n2 < NN) out[(size_t)n2 * NN] = acc[t];
        }
    }
}

template <typename T, int NN, int JC>
__global__ void __launch_bounds__(kPass3Threads) pass3f_kernel(PairBatch B, const cplx<T>* __restrict__ X, cplx<T>* __restrict__ Wpart, cplx<T>* __restrict__ W, const cplx<T>* __restrict__ twg) {
    pass3f_body<T, NN, JC>(B, X, Wpart, W, twg, (int)blockIdx.x);
}

// Pass 3 for the compiled cubic sizes with at most 8 output orbitals: the column
// block transform along m2 as two-stage lines, stage A fed from the prefetched
// registers and stage B kept in registers, where the a-side sum (and the b-side
// product) is formed.  Three LDS buffers rotate between summed pairs, so that the
// b-side sum over a pair's partner orbitals is read one pair later, behind the
// next pair's only barrier: per pair one barrier and 2 LDS accesses per point,
// against six barriers and 6 accesses in pass3f_kernel.  The column block is 128
// bytes wide (16 complex64 or 8 complex128 columns).  The next pair's column is
// loaded in one of three forms: 16 bytes per lane through lane pairs (complex64 with
// an even column block and stage-A radix), 8 bytes per lane (other complex64 grids),
// or, in complex128, with every load issued on every path so that stage B waits
// exactly for this pair's summed orbital.
template <typename T, int NN>
struct P3S {
    static constexpr int R0 = Split2<NN>::R0, R1 = Split2<NN>::R1;
    static constexpr int WB = colblock(NN, (int)sizeof(cplx<T>));
    static constexpr int LN = 8 * WB;                   // lines (j, column) of the tile
    static constexpr int LNP = pow2_at_least(LN);       // padded line count (tile row)
    static constexpr int NA = LNP * R1, NBI = LNP * R0;
    static constexpr int NT = ((NA > NBI ? NA : NBI) + 63) / 64 * 64;
};

template <typename T, int NN>
__device__ __forceinline__ void pass3s_body(const PairBatch& B, const cplx<T>* __restrict__ X, cplx<T>* __restrict__ Wpart, cplx<T>* __restrict__ W, const cplx<T>* __restrict__ twg, const int bid) {
    using C = P3S<T, NN>;
    constexpr int R0 = C::R0, R1 = C::R1, WB = C::WB, LN = C::LN, LNP = C::LNP, NT = C::NT;
    constexpr int NCB = NN / WB;
    constexpr int PLANE = NN * NN;
    constexpr int BP = NN * WB;                         // points of one column block
    constexpr int BPT = (BP + NT - 1) / NT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* buf0 = reinterpret_cast<cplx<T>*>(smem_raw);
    const int n1 = bid % NN;
    const int cb = (bid / NN) % NCB;
    const int s = bid / (NN * NCB);
    const int c0 = cb * WB;
    const int nocc = B.nocc, nout = B.nout;
    const int nn = nocc * nout;
    const int total = B.nb * nocc;
    const int chunk = (total + B.splits - 1) / B.splits;
    const int q0 = s * chunk;
    const int q1 = min(total, q0 + chunk);
    const int first_full = B.b0 + (B.diag ? 1 : 0);
    const int full_base = B.diag ? B.ntri : 0;
    const int tid = threadIdx.x;
    const int line = tid % LNP;                         // (orbital jl, column w) of both stages
    const int sj = tid / LNP;                           // stage A index (< R1) or stage B index (< R0)
    const bool ha = tid < C::NA, hb = tid < C::NBI;
    const int jl = line / WB;
    const int w = line - jl * WB;
    const bool active = line < LN && jl < nout;
    const size_t plane_off = (size_t)n1 * PLANE + c0 + w;
    // stored slot of (bb, i; jl, a) and whether it holds the conjugate (lower triangle
    // of the diagonal block); the summed pairs q = (bb - b0) nocc + i are walked
    // incrementally, without divisions
    auto slot_of = [&](int bb, int i, bool& cj) {
        cj = false;
        if (B.diag && bb == B.a) {
            cj = jl < i;
            return cj ? tri_index(jl, i, nocc) : tri_index(i, jl, nocc);
        }
        return full_base + (bb - first_full) * nn + i * nout + jl;
    };
    // stage A inputs: rows m2 = sj + r R1 of this line
    cplx<T> xn[R0];
    auto load_column = [&](int bb, int i) {
        bool cj;
        const cplx<T>* src = X + (size_t)(active ? slot_of(bb, i, cj) : 0) * B.ng + plane_off;
#pragma unroll
        for (int r = 0; r < R0; ++r) xn[r] = (ha && active) ? load_nt<T>(src + (size_t)(sj + r * R1) * NN) : mk<T>(T(0), T(0));
    };
    // Complex64 with an even column block and an even stage-A radix loads the column 16
    // bytes per lane: of two adjacent lanes (adjacent columns w, w + 1 of one orbital),
    // the even one loads both columns of row sj + 2m R1 and the odd one both columns of
    // row sj + (2m + 1) R1, and one swap between the two lanes (DPP) leaves each with
    // its own column of both rows.  Half the load instructions, each moving 16 bytes.
    constexpr bool kWide = sizeof(T) == 4 && WB % 2 == 0 && R0 % 2 == 0;
    typedef T w4 __attribute__((ext_vector_type(4)));
    w4 raw[R0 / 2];
    const int odd = line & 1;
    auto load_column_wide = [&](int bb, int i) {
        bool cj;
        const cplx<T>* src = X + (size_t)(active ? slot_of(bb, i, cj) : 0) * B.ng + plane_off - odd;
#pragma unroll
        for (int m = 0; m < R0 / 2; ++m) {
            const w4 z = {T(0), T(0), T(0), T(0)};
            raw[m] = (ha && active) ? __builtin_nontemporal_load(reinterpret_cast<const w4*>(
                                          src + (size_t)(sj + (2 * m + odd) * R1) * NN))
                                    : z;
        }
    };
    // with every lane of the wave active: xn[2m] is row sj + 2m R1, xn[2m + 1] row
    // sj + (2m + 1) R1 of this lane's column
    auto unpack_column = [&]() {
        if constexpr (kWide)
#pragma unroll
        for (int m = 0; m < R0 / 2; ++m) {
            const T sx = odd ? raw[m].x : raw[m].z, sy = odd ? raw[m].y : raw[m].w;
            const T rx = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(sx), 0xB1, 0xF, 0xF, false));
            const T ry = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(sy), 0xB1, 0xF, 0xF, false));
            xn[2 * m] = odd ? mk<T>(rx, ry) : mk<T>(raw[m].x, raw[m].y);
            xn[2 * m + 1] = odd ? mk<T>(raw[m].z, raw[m].w) : mk<T>(rx, ry);
        }
    };
    // In complex128 (half the waves of the complex64 kernel per CU, so exposed waits
    // cost more) the loop waits exactly: there every thread issues every load (a thread
    // without a stage-A item, or on a line past the output orbitals, reads rows of slot
    // 0 that it never uses), the loads that follow the summed orbital are the same on
    // every path, and stage B waits for that orbital alone.  Per paper-sized build,
    // complex128 pass 3 took 670-687 ms against 686-730 in same-session runs; in
    // complex64 the extra loads cost more than the exact wait gains (395 -> 408 ms).
    constexpr bool kExact = sizeof(T) == 8;
    const int sa = ha ? sj : 0, sb = hb ? sj : 0;
    auto load_column_all = [&](int bb, int i) {
        bool cj;
        const cplx<T>* src = X + (size_t)(ha && active ? slot_of(bb, i, cj) : 0) * B.ng + plane_off;
#pragma unroll
        for (int r = 0; r < R0; ++r) xn[r] = load_nt<T>(src + (size_t)(sa + r * R1) * NN);
    };
    // stage B rows n2 = sj + r R0: twiddles, the a-side partner orbital (held) and the sums
    const bool bact = hb && active;
    cplx<T> tw[R1 - 1], pa[R1], acc[R1];
    const cplx<T>* pa_src = static_cast<const cplx<T>*>(B.outp) + (size_t)(active ? jl : 0) * B.ng + plane_off;
    if (hb) stage_b_twiddles<T, NN>(tw, twg + kMaxN, sj);
    else {
#pragma unroll
        for (int r = 0; r < R1 - 1; ++r) tw[r] = mk<T>(T(0), T(0));
    }
#pragma unroll
    for (int r = 0; r < R1; ++r) {
        pa[r] = bact && B.reuse ? pa_src[(size_t)(sj + r * R0) * NN] : mk<T>(T(0), T(0));
        acc[r] = mk<T>(T(0), T(0));
    }
    int bb = B.b0 + q0 / nocc, i = q0 - (q0 / nocc) * nocc;
    if (q0 < q1) {
        if constexpr (kWide) load_column_wide(bb, i);
        else load_column(bb, i);
    }
    // The twiddle and held-orbital loads above sit in branches; without a wait here the
    // compiler's counter bookkeeping carries them into the loop as possibly outstanding,
    // and its waits inside the loop then cover every load in flight.
    __builtin_amdgcn_s_waitcnt(0);
    // Pb: this pair's buffer; Rb: the previous pair's, whose b-side products are summed
    // behind this pair's barrier (written before it, rewritten two pairs later, after
    // the barrier that follows the sum)
    cplx<T>* Pb = buf0;
    cplx<T>* Rb = buf0 + 2 * NN * LNP;
    bool pending = false;                               // the previous pair's b-side sum is due
    cplx<T> wprev[BPT], wv[BPT];
    cplx<T>* wout_prev = W;
    auto bside_sum = [&](const cplx<T>* Sb, const cplx<T>* wv_in, cplx<T>* dst) {
#pragma unroll
        for (int t = 0; t < BPT; ++t) {
            const int e = tid + t * NT;
            if (e < BP) {
                const int n2 = e / WB, ww = e - n2 * WB;
                cplx<T> sum = wv_in[t];
                for (int j = 0; j < nocc; ++j) sum = cadd<T>(sum, Sb[n2 * LNP + j * WB + ww]);
                store_nt<T>(dst + (size_t)n2 * NN + ww, sum);
            }
        }
    };
    for (int q = q0; q < q1; ++q) {
        const int bn = i + 1 == nocc ? bb + 1 : bb, in = i + 1 == nocc ? 0 : i + 1;   // pair q + 1
        const bool bside = B.reuse && !(B.diag && bb == B.a);
        bool cj;
        (void)slot_of(bb, i, cj);
        // this pair's column and the last pair's W block were loaded a pair ago: one wait
        // for everything in flight (in complex128 the only wait for them; in complex64
        // stage B's wait for the summed orbital has already covered them)
        __builtin_amdgcn_s_waitcnt(0);
        if constexpr (kWide) unpack_column();
        if (ha) {
            cplx<T> a[R0];
#pragma unroll
            for (int r = 0; r < R0; ++r) a[r] = xn[r];
            stage_a_store<T, NN, +1>(a, Pb + line, sj, LNP);
        }
        const cplx<T>* ui_src = static_cast<const cplx<T>*>(B.accp) + ((size_t)bb * B.kstride + i) * B.ng + plane_off;
        cplx<T>* wout;
        cplx<T> ui[R1];
        if constexpr (kExact) {
            // in flight during this pair's transform: this pair's summed orbital and the
            // next pair's column (the last pair reloads its own), issued unconditionally
            // and in that order; every address is in bounds
#pragma unroll
            for (int r = 0; r < R1; ++r) ui[r] = load_nt<T>(ui_src + (size_t)(sb + r * R0) * NN);
            const bool more = q + 1 < q1;
            load_column_all(more ? bn : bb, more ? in : i);
            __syncthreads();
            // The summed orbital has arrived once at most the R0 column loads issued
            // after it are in flight (loads complete in order, every path issues the
            // same loads, and no store has been issued since the wait at the top of the
            // pair), so stage B waits for nothing else; the column stays in flight
            // until the next pair.
            __builtin_amdgcn_s_waitcnt(waitcnt_vm(R0));
            if (pending) bside_sum(Rb, wprev, wout_prev);
            // this pair's W block, summed into one pair later, straight into the
            // registers the sum above has just read (no copy that would wait for it);
            // only b-side pairs have one (without conjugate-pair reuse W is not indexed
            // by (b, i) at all), and this load follows the exact wait above, so it may
            // be conditional
            wout = W + ((size_t)bb * B.kstride + i) * B.ng + (size_t)n1 * PLANE + c0;
            if (bside) {
#pragma unroll
                for (int t = 0; t < BPT; ++t) {
                    const int e = tid + t * NT < BP ? tid + t * NT : (tid + t * NT) % BP;
                    const int n2 = e / WB, ww = e - n2 * WB;
                    wprev[t] = load_nt<T>(wout + (size_t)n2 * NN + ww);
                }
            }
        } else {
            // in flight during this pair's transform: the next pair's column, this
            // pair's summed orbital and its W block (stage B's first use of the summed
            // orbital waits for all of them: the b-side stores below are in flight too)
            if (q + 1 < q1) {
                if constexpr (kWide) load_column_wide(bn, in);
                else load_column(bn, in);
            }
#pragma unroll
            for (int r = 0; r < R1; ++r) ui[r] = bact ? load_nt<T>(ui_src + (size_t)(sj + r * R0) * NN) : mk<T>(T(0), T(0));
            wout = W + ((size_t)bb * B.kstride + i) * B.ng + (size_t)n1 * PLANE + c0;
#pragma unroll
            for (int t = 0; t < BPT; ++t) {
                const int e = tid + t * NT;
                const int n2 = e / WB, ww = e - n2 * WB;
                wv[t] = bside && e < BP ? load_nt<T>(wout + (size_t)n2 * NN + ww) : mk<T>(T(0), T(0));
            }
            __syncthreads();
            if (pending) bside_sum(Rb, wprev, wout_prev);
        }
        if (hb) {
            cplx<T> y[R1];
            stage_b_load<T, NN>(y, Pb + line, sj, LNP);
            stage_b<T, NN, +1>(y, tw);
            if (active) {
#pragma unroll
                for (int r = 0; r < R1; ++r) {
                    cplx<T> v = y[r];
                    if (cj) v.y = -v.y;
                    acc[r] = mk<T>(acc[r].x + ui[r].x * v.x - ui[r].y * v.y, acc[r].y + ui[r].x * v.y + ui[r].y * v.x);
                    // b-side product o conj(v), in this item's own rows of the buffer
                    if (bside) Pb[(sj + r * R0) * LNP + line] = mk<T>(pa[r].x * v.x + pa[r].y * v.y,
                                                                     pa[r].y * v.x - pa[r].x * v.y);
                }
            }
        }
        pending = bside;
        if constexpr (!kExact) {
#pragma unroll
            for (int t = 0; t < BPT; ++t) wprev[t] = wv[t];
        }
        wout_prev = wout;
        Rb = Pb;
        Pb = Pb == buf0 + 2 * NN * LNP ? buf0 : Pb + NN * LNP;
        bb = bn;
        i = in;
    }
    if (pending) {
        __syncthreads();
        bside_sum(Rb, wprev, wout_prev);
    }
    if (bact) {
        cplx<T>* out = Wpart + ((size_t)s * nout + jl) * B.ng + plane_off;
#pragma unroll
        for (int r = 0; r < R1; ++r) out[(size_t)(sj + r * R0) * NN] = acc[r];
    }
}

template <typename T, int NN>
__global__ void __launch_bounds__((P3S<T, NN>::NT)) pass3s_kernel(PairBatch B, const cplx<T>* __restrict__ X, cplx<T>* __restrict__ Wpart, cplx<T>* __restrict__ W, const cplx<T>* __restrict__ twg) {
    pass3s_body<T, NN>(B, X, Wpart, W, twg, (int)blockIdx.x);
}

template <typename T>
__device__ __forceinline__ void wreduce_body(const PairBatch& B, const cplx<T>* __restrict__ Wpart,
                                             cplx<T>* __restrict__ W, const int bid) {
    const size_t n = (size_t)bid * kReduceThreads + threadIdx.x;
    const size_t tot = (size_t)B.nout * B.ng;               // partials: [split][nout][ng]
    if (n < tot) {
        cplx<T>* w = W + B.woff;                            // the output orbitals at k_a
        cplx<T> acc = w[n];
        for (int s = 0; s < B.splits; ++s) acc = cadd<T>(acc, Wpart[(size_t)s * tot + n]);
        w[n] = acc;
    }
}

template <typename T>
__global__ void __launch_bounds__(kReduceThreads) wreduce_kernel(PairBatch B, const cplx<T>* __restrict__ Wpart,
                                                                 cplx<T>* __restrict__ W) {
    wreduce_body<T>(B, Wpart, W, (int)blockIdx.x);
}

template <typename T>
__global__ void fill_zero_kernel(cplx<T>* p, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = mk<T>(T(0), T(0));
}

__global__ void fill_zero_f64_kernel(double* p, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0.0;
}

template <typename T>
size_t lds_plane_bytes(int rows, int cols) {
    return sizeof(cplx<T>) * (3 * kMaxN + (size_t)rows * (cols + 1));
}

// compile-time specialisations of cubic grids; 0 = sizes read at run time
inline int specialised(const PairBatch& B) {
    if (B.N1 != B.N2 || B.N2 != B.N3) return 0;
    switch (B.N1) {
        case 24: case 30: case 32: case 36: case 40: case 48: return B.N1;
        default: return 0;
    }
}

#define OCCRIK_DISPATCH(NNV, CALL)          \
    switch (NNV) {                          \
        case 24: { constexpr int NN = 24; CALL; } break; \
        case 30: { constexpr int NN = 30; CALL; } break; \
        case 32: { constexpr int NN = 32; CALL; } break; \
        case 36: { constexpr int NN = 36; CALL; } break; \
        case 40: { constexpr int NN = 40; CALL; } break; \
        case 48: { constexpr int NN = 48; CALL; } break; \
        default: { constexpr int NN = 0; CALL; } break;  \
    }

template <typename T, int NN>
void launch_pass1g(const PairBatch& B, const cplx<T>* psi, cplx<T>* X, const cplx<T>* tw, hipStream_t s) {
    if constexpr (NN > 0) {
        using C = P1G<NN>;
        const size_t lds = 2 * sizeof(cplx<T>) * NN * C::S;
        const int rows = pass1_rows(B, NN);
        const dim3 grid((unsigned)((size_t)NN * pass1_groups(B, rows)));
        if (rows == kPass1Rows)
            hipLaunchKernelGGL((pass1g_kernel<T, NN, kPass1Rows>), grid, dim3(pass1g_threads<T, NN, kPass1Rows>()), lds, s,
                               B, psi, X, tw);
        else
            hipLaunchKernelGGL((pass1g_kernel<T, NN, 1>), grid, dim3(C::NT), lds, s, B, psi, X, tw);
    }
}

template <typename T, int NN>
void launch_pass2s(const PairBatch& B, cplx<T>* X, const cplx<T>* tw, double* parts, int deriv_only, unsigned grid,
                   hipStream_t s) {
    if constexpr (NN > 0) {
        using C = P2S<NN>;
        const size_t lds = sizeof(double) * C::NT + 2 * sizeof(cplx<T>) * NN * C::S;
        hipLaunchKernelGGL((pass2s_kernel<T, NN>), dim3(grid), dim3(C::NT), lds, s, B, X, tw, parts, deriv_only);
    }
}

template <typename T, int NN>
void launch_pass3s(const PairBatch& B, const cplx<T>* X, cplx<T>* Wpart, cplx<T>* W, const cplx<T>* tw,
                   hipStream_t s) {
    if constexpr (NN > 0) {
        using C = P3S<T, NN>;
        const unsigned grid = (unsigned)((size_t)NN * (NN / C::WB) * B.splits);
        const size_t lds = 3 * sizeof(cplx<T>) * NN * C::LNP;
        hipLaunchKernelGGL((pass3s_kernel<T, NN>), dim3(grid), dim3(C::NT), lds, s, B, X, Wpart, W, tw);
    }
}

}  // namespace

size_t kcache_tables(int M1, int M2, int M3) { return (size_t)(2 * M1 - 1) * (2 * M2 - 1) * (2 * M3 - 1); }

template <typename T>
hipError_t launch_kcache(const PairBatch& B, void* out, hipStream_t s) {
    const int nq = (int)kcache_tables(B.M1, B.M2, B.M3);
    const size_t nv = (size_t)nq * B.ng;
    const unsigned grid = (unsigned)std::min<size_t>((nv + 255) / 256, 65536);
    hipLaunchKernelGGL((kcache_kernel<T>), dim3(grid), dim3(256), 0, s, B, static_cast<T*>(out), nq);
    return hipGetLastError();
}

int pair_groups(const PairBatch& B) {
    const int nn = B.nocc * B.nout;
    const int gd = B.diag ? (B.ntri + B.group - 1) / B.group : 0;
    const int nfull = B.nb - (B.diag ? 1 : 0);
    return gd + nfull * ((nn + B.group - 1) / B.group);
}

template <typename T>
hipError_t launch_pass1(const PairBatch& B, const cplx<T>* psi, cplx<T>* X, const cplx<T>* tw, hipStream_t s) {
    if constexpr (std::is_same_v<T, float>)
        if (B.regfft & REGFFT_PASS1) return launch_pass1_reg(B, psi, X, s);
    if (const int nnv = specialised(B)) {
        OCCRIK_DISPATCH(nnv, (launch_pass1g<T, NN>(B, psi, X, tw, s)));
        return hipGetLastError();
    }
    const unsigned grid = (unsigned)((size_t)B.N1 * B.nslots);
    const size_t lds = lds_plane_bytes<T>(B.N2, B.N3);
    OCCRIK_DISPATCH(specialised(B),
                    hipLaunchKernelGGL((pass1_kernel<T, NN>), dim3(grid), dim3(kFftThreads), lds, s, B, psi, X, tw));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pass2(const PairBatch& B, cplx<T>* X, const cplx<T>* tw, double* parts, int deriv_only,
                        hipStream_t s) {
    if (!B.kvals || (B.kcache && deriv_only)) return hipErrorInvalidValue;   // the cache holds f only
    if (!B.kcache) {
        const size_t nv = (size_t)B.nb * B.ng;
        const unsigned kgrid = (unsigned)std::min<size_t>((nv + 255) / 256, 16384);
        hipLaunchKernelGGL((kvals_kernel<T>), dim3(kgrid), dim3(256), 0, s, B, static_cast<T*>(B.kvals), deriv_only);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if constexpr (std::is_same_v<T, float>)
        if (B.regfft & REGFFT_PASS2) return launch_pass2_reg(B, X, parts, deriv_only, s);
    const unsigned grid = (unsigned)((size_t)B.N2 * pair_groups(B));
    if (const int nnv = specialised(B)) {
        OCCRIK_DISPATCH(nnv, (launch_pass2s<T, NN>(B, X, tw, parts, deriv_only, grid, s)));
        return hipGetLastError();
    }
    const size_t lds = lds_plane_bytes<T>(B.N1, B.N3) + sizeof(double) * kFftThreads;
    OCCRIK_DISPATCH(specialised(B), hipLaunchKernelGGL((pass2_kernel<T, NN>), dim3(grid), dim3(kFftThreads), lds, s,
                                                       B, X, tw, parts, deriv_only));
    return hipGetLastError();
}

int pass3_splits(const PairBatch& B, int elem) {
    // at least ~2048 workgroups; then, within twice that split count, the first whose
    // workgroup count is a whole number of rounds over the 256 compute units: the compiled
    // complex64 kernels hold one 1024-thread workgroup per CU, every workgroup walks the
    // same number of pairs, and a last round that fills part of the chip is idle time.
    // The count depends on the batch only through its cap, so a plan's Wpart buffer,
    // sized for its largest batch, holds every smaller batch's partial sums.
    const int target_wg = 2048, cus = 256;
    const int nn = specialised(B);
    const int base_wg = nn > 0 && B.nout <= 16 ? nn * (nn / colblock(nn, elem)) : B.N1 * B.nout;
    const int s0 = (target_wg + base_wg - 1) / base_wg;
    int sp = s0;
    while ((size_t)base_wg * sp % cus != 0 && sp < 2 * s0) ++sp;
    if ((size_t)base_wg * sp % cus != 0) sp = s0;
    return std::max(1, std::min(B.nb * B.nocc, sp));
}

template <typename T>
hipError_t launch_pass3(const PairBatch& B, const cplx<T>* X, const cplx<T>* psi, cplx<T>* Wpart, cplx<T>* W,
                        const cplx<T>* tw, hipStream_t s) {
    if constexpr (std::is_same_v<T, float>)
        if ((B.regfft & REGFFT_PASS3) && B.nout <= 8) return launch_pass3_reg(B, X, psi, Wpart, W, s);
    const int nnv = specialised(B);
    if (nnv > 0 && B.nout <= 8) {
        OCCRIK_DISPATCH(nnv, (launch_pass3s<T, NN>(B, X, Wpart, W, tw, s)));
        return hipGetLastError();
    }
    if (nnv > 0 && B.nout <= 16) {
        // 9-16 output orbitals: 16 orbital lines per column
        constexpr int JC = 16;
        const int wb = colblock(nnv, (int)sizeof(cplx<T>));
        const unsigned grid = (unsigned)((size_t)nnv * (nnv / wb) * B.splits);
        int lnp = 1;
        while (lnp < JC * wb) lnp *= 2;
        const size_t lds = sizeof(cplx<T>) * (3 * kMaxN + (size_t)nnv * lnp);
        OCCRIK_DISPATCH(nnv, if constexpr (NN > 0) hipLaunchKernelGGL((pass3f_kernel<T, NN, JC>), dim3(grid),
                                                                   dim3(kPass3Threads), lds, s, B, X, Wpart, W,
                                                                   tw));
        return hipGetLastError();
    }
    const int nfull_b = B.reuse ? B.nb - (B.diag ? 1 : 0) : 0;
    const unsigned grid = (unsigned)((size_t)B.N1 * B.nout * B.splits + (size_t)nfull_b * B.nocc * B.N1);
    const size_t lds = lds_plane_bytes<T>(B.N2, B.N3);
    hipLaunchKernelGGL((pass3_kernel<T, 0>), dim3(grid), dim3(kFftThreads), lds, s, B, X, Wpart, W, tw);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_wreduce(const PairBatch& B, const cplx<T>* Wpart, cplx<T>* W, hipStream_t s) {
    const size_t tot = (size_t)B.nout * B.ng;
    hipLaunchKernelGGL(wreduce_kernel<T>, dim3((unsigned)((tot + kReduceThreads - 1) / kReduceThreads)),
                       dim3(kReduceThreads), 0, s, B, Wpart, W);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fused rounds of a ragged batch
// ---------------------------------------------------------------------------
namespace {

// the item of fused workgroup g in `stage`: the last one whose first workgroup is <= g
__device__ __forceinline__ int fused_item(const FusedItem* __restrict__ items, int nitems, int stage, int g) {
    int lo = 0, hi = nitems - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].wg0[stage] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Every workgroup of a fused launch runs one workgroup of one item's own launch, with
// the block size and LDS of the plan's own launcher.
template <typename T, int NN>
__global__ void __launch_bounds__(P1G<NN>::NT) pass1g_fused(const FusedItem* __restrict__ items, int nitems,
                                                            int total) {
    const int g = blockIdx.x;
    if (g >= total) return;
    const FusedItem& it = items[fused_item(items, nitems, 0, g)];
    pass1g_body<T, NN, 1>(it.B, static_cast<const cplx<T>*>(it.psi), static_cast<cplx<T>*>(it.X),
                          static_cast<const cplx<T>*>(it.tw), g - it.wg0[0]);
}

template <typename T, int NN>
__global__ void __launch_bounds__(P2S<NN>::NT) pass2s_fused(const FusedItem* __restrict__ items, int nitems,
                                                            int total) {
    const int g = blockIdx.x;
    if (g >= total) return;
    const FusedItem& it = items[fused_item(items, nitems, 1, g)];
    pass2s_body<T, NN>(it.B, static_cast<cplx<T>*>(it.X), static_cast<const cplx<T>*>(it.tw), it.parts, 0,
                       g - it.wg0[1]);
}

template <typename T, int NN>
__global__ void __launch_bounds__((P3S<T, NN>::NT)) pass3s_fused(const FusedItem* __restrict__ items, int nitems,
                                                                int total) {
    const int g = blockIdx.x;
    if (g >= total) return;
    const FusedItem& it = items[fused_item(items, nitems, 2, g)];
    pass3s_body<T, NN>(it.B, static_cast<const cplx<T>*>(it.X), static_cast<cplx<T>*>(it.Wpart),
                       static_cast<cplx<T>*>(it.W), static_cast<const cplx<T>*>(it.tw), g - it.wg0[2]);
}

template <typename T, int NN>
__global__ void __launch_bounds__(kPass3Threads) pass3f_fused(const FusedItem* __restrict__ items, int nitems,
                                                              int total) {
    const int g = blockIdx.x;
    if (g >= total) return;
    const FusedItem& it = items[fused_item(items, nitems, 2, g)];
    pass3f_body<T, NN, 16>(it.B, static_cast<const cplx<T>*>(it.X), static_cast<cplx<T>*>(it.Wpart),
                           static_cast<cplx<T>*>(it.W), static_cast<const cplx<T>*>(it.tw), g - it.wg0[2]);
}

template <typename T>
__global__ void __launch_bounds__(kReduceThreads) wreduce_fused(const FusedItem* __restrict__ items, int nitems,
                                                                int total) {
    const int g = blockIdx.x;
    if (g >= total) return;
    const FusedItem& it = items[fused_item(items, nitems, 3, g)];
    wreduce_body<T>(it.B, static_cast<const cplx<T>*>(it.Wpart), static_cast<cplx<T>*>(it.W), g - it.wg0[3]);
}

// the pass kernels of one fused stage, with the block size and LDS of the plan's own
// launchers (launch_pass1g, launch_pass2s, launch_pass3s and the 16-line pass 3)
template <typename T, int NN>
void launch_fused_pass(int stage, int nout, const FusedItem* items, int nitems, int total, hipStream_t s) {
    const unsigned grid = (unsigned)total;
    if constexpr (NN > 0) {
        if (stage == 0) {
            using C = P1G<NN>;
            hipLaunchKernelGGL((pass1g_fused<T, NN>), dim3(grid), dim3(C::NT), 2 * sizeof(cplx<T>) * NN * C::S, s,
                               items, nitems, total);
        } else if (stage == 1) {
            using C = P2S<NN>;
            hipLaunchKernelGGL((pass2s_fused<T, NN>), dim3(grid), dim3(C::NT),
                               sizeof(double) * C::NT + 2 * sizeof(cplx<T>) * NN * C::S, s, items, nitems, total);
        } else if (nout <= 8) {
            using C = P3S<T, NN>;
            hipLaunchKernelGGL((pass3s_fused<T, NN>), dim3(grid), dim3(C::NT), 3 * sizeof(cplx<T>) * NN * C::LNP, s,
                               items, nitems, total);
        } else {
            constexpr int lnp = pow2_at_least(16 * colblock(NN, (int)sizeof(cplx<T>)));
            hipLaunchKernelGGL((pass3f_fused<T, NN>), dim3(grid), dim3(kPass3Threads),
                               sizeof(cplx<T>) * (3 * kMaxN + (size_t)NN * lnp), s, items, nitems, total);
        }
    }
}

}  // namespace

bool fusable(const PairBatch& B) {
    return specialised(B) > 0 && B.regfft == 0 && B.kcache && B.kvals && B.nout <= 16 && !B.parseval;
}

void fused_workgroups(const PairBatch& B, int elem, int out[kFusedStages]) {
    const int nn = specialised(B);
    out[0] = nn * pass1_groups(B, 1);                                    // pass1g_fused: one row per group
    out[1] = B.N2 * pair_groups(B);                                      // launch_pass2s
    out[2] = nn * (nn / colblock(nn, elem)) * B.splits;                  // launch_pass3s / pass3f
    out[3] = (int)(((size_t)B.nout * B.ng + kReduceThreads - 1) / kReduceThreads);   // launch_wreduce
}

template <typename T>
hipError_t launch_fused(int stage, const PairBatch& B0, const FusedItem* items, int nitems, unsigned total,
                        hipStream_t s) {
    if (total == 0 || total > (unsigned)INT32_MAX || nitems <= 0 || !fusable(B0) || stage < 0 ||
        stage >= kFusedStages)
        return hipErrorInvalidValue;
    if (stage == 3) {
        hipLaunchKernelGGL((wreduce_fused<T>), dim3(total), dim3(kReduceThreads), 0, s, items, nitems, (int)total);
    } else {
        OCCRIK_DISPATCH(specialised(B0), (launch_fused_pass<T, NN>(stage, B0.nout, items, nitems, (int)total, s)));
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill_zero(cplx<T>* p, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill_zero_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_fill_zero_f64(double* p, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill_zero_f64_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

#define OCCRIK_INST(T)                                                                                         \
    template hipError_t launch_pass1<T>(const PairBatch&, const cplx<T>*, cplx<T>*, const cplx<T>*, hipStream_t); \
    template hipError_t launch_pass2<T>(const PairBatch&, cplx<T>*, const cplx<T>*, double*, int, hipStream_t);   \
    template hipError_t launch_pass3<T>(const PairBatch&, const cplx<T>*, const cplx<T>*, cplx<T>*, cplx<T>*,  \
                                        const cplx<T>*, hipStream_t);                                           \
    template hipError_t launch_kcache<T>(const PairBatch&, void*, hipStream_t);                              \
    template hipError_t launch_wreduce<T>(const PairBatch&, const cplx<T>*, cplx<T>*, hipStream_t);            \
    template hipError_t launch_fill_zero<T>(cplx<T>*, size_t, hipStream_t);                                  \
    template hipError_t launch_fused<T>(int, const PairBatch&, const FusedItem*, int, unsigned, hipStream_t);
OCCRIK_INST(float)
OCCRIK_INST(double)
#undef OCCRIK_INST

}  // namespace occrik
