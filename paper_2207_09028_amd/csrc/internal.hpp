// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/occrik.h"
#include "common.hpp"

namespace occrik {

// One batch of pair round trips: output k-point a, blocks (a, b) for b in
// [b0, b0 + nb).  Stored pairs ("slots"): block b holds the nocc x nout pairs
// (i at b summed, j at a output) at slot base + i * nout + j; with conjugate-pair
// reuse (square pair sets only, nout == nocc) the
// batch starts at b0 >= a and, when b0 == a, the diagonal block comes first and
// holds only the pairs i <= j (nocc (nocc + 1) / 2 slots, upper-triangle rows).
// The density of a slot is conj(psi~_{i b}) psi~_{j a}, momentum q = k_a - k_b.
struct PairBatch {
    int N1, N2, N3, ng;
    int M1, M2, M3;
    int nocc;                 // summed (occupied) orbitals per k: pair index i
    int nout;                 // output orbitals of the pairs: index j (nocc + conduction bands)
    int kstride;              // orbitals per k in the psi~ and W~ arrays
    int a, b0, nb;
    int reuse;                // conjugate-pair reuse (symmetric Nyquist mode)
    int diag;                 // the first block is the diagonal block (a, a)
    int ntri;                 // nocc (nocc + 1) / 2
    int nslots;               // stored pairs in the batch
    int group;                // stored pairs per pass-2 workgroup
    int kernel, nyquist;
    double omega;
    double rcut;              // truncated Coulomb radius R_c (4 pi R_c^3 / 3 = N_k Omega)
    int madelung;             // 1: G+q=0 term of Coulomb / ERF_LR from g0 instead of zero
    double g0;                // N_k Omega M_s (Madelung constant of the k-mesh supercell)
    double inv_ng;
    double recip[9];          // reciprocal vectors b_1, b_2, b_3 (rows)
    int splits;               // pass-3 splits of the (b, i) sum of the a-side
    int parseval;             // 1: accumulate sum f |u^|^2 per pass-2 workgroup
    int regfft;               // REGFFT_PASS* bits: passes run with register-resident line FFTs
    void* kvals;              // [nb][m2][m1][m3] kernel values of the batch, working precision (plan workspace)
    int kcache;               // 1: kvals is the plan's table of every k-point difference k_a - k_b
                              //    ([(2M1-1)(2M2-1)(2M3-1)][m2][m1][m3]), filled once per omega
    // Orbital sources of the passes (working precision, complex).  The density of a
    // slot is conj(D_{i b}) O_j and the a-side sum is W_j += A_{i b} Vt_ij, with
    //   D_{i b} = psi[(b kstride + i) ng]   (the psi argument of the launchers)
    //   O_j     = outp[j ng]                the output orbitals of k_a
    //   A_{i b} = accp[(b kstride + i) ng]
    // and W_j at W[woff + j ng] (the W argument).  occ-RI-K: D = A = psi~,
    // O = psi~ at k_a, woff = a kstride ng.  The conventional algorithms pair the
    // occupied orbitals (MO-RI-K) or the AOs (AO-RI-K) with a group of AOs of k_a.
    const void* outp;
    const void* accp;
    size_t woff;
};

// pass-2 workgroups per m2-slab of a batch
int pair_groups(const PairBatch& B);
// pass-3 splits of the (b, i) sum for a batch (B.nb, B.nocc and the grid set), elem = bytes per complex
int pass3_splits(const PairBatch& B, int elem);

// Launchers (templated on the working real type: float or double).
template <typename T>
hipError_t launch_pass1(const PairBatch& B, const cplx<T>* psi, cplx<T>* X, const cplx<T>* tw, hipStream_t s);
template <typename T>
hipError_t launch_pass2(const PairBatch& B, cplx<T>* X, const cplx<T>* tw, double* parts, int deriv_only,
                        hipStream_t s);
template <typename T>
hipError_t launch_pass3(const PairBatch& B, const cplx<T>* X, const cplx<T>* psi, cplx<T>* Wpart, cplx<T>* W,
                        const cplx<T>* tw, hipStream_t s);
// register-FFT variants of the three passes (pairs_reg.hip), complex64 only;
// pass 3 takes at most 8 occupied orbitals.  Plans use them only when asked
// (OCCRIK_FLAG_REG_FFT_ALL): with the next pair prefetched into registers, the
// LDS Stockham passes measured as fast or faster on gfx950 (their radix-8/6
// stages issue fewer VALU instructions, and they keep more waves resident).
enum { REGFFT_PASS1 = 1, REGFFT_PASS2 = 2, REGFFT_PASS3 = 4, REGFFT_DEFAULT = 0 };
bool reg_fft_size(int n1, int n2, int n3);
hipError_t launch_pass1_reg(const PairBatch& B, const cplx<float>* psi, cplx<float>* X, hipStream_t s);
hipError_t launch_pass2_reg(const PairBatch& B, cplx<float>* X, double* parts, int deriv_only, hipStream_t s);
hipError_t launch_pass3_reg(const PairBatch& B, const cplx<float>* X, const cplx<float>* psi, cplx<float>* Wpart,
                            cplx<float>* W, hipStream_t s);

// the plan's cache of kernel values: f(|G+q|) for every k-point difference q of the mesh
template <typename T>
hipError_t launch_kcache(const PairBatch& B, void* out, hipStream_t s);
size_t kcache_tables(int M1, int M2, int M3);

template <typename T>
hipError_t launch_wreduce(const PairBatch& B, const cplx<T>* Wpart, cplx<T>* W, hipStream_t s);

// Fused rounds of a ragged batch: one launch per stage (pass 1, pass 2, pass 3, the W
// reduction) runs one k batch of each of several plans that share the working
// precision, a compiled cubic grid and the pass-3 form.  Workgroup g of a fused launch
// belongs to the last item whose first workgroup of that stage is <= g and runs that
// item's batch as workgroup g - wg0 of the plan's own launch, so every result is the
// plan's own, bit for bit.
constexpr int kFusedStages = 4;
struct FusedItem {
    PairBatch B;
    const void* psi;          // pass-1 density source (the psi argument of launch_pass1)
    void* X;                  // the plan's stored pair spectra
    void* Wpart;              // the plan's pass-3 partial sums
    void* W;                  // the plan's W~
    const void* tw;           // the plan's twiddles
    double* parts;            // the plan's pass-2 partials (unused: no Parseval sums in a build)
    int wg0[kFusedStages];    // first workgroup of this item in each stage's fused grid
};
// a batch can join a fused round: compiled cubic grid, the LDS pass kernels (no
// register-FFT pass), kernel values from the plan's cache, at most 16 output orbitals
bool fusable(const PairBatch& B);
// workgroups of each stage for one batch (elem = bytes per complex)
void fused_workgroups(const PairBatch& B, int elem, int out[kFusedStages]);
// one fused launch of `stage` over items[0, nitems) (device memory), `total` workgroups
// in all; B0 is any item's batch (they share the kernel form)
template <typename T>
hipError_t launch_fused(int stage, const PairBatch& B0, const FusedItem* items, int nitems, unsigned total,
                        hipStream_t s);

template <typename T>
hipError_t launch_fill_zero(cplx<T>* p, size_t n, hipStream_t s);
hipError_t launch_fill_zero_f64(double* p, size_t n, hipStream_t s);

// Grid contractions on the matrix cores; mode = OCCRIK_PREC_* (FP32_SPLIT uses split-bf16).
// psi[k][j][n0 + t] = sum_mu C[k][mu][j] chi[k][mu][t] for t < cnt; chi rows have stride ldc
template <typename T>
hipError_t launch_orbitals(const cplx<T>* chi, size_t ldc, const double2* C, cplx<T>* psi, int nk, int nao, int nocc,
                           int ng, int n0, int cnt, int mode, hipStream_t s);
// grid points per partial sum of the contraction
int contract_chunk(int ng, int nchunks);
// chunks of contract_chunk(ng, nchunks) points that hold grid points (<= nchunks)
int contract_chunk_count(int ng, int nchunks);
// FP64 partial sums Kpart[k][mu][j][c] for chunks c in [c0, c0 + nc) of the grid
// (nchunks chunks of contract_chunk points); chi holds the points from chi_n0 on,
// rows of stride ldc
template <typename T>
hipError_t launch_contract_part(const cplx<T>* chi, size_t ldc, int chi_n0, const cplx<T>* W, double2* Kpart, int nk,
                                int nao, int nocc, int ng, int nchunks, int c0, int nc, int mode, hipStream_t s);
// Kmi = scale * sum_c Kpart[..][c], c in chunk order
hipError_t launch_contract_reduce(const double2* Kpart, double2* Kmi, size_t n, int nchunks, double scale,
                                  hipStream_t s);

hipError_t launch_check_finite(const double2* C, size_t n, int* flags, hipStream_t s);
hipError_t launch_reset_flags_n(int* flags, int n, hipStream_t s);
// K_pq = C^H K_{mu q} (ncol x ncol per k), its Cholesky factor, and the energy term
// Re tr over the first nocc (occupied) orbitals / (2 N_k)
hipError_t launch_kij(const double2* C, const double2* Kmi, double2* Kij, double2* L, double* eterm, int* flags,
                      int nk, int nao, int ncol, int nocc, hipStream_t s);
hipError_t launch_xi(const double2* Kmi, const double2* L, double2* Y, const int* flags, int nk, int nao, int nocc,
                     hipStream_t s);
hipError_t launch_ktilde(const double2* Y, double2* K, const int* flags, int nk, int nao, int nocc, hipStream_t s);
hipError_t launch_energy(const double* eterm, int nk, double* out, hipStream_t s);
hipError_t launch_sum_f64(const double* parts, size_t n, double scale, double* out, hipStream_t s);
hipError_t launch_scale_copy(const double2* src, double2* dst, size_t n, double scale, hipStream_t s);
// dst[r][c] = scale * src[r][c] for c < nkeep, 0 for nkeep <= c < ncol
hipError_t launch_grad_columns(const double2* src, double2* dst, size_t rows, int ncol, int nkeep, double scale,
                               hipStream_t s);

// Conventional algorithms (AO-RI-K, MO-RI-K).
// psit[k][sigma][n] = sum_{i < nocc} conj(C[k][sigma][i]) psi[k][i][n]; C and psi have ncol columns
template <typename T>
hipError_t launch_density_orbitals(const double2* C, const cplx<T>* psi, cplx<T>* psit, int nk, int nao, int ncol,
                                   int nocc, int ng, hipStream_t s);
// dst[r ld + col0 + j] = scale * sum_c Kpart[(r ncols + j) nchunks + c], c in chunk order
hipError_t launch_reduce_columns(const double2* Kpart, double2* dst, int rows, int ncols, int ld, int col0,
                                 int nchunks, double scale, hipStream_t s);
// eterm[k] = Re tr(C^H K C) / (2 N_k) over the first nocc of the ncol columns of C
hipError_t launch_conv_energy(const double2* C, const double2* K, double* eterm, int nk, int nao, int ncol, int nocc,
                              hipStream_t s);

// Collocation: at plan time into the stored chi~, or per build and per grid chunk in
// integral-direct plans; both run the same per-point arithmetic.
struct CollocGeom {
    double lat[9];            // rows a_1, a_2, a_3
    int N[3];                 // grid
    int M[3];                 // k-mesh
    int nk, ng;
    int n0, cnt;              // the grid points [n0, n0 + cnt) collocated by one call
};
struct ShellDev {
    double R[3];
    double alpha;
    int l;
    int ncomp;
    double norm[10];
};
hipError_t launch_colloc_fold(double* phi, const double4* img, const int* bucket, const ShellDev& sh,
                              const CollocGeom& g, hipStream_t s);
// Bloch-phase DFT over the image cells of one component: phi_real [L][n] ->
// result [k][n] (complex128) = sum_L e^{ik.L} phi[L][n].  Uses work0/work1 as
// ping-pong buffers and returns the one holding the result.
hipError_t launch_colloc_kdft(const double* phi_real, double2* work0, double2* work1, const CollocGeom& g,
                              hipStream_t s, double2** result);
// chi~ of component mu for the points of g: dst[(k nao + mu) ldc + coff + (n - g.n0)]
template <typename T>
hipError_t launch_colloc_store(const double2* chik, cplx<T>* dst, int mu, int nao, size_t ldc, size_t coff,
                               const CollocGeom& g, hipStream_t s);

template <typename T>
hipError_t launch_convert_to_c128(const cplx<T>* src, double2* dst, size_t n, hipStream_t s);

}  // namespace occrik
