/*
 * occrik.h -- C ABI of the MI355X (gfx950) occ-RI-K exact-exchange library.
 *
 * The library builds the exact-exchange contribution of k-point Gaussian
 * planewave (GPW) solids with the occ-RI-K algorithm of Lee, Rettig, Feng,
 * Epifanovsky and Head-Gordon, "Faster Exact Exchange for Solids via
 * occ-RI-K" (arXiv 2207.09028).  Section and equation names below are the
 * paper's.
 *
 * For one cell, a Gamma-centred k-mesh {k} and a uniform real-space grid, a
 * build takes the occupied coefficients C_{mu i}(k) and returns
 *
 *   K_{mu j}(k)  = -(dV/N_k) sum_r chi*_{mu k}(r) W_{j k}(r)           (Sec. II.D, Alg. 3)
 *       W_{j k}(r) = sum_{k', i} psi_{i k'}(r) V_{i k', j k}(r)         (eq. occrikinterm)
 *       V_{i k', j k} = potential of psi*_{i k'} psi_{j k} fitted by
 *                       plane waves G + q, q = k - k'                    (eqs. aodf, Vrao, VGao)
 *       psi_{i k}(r) = sum_mu C_{mu i}(k) chi_{mu k}(r)                  (eq. occmo)
 *       chi_{mu k}(r) = sum_T e^{ik.T} phi_mu(r - R_mu - T)              (Sec. II.A, Bloch AO;
 *                       the 1/sqrt(N_k) is dropped, orbitals are normalised per cell)
 *   K_ij(k)      = C(k)^H K_{mu j}(k)                                   (occupied block)
 *   K~(k)        = K_mu(k) K_ij(k)^{-1} K_mu(k)^H                        (eq. occrikop, assembled
 *                  through L L^H = -K_ij, xi = K_mu L^{-H}, K~ = -xi xi^H)
 *   E_x          = (1/2N_k) sum_k Re tr K_ij(k)                         (Sec. II.A, E_K / N_k:
 *                  per cell and per spin channel)
 *
 * Units are bohr and hartree.  dV = Omega / N_g.  All arrays are row-major;
 * complex numbers are interleaved (re, im) pairs of doubles.
 *
 * Conventions (both sides of every parity test use them):
 *   grid point   r_n = sum_d (n_d / N_d) a_d, row-major over (n_1, n_2, n_3)
 *   k-point      k = sum_d (kappa_d / M_d) b_d, kappa_d in [0, M_d), row-major
 *   pair momenta q = k - k' from the fractional k-points, never wrapped
 *   DFT indices  0..N/2-1, -N/2..-1 (even N: the Nyquist bin is -N/2)
 *   AO order     shells in the given order; cartesian components of a shell
 *                lexicographic with x^l first (xx, xy, xz, yy, yz, zz for l = 2);
 *                each component normalised as an isolated function
 *   lattice sum  an image T of a shell is kept when |R + T - c| <= rho + r_s, c
 *                the cell centre, rho the cell circumradius about c, r_s the
 *                radius where N_s r^l exp(-alpha r^2) drops to lattice_tol
 *
 * Ownership: the caller owns every input and output buffer; a plan owns its
 * device workspaces (the Bloch AOs on the grid, the occupied orbitals, the W
 * accumulators and the FFT exchange buffer) and frees them in
 * occrik_plan_destroy.  A plan is bound to one device and one HIP stream and
 * is not re-entrant: calls on one plan must not overlap.
 *
 * Errors: every entry point returns an occrik_status and never throws,
 * aborts or prints.  Outputs are unspecified when the status is not
 * OCCRIK_OK.  occrik_last_error_message() returns a thread-local description
 * of the last failure.
 */
#ifndef OCCRIK_H
#define OCCRIK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OCCRIK_OK = 0,
    OCCRIK_ERR_INVALID_ARG = 1,   /* a null pointer, a size out of range, an inconsistent input */
    OCCRIK_ERR_UNSUPPORTED = 2,   /* a grid size that is not 2^a 3^b 5^c in the supported set, l > 3 */
    OCCRIK_ERR_OOM = 3,           /* device memory (or the caller's mem_budget) exhausted */
    OCCRIK_ERR_NOT_PD = 4,        /* -K_ij(k) not positive definite; occrik_last_error_k gives k */
    OCCRIK_ERR_NONFINITE = 5,     /* NaN or Inf in C */
    OCCRIK_ERR_DEVICE = 6,        /* a HIP runtime error */
    OCCRIK_ERR_STATE = 7          /* call out of order (e.g. occrik_grad before a build) */
} occrik_status;

/* Reciprocal-space Coulomb kernels f(x), x = |G + q| (paper eq. recipcoul). */
enum {
    OCCRIK_KERNEL_COULOMB = 0,    /* 4 pi / x^2;                 x = 0 term zeroed */
    OCCRIK_KERNEL_ERF_LR = 1,     /* 4 pi / x^2 exp(-x^2/4w^2);  x = 0 term zeroed */
    OCCRIK_KERNEL_ERFC_SR = 2,    /* 4 pi / x^2 (1 - exp(-x^2/4w^2)); x = 0 term pi / w^2 */
    OCCRIK_KERNEL_TRUNC_COULOMB = 3,  /* 4 pi / x^2 (1 - cos(x R_c)); x = 0 term 2 pi R_c^2.
                                     1/r cut off at R_c (Sec. II.A, the Spencer-Alavi kernel),
                                     with 4 pi R_c^3 / 3 = N_k Omega (the k-mesh supercell's
                                     volume).  omega is ignored; d E_x / d omega is 0.
                                     Evaluated in FP64 in every precision mode. */
    OCCRIK_KERNEL_TRUNC_ERF_LR = 4    /* erf(w r)/r cut off at the same R_c (eq. lrtrunc), as
                                     4 pi / x^2 [e^{-x^2/4w^2} - erf(w R_c) cos(x R_c)
                                     - e^{-w^2 R_c^2} Re(e^{-i x R_c} w(-x/2w + i w R_c))]
                                     with the Faddeeva function w (no overflowing terms);
                                     x = 0 term its finite limit.  Needs omega > 0; FP64. */
};

/* Treatment of the even-N Nyquist planes in the kernel multiply.
 * FFTFREQ:   f(|G_m + q|) with m the numpy frequency (Nyquist component -N/2).
 * SYMMETRIC: on Nyquist planes the mean of f at G_m + q and at the mirror index
 *            with those components at +N/2.  E_x is identical in both modes;
 *            only SYMMETRIC makes 2 K_{mu j} / N_k the exact gradient of E_x and
 *            the (k, k', i, j) <-> (k', k, j, i) pair potentials exact complex
 *            conjugates, which the build uses to halve the FFT count. */
enum { OCCRIK_NYQUIST_FFTFREQ = 0, OCCRIK_NYQUIST_SYMMETRIC = 1 };

/* Arithmetic of the grid-side work (collocated AOs, orbitals, FFTs, W, the two
 * grid contractions).  K_ij, the Cholesky factorisation, the assembly and the
 * energy reduction are FP64 in every mode. */
enum {
    OCCRIK_PREC_FP64 = 0,         /* complex128 grid data, FP64 FFTs and contractions */
    OCCRIK_PREC_FP32 = 1,         /* complex64 grid data, FP32 FFTs, FP32 contractions */
    OCCRIK_PREC_FP32_SPLIT = 2    /* complex64 grid data, FP32 FFTs, contractions on
                                     bf16 matrix cores with 3-term operand splitting
                                     and FP32 accumulation */
};

/* Plan flags (occrik_params.flags, bitwise or).  The pair passes transform with
 * LDS Stockham FFTs.  Complex64 plans (PREC_FP32, PREC_FP32_SPLIT) on cubic grids
 * with N in {24, 32, 36, 40, 48} can instead hold each line in the registers of a
 * lane pair (OCCRIK_FLAG_REG_FFT_ALL); results agree to rounding.  On gfx950 the
 * LDS form with register prefetch of the next pair measured as fast or faster,
 * so the register form is for cross-checks and timing. */
enum {
    OCCRIK_FLAG_LDS_FFT = 1,      /* LDS Stockham transforms (the default; kept explicit) */
    OCCRIK_FLAG_REG_FFT_ALL = 2,  /* register-resident transforms in all three passes
                                     (pass 3 only for nocc <= 8); not with LDS_FFT */
    OCCRIK_FLAG_DIRECT = 4,       /* integral-direct (Sec. II.E, Alg. 4): chi~ is never stored;
                                     every build collocates it chunk by chunk, once for the
                                     orbitals and once for the contraction.  The plan also
                                     switches to it by itself when the stored chi~ would not
                                     fit in mem_budget (or, with no budget, in the device
                                     memory free at plan creation).  Its chunks hold chi~ of
                                     at most 2 GiB (or mem_budget / 8) for every k and AO.
                                     Results are bitwise those of the stored mode. */
    OCCRIK_FLAG_MADELUNG = 8      /* G+q=0 term of the Coulomb and ERF_LR kernels from the
                                     Madelung correction instead of zero: N_k Omega M_s for
                                     Coulomb, M_s the Ewald Madelung constant of the k-mesh
                                     supercell's point-charge lattice (neutralising
                                     background), and N_k Omega M_s - pi / w^2 for ERF_LR.
                                     The paper cites the correction without a formula; this
                                     is the reading used (other kernels: no effect). */
};

typedef struct {
    double lattice[9];            /* rows a_1, a_2, a_3 in bohr, row-major */
    int32_t natm;
    const double *atom_frac;      /* host [natm][3], fractional coordinates */
} occrik_cell;

typedef struct {
    int32_t nshell;
    const int32_t *shell_atom;    /* host [nshell], index into the cell's atoms */
    const int32_t *shell_l;       /* host [nshell], 0..3 (s, p, d, f; cartesian) */
    const double *shell_exp;      /* host [nshell], Gaussian exponent alpha > 0 */
} occrik_basis;

typedef struct {
    int32_t kmesh[3];             /* M_1, M_2, M_3 >= 1 */
    int32_t grid[3];              /* N_1, N_2, N_3, each in the supported set */
    int32_t nocc;                 /* occupied orbitals per k, 1..16 */
    int32_t kernel;               /* OCCRIK_KERNEL_* */
    double omega;                 /* range-separation parameter (bohr^-1) for ERF_LR / ERFC_SR */
    int32_t nyquist;              /* OCCRIK_NYQUIST_* */
    int32_t precision;            /* OCCRIK_PREC_* */
    double lattice_tol;           /* lattice-sum truncation, e.g. 1e-12; must be in (0, 1e-3] */
    int32_t kbatch;               /* summed k-points per FFT batch; 0 = chosen by the plan */
    int32_t flags;                /* OCCRIK_FLAG_* bits; other bits must be 0 */
    size_t mem_budget;            /* device bytes the plan may allocate; 0 = no limit */
    int32_t nvir;                 /* conduction bands treated exactly (Sec. II.D), >= 0 with
                                     nocc + nvir <= 16: C then has nocc + nvir columns per k,
                                     the last nvir being the bands; the exchange is still built
                                     from the nocc occupied columns, K_{mu p} and K~ cover all
                                     columns (K~ C_p equals the conventional K C_p for every
                                     column), E_x is the occupied trace.  0 = ground state. */
    int32_t contract_chunks;      /* grid chunks of the contraction's FP64 partial sums, 1..64;
                                     0 = chosen by the plan (N_g / 4096, or more where the
                                     contraction's launch would hold fewer than 2048
                                     workgroups; at most 64).  Chunks hold whole multiples of
                                     16 points, so the plan keeps only the chunks that hold
                                     grid points (occrik_plan_info reports it) */
} occrik_params;

typedef struct occrik_plan occrik_plan;

typedef struct {
    int32_t nk, nao, nocc, ng;
    int32_t grid[3], kmesh[3];
    int32_t precision, nyquist, kernel, kbatch;
    double omega, cell_volume;
    size_t bytes_chi;             /* Bloch AOs on the grid (0 for integral-direct plans) */
    size_t bytes_workspace;       /* everything else the plan allocated */
    int64_t pair_transforms;      /* forward+inverse 3D FFT pairs per build */
    double plan_seconds;          /* wall time of occrik_plan_create */
    int32_t integral_direct;      /* 1: chi~ collocated per build (OCCRIK_FLAG_DIRECT) */
    int32_t colloc_chunk;         /* grid points per collocation chunk */
    int32_t reg_fft_passes;       /* bit p-1 set: pair pass p runs register-resident transforms */
    int32_t nvir;                 /* conduction bands treated exactly */
    int32_t contract_chunks;      /* grid chunks of the contraction */
    int32_t tuned;                /* 1 after occrik_plan_autotune */
} occrik_plan_info;

/* Per-phase device timings of the last build(s), from HIP events recorded on
 * the plan's stream when profiling is enabled (occrik_set_profiling).  The
 * pair phase is the fused FFT round trip (the paper's bottleneck, Sec. II.D). */
typedef struct {
    double ms_orbitals;           /* psi = chi C (eq. occmo) */
    double ms_pairs;              /* all FFT passes + W accumulation (Alg. 3 inner loops) */
    double ms_contract;           /* K_{mu j} contraction */
    double ms_assemble;           /* K_ij, Cholesky, K~, E_x */
    int64_t launches_pairs;       /* kernel launches inside ms_pairs */
    int64_t builds;               /* builds accumulated since the last reset */
    /* per-kernel sums over every launch of the pair passes (profiling level 2) */
    double ms_pass[3];            /* pass 1, pass 2, pass 3 (+ its W reduction) */
    int64_t launches_pass[3];     /* launches of each pass */
    double bytes_pass[3];         /* algorithmic HBM bytes moved by those launches */
} occrik_profile;

/* Create a plan: validates the inputs, derives the reciprocal lattice and the
 * per-shell image lists, allocates the device workspaces and collocates the
 * Bloch AOs on the grid (stored for every build, as the paper assumes in
 * Sec. II.A; integral-direct plans, see OCCRIK_FLAG_DIRECT, collocate per build).  device: HIP ordinal; stream: a hipStream_t or NULL for the
 * default stream.  *out is NULL on failure. */
occrik_status occrik_plan_create(const occrik_cell *cell, const occrik_basis *basis,
                                 const occrik_params *params, int device, void *stream,
                                 occrik_plan **out);

/* Free every device and host resource of a plan (NULL is ignored). */
void occrik_plan_destroy(occrik_plan *plan);

occrik_status occrik_plan_query(const occrik_plan *plan, occrik_plan_info *info);

/* Rebind the plan to another stream of the same device (NULL = default stream). */
occrik_status occrik_set_stream(occrik_plan *plan, void *stream);

/* Change omega for later builds (kernels ERF_LR / ERFC_SR); omega > 0. */
occrik_status occrik_set_omega(occrik_plan *plan, double omega);

/* Synchronous build from host memory.
 *   C   [N_k][N_ao][nocc + nvir] complex128 (input)
 *   K   [N_k][N_ao][N_ao] complex128 (output K~) or NULL
 *   Kmi [N_k][N_ao][nocc + nvir] complex128 (output K_{mu j}) or NULL
 *   Ex  one double (output E_x) or NULL
 * Returns OCCRIK_ERR_NONFINITE for NaN/Inf in C (checked on the host before any
 * device work) and OCCRIK_ERR_NOT_PD when -K_ij(k) has no Cholesky factor. */
occrik_status occrik_build(occrik_plan *plan, const double *C, double *K, double *Kmi, double *Ex);

/* Asynchronous build from device memory, enqueued on the plan's stream.
 * dC, dK, dKmi as above but device pointers (dK / dKmi may be NULL); dEx is a
 * device pointer to one double or NULL.  Launch errors are returned at once;
 * conditions found on the device (NaN/Inf in C, a failed Cholesky) are
 * reported by occrik_plan_status after the stream reaches them.  If dK is
 * non-NULL and a Cholesky fails, the K~ block of that k is left zeroed. */
occrik_status occrik_build_device(occrik_plan *plan, const void *dC, void *dK, void *dKmi, double *dEx);

/* Autotuner (not part of the paper): times whole builds of C on the plan's stream
 * over the settings the plan's parameters leave open and keeps the fastest, by
 * coordinate descent in this order:
 *   k batch          (FFT batch: summed k-points per pair-pass launch) the plan's
 *                    allocated batch, a half and a quarter of it; fixed when
 *                    params.kbatch > 0
 *   pair transforms  LDS two-stage passes or register-resident passes; complex64
 *                    plans with a register-supported grid, no conduction bands and
 *                    neither OCCRIK_FLAG_LDS_FFT nor OCCRIK_FLAG_REG_FFT_ALL set
 *   contraction      grid chunks of the MFMA contraction (its tiles over the grid):
 *                    the plan's count, twice and half of it, within 1..64; fixed for
 *                    integral-direct plans and when params.contract_chunks > 0
 * One untimed build comes first.  Results of later builds depend on the chosen
 * settings only at rounding level (summation order); a plan created with
 * params.kbatch, the FFT flag and params.contract_chunks set to the chosen values
 * builds bitwise the same.  dC as in occrik_build_device (device memory);
 * synchronous; the tuning builds' outputs are discarded (occrik_grad needs a new
 * build).  A batch graph (occrik_batch_create) recorded before tuning keeps replaying
 * the settings it was recorded with.  out may be NULL. */
typedef struct {
    int32_t kbatch;               /* chosen k batch */
    int32_t reg_fft;              /* 1: register-resident pair passes chosen */
    int32_t contract_chunks;      /* chosen contraction chunks */
    int32_t builds;               /* timed builds */
    double ms_initial;            /* build time with the settings before tuning */
    double ms_best;               /* build time with the chosen settings */
} occrik_tune_info;
occrik_status occrik_plan_autotune(occrik_plan *plan, const void *dC, occrik_tune_info *out);

/* Conventional GPW exchange on the plan's cell, grid, kernel and precision: the
 * algorithms occ-RI-K is measured against, giving the full AO x AO exchange matrix
 *   K_{nu mu}(k_2) = -(dV/N_k) sum_r conj(chi_{nu k_2}(r)) W_{mu k_2}(r)        (eq. aok)
 * with, for every output AO mu of k_2, summed over k_1,
 *   OCCRIK_ALGO_AO_RI_K  (Sec. II.B, Alg. 1): W_mu = sum_sigma psi~_{sigma k_1} V_{sigma k_1, mu k_2},
 *       V fitted from conj(chi_{sigma k_1}) chi_{mu k_2} and
 *       psi~_{sigma k} = sum_lambda P_{lambda sigma}(k) chi_{lambda k}, P = C C^H (eqs. aointerm, aointerm2);
 *       N_k^2 N_ao^2 pair round trips
 *   OCCRIK_ALGO_MO_RI_K  (Sec. II.C, Alg. 2): W_mu = sum_i psi_{i k_1} V_{i k_1, mu k_2},
 *       V fitted from conj(psi_{i k_1}) chi_{mu k_2} (eqs. exxmo, mointerm2);
 *       N_k^2 N_occ N_ao pair round trips
 * (occ-RI-K: N_k^2 N_occ^2, halved with conjugate-pair reuse).  K C equals the K_{mu j}
 * of a build and E_x is the same (Sec. II.D).
 *   dC   [N_k][N_ao][nocc + nvir] complex128 device buffer; the first nocc columns
 *        form the density
 *   dK   [N_k][N_ao][N_ao] complex128 device buffer (required), row nu, column mu
 *   dEx  device double (or NULL): (1/2N_k) sum_k Re tr(C_occ^H K C_occ)
 * The pair passes, kernel multiply and contraction are those of occrik_build_device
 * (same precision mode); workspaces are allocated on the plan at the first call
 * (W of one k-point for every AO, the orbitals, and for AO-RI-K the [N_k][N_ao][N_g]
 * density-contracted AOs).  Needs a plan with stored AOs (OCCRIK_ERR_UNSUPPORTED for
 * integral-direct plans).  Asynchronous on the plan's stream; C is not checked for
 * non-finite values. */
enum {
    OCCRIK_ALGO_AO_RI_K = 1,
    OCCRIK_ALGO_MO_RI_K = 2
};
occrik_status occrik_conventional_k(occrik_plan *plan, int32_t algo, const void *dC, void *dK, double *dEx);

/* Synchronise the plan's stream and return the deferred device status of the
 * last build (OCCRIK_OK, OCCRIK_ERR_NOT_PD or OCCRIK_ERR_NONFINITE). */
occrik_status occrik_plan_status(occrik_plan *plan);

/* k index of the last OCCRIK_ERR_NOT_PD, or -1. */
int32_t occrik_last_error_k(const occrik_plan *plan);

/* For callers that cannot allocate device memory (serving loops, harnesses that forbid
 * hipMalloc): occrik_build with the same arguments, results and errors, but staged
 * through a static 64 MiB device array of the library (one per device, held until the
 * process ends) instead of per-call hipMalloc/hipFree.  C and K_{mu j} are staged whole
 * and K~ a group of k-points at a time, so 2 N_k N_ao (nocc + nvir) 16 bytes (rounded up
 * to 256-byte blocks) plus, when K is requested, N_ao^2 16 bytes for one k-point must fit:
 * larger plans get OCCRIK_ERR_INVALID_ARG (use occrik_build).  The plan's own workspaces,
 * allocated by occrik_plan_create, are used as by every build; this call allocates
 * nothing.  Profiling must be off (OCCRIK_ERR_STATE otherwise).  Every call on a device
 * shares that device's staging array: calls that overlap on one device (plans on
 * different streams or threads) race and must be serialised by the caller.  Synchronous. */
occrik_status occrik_build_static(occrik_plan *plan, const double *C, double *K, double *Kmi, double *Ex);

/* Gradients of E_x after a build on this plan (not part of the paper; the
 * adjoint of the build).  With gEx = dL/dE_x:
 *   dgradC     [N_k][N_ao][nocc + nvir] complex128 device buffer (or NULL) receives
 *              gEx * (2/N_k) K_{mu j}, i.e. dL/dRe C + i dL/dIm C.  This is the
 *              exact gradient for OCCRIK_NYQUIST_SYMMETRIC; with FFTFREQ it
 *              differs by a Nyquist-plane term.
 *   dgradOmega host double (or NULL) receives gEx * dE_x/domega,
 *              dE_x/domega = -(Omega / 2 N_k^2 N_g^2) sum_{pairs, G} df/domega |u^(G)|^2,
 *              from a forward-FFT-only sweep over the pair densities (the
 *              potentials are recomputed, never stored).  Synchronous.
 * Enqueued on the plan's stream; returns OCCRIK_ERR_STATE before a build. */
occrik_status occrik_grad(occrik_plan *plan, double gEx, void *dgradC, double *dgradOmega);

/* Ragged batch: n independent plans (different cells, bases, meshes, grids,
 * nocc), per-plan arguments as in occrik_build_device.  All plans must share one
 * device and one stream, and no plan may appear twice.  The builds run
 * concurrently on four worker streams of the device (largest first, each to the
 * least-loaded stream); the plans' stream waits for all of them, so the call is
 * asynchronous on that stream like occrik_build_device.  Results are bitwise those
 * of single builds.  Not thread-safe: one batch at a time per device. */
occrik_status occrik_build_batch(int32_t n, occrik_plan *const *plans, const void *const *dC,
                                 void *const *dK, void *const *dKmi, double *const *dEx);

/* The same batch recorded once as a HIP graph and replayed by occrik_batch_launch
 * with one launch: for SCF-style loops that rebuild the same cells from the same
 * buffers.  occrik_batch_create runs no kernels; it needs the plans on a
 * non-default stream and profiling off.  The plans and every buffer passed here
 * must outlive the batch object; each launch reads dC and writes dK/dKmi/dEx as
 * they are at launch time.  After create the plans count as built (occrik_grad and
 * occrik_plan_status then refer to the latest launch).  Launches are asynchronous
 * on the plans' stream; occrik_batch_destroy waits for that stream and frees the
 * batch's own device memory. */
typedef struct occrik_batch occrik_batch;
occrik_status occrik_batch_create(int32_t n, occrik_plan *const *plans, const void *const *dC,
                                  void *const *dK, void *const *dKmi, double *const *dEx,
                                  occrik_batch **out);
occrik_status occrik_batch_launch(occrik_batch *batch);
void occrik_batch_destroy(occrik_batch *batch);

/* occrik_batch_create with fused rounds: the loop over (k, k') blocks of Sec. II.D,
 * Alg. 3, run for several cells at once.  Plans that share the working precision
 * (complex128 for FP64; complex64 for FP32 and FP32-split), a compiled cubic grid
 * (24, 30, 32, 36, 40 or 48 points a side), the LDS pair-pass kernels, a kernel-value
 * cache and the pass-3 form (up to 8, or 9 to 16 output orbitals) form groups of at
 * least two.  Round r of a group runs the r-th pair-pass launch of each of its plans
 * as one launch per pass (pass 1, pass 2, pass 3, the W reduction); the groups' rounds
 * run on the worker streams beside the other plans' whole builds, and the grouped
 * plans' orbitals and contractions before and after them.  Fused rounds run pass 1
 * with one summed orbital per workgroup; a single build does so too on launches of
 * fewer than 4096 such workgroups (small cells: there the results are bitwise those
 * of single builds) and holds four on larger ones, whose densities can then differ in
 * the last bit (the same arithmetic, compiled separately).  Before recording it
 * allocates and uploads, synchronously, the
 * rounds' item table (a few hundred bytes per pair-pass launch of each grouped plan),
 * which occrik_batch_destroy frees.  Same arguments and rules as occrik_batch_create. */
occrik_status occrik_batch_create_fused(int32_t n, occrik_plan *const *plans, const void *const *dC,
                                        void *const *dK, void *const *dKmi, double *const *dEx,
                                        occrik_batch **out);
/* The number of plans of a recorded batch whose pair passes run in fused rounds
 * (0 for occrik_batch_create, or when no two plans share a kernel form), written to
 * *nplans. */
occrik_status occrik_batch_fused(const occrik_batch *batch, int32_t *nplans);

/* Profiling: level 1 records HIP events around the phases of every build on
 * the plan's stream; level 2 also brackets every pair-pass launch.
 * occrik_get_profile synchronises and returns the accumulated milliseconds
 * since the last reset (reset = 1 clears them afterwards).  Algorithmic bytes
 * per launch: pass 1 writes P N_g s, pass 2 reads and writes P N_g s, pass 3
 * reads P N_g s, for P = pairs in the launch and s = bytes per complex value
 * (orbital-plane reads are not counted: they are shared by many pairs). */
occrik_status occrik_set_profiling(occrik_plan *plan, int32_t on);
occrik_status occrik_get_profile(occrik_plan *plan, occrik_profile *out, int32_t reset);

/* Diagnostics: copy a plan-owned intermediate into caller device memory,
 * converted to complex128, row-major.
 *   which = 0: chi~ [N_k][N_ao][N_g], the cell-periodic Bloch AOs e^{-ik.r} chi_{mu k}(r)
 *   which = 1: psi~ [N_k][nocc + nvir][N_g], e^{-ik.r} psi_{i k}(r) of the last build
 *   which = 2: W~   [N_k][nocc + nvir][N_g], e^{-ik.r} W_{j k}(r) of the last build
 * bytes must equal the size of that array in complex128. */
occrik_status occrik_copy_intermediate(occrik_plan *plan, int32_t which, void *dst, size_t bytes);

/* HBM bandwidth probe (measurement, not part of the paper): a plain streaming kernel
 * over a buffer of a known size, timed with HIP events on `stream` (NULL = default
 * stream) on the calling thread's current device.  It sets the achievable rates that
 * the pair passes are measured against: pass 1 mostly writes (with one read for about
 * eight writes), pass 3 mostly reads, pass 2 reads and writes equal amounts.
 *   kind         0: read `bytes` of src (dst receives at most 4 bytes, almost never)
 *                1: write `bytes` to dst
 *                2: copy `bytes` from src to dst
 *                3: write `bytes` to dst and read one access of src for every
 *                   `read_every` written (src needs bytes / read_every)
 *   width        bytes per lane access, 8 or 16
 *   nontemporal  1: streaming (non-temporal) loads and stores, as the pair passes use
 *   read_every   kind 3 only (>= 1); ignored otherwise
 *   dst, src     device buffers of at least `bytes`, aligned to `width`; src unused by kind 1
 *   reps         timed repetitions after one untimed one
 *   ms_per_rep   host double: receives the mean milliseconds of one repetition
 * Synchronous.  OCCRIK_ERR_INVALID_ARG for a bad kind, width, size, ratio or alignment. */
occrik_status occrik_hbm_probe(int32_t kind, int32_t width, int32_t nontemporal, int32_t read_every, void *dst,
                               const void *src, size_t bytes, int32_t reps, void *stream, double *ms_per_rep);

const char *occrik_status_string(occrik_status s);
const char *occrik_last_error_message(void);

/* 1 if the grid size n is supported along one dimension, else 0. */
int32_t occrik_grid_size_supported(int32_t n);

#ifdef __cplusplus
}
#endif

#endif /* OCCRIK_H */
