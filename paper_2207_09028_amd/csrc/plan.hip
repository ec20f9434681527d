// Plans and the C ABI of the occ-RI-K library.
//
// A plan fixes the cell, basis, k-mesh, grid and kernel, collocates the Bloch
// AOs on the grid once (the stored-AO variant of the paper's Sec. II.A/II.D)
// and owns every device workspace of a build:
//
//   build = orbitals (eq. occmo) -> pair round trips over all (k, k') blocks
//           (Alg. 3 loops, batched over the summed k-points) -> contraction ->
//           FP64 occupied block, Cholesky, assembly and energy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fft.hpp"
#include "internal.hpp"

using namespace occrik;

// Staging area of occrik_build_static (see below): 64 MiB per device.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

thread_local std::string g_last_error;

occrik_status fail(occrik_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

occrik_status hip_fail(hipError_t e, const char* where) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(OCCRIK_ERR_OOM, std::string(where) + ": " + hipGetErrorString(e));
    return fail(OCCRIK_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define OCCRIK_HIP(call)                                      \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return hip_fail(e_, #call);     \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// output AOs of k_a per group of the conventional pair passes (the occ-RI-K pass-3
// tile of eight output orbitals, with the next pair prefetched)
constexpr int kConvGroup = 8;
// largest number of grid chunks of the contraction's partial sums
constexpr int kMaxContractChunks = 64;

// Staging area of occrik_build_static, for callers that cannot allocate device memory:
// one file-scope array per device, held until the process ends.  Host code never
// passes `scratch` itself to the runtime (on the host it is only a stand-in symbol);
// it uses the device address that hipGetSymbolAddress returns for the current device,
// looked up once per device on the first call there.
constexpr int kMaxStaticDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxStaticDevices] = {};

struct ProfileEvents {
    hipEvent_t e[5];
    int64_t pair_launches;
    std::vector<hipEvent_t> pe;    // level 2: 4 events per batch (before pass 1, after 1, 2, 3)
    std::vector<double> pbytes;    // algorithmic bytes of each batch's passes (3 per batch)
};

}  // namespace

struct occrik_plan {
    int device = 0;
    hipStream_t stream = nullptr;
    occrik_params params{};
    double lat[9]{}, recip[9]{}, volume = 0.0, dv = 0.0;
    int N[3]{}, M[3]{};
    int nk = 0, ng = 0, nao = 0, nocc = 0, natm = 0;
    int nvir = 0, nout = 0;     // conduction bands treated exactly; nout = nocc + nvir columns of C
    std::vector<double> atom_cart;
    std::vector<int> shell_atom, shell_l;
    std::vector<double> shell_exp;
    bool fp64 = true;
    size_t elem = 16;
    int kbatch = 1, splits = 1, nchunks = 1, group = 8;
    int kbatch_max = 1;        // k batch the pair workspaces were sized for
    int kpart_chunks = 1;      // contraction chunks the partial-sum buffer holds
    bool tuned = false;        // occrik_plan_autotune has chosen kbatch / regfft / nchunks

    // device memory
    std::vector<void*> allocations;
    std::vector<size_t> sizes;
    size_t bytes_alloc = 0, bytes_chi = 0;
    void* chi = nullptr;       // [nk][nao][ng] cplx<T>
    void* psi = nullptr;       // [nk][nout][ng]
    void* W = nullptr;         // [nk][nout][ng]
    void* X = nullptr;         // [kbatch * nocc * nout][ng]
    void* Wpart = nullptr;     // [splits][nout][ng]
    void* tw = nullptr;        // [3][kMaxN]
    double* parts = nullptr;   // [kbatch * nocc^2 * N2]
    void* kvals = nullptr;     // [kbatch][ng] kernel values of a batch, working precision
    void* kcache = nullptr;    // kernel values of every k-point difference (see PairBatch::kcache), or null
    bool kcache_valid = false; // filled for kcache_omega
    double kcache_omega = 0.0;
    // collocation: image tables (whole plan) and per-chunk scratch
    double4* cimg = nullptr;   // images of every shell, bucketed by image cell
    int* cbucket = nullptr;    // [nshell][nk + 1] offsets into cimg
    std::vector<ShellDev> cshell;
    int maxcomp = 1;
    int cchunk = 0;            // grid points per collocation chunk (a multiple of the contraction chunk)
    double* cphi = nullptr;    // [maxcomp][nk][cchunk]
    double2* cw0 = nullptr;    // [nk][cchunk]
    double2* cw1 = nullptr;
    bool direct = false;       // integral-direct: chi~ collocated per build, chunk by chunk, never stored
    double madelung_g0 = 0.0;  // Madelung mode: N_k Omega M_s of the k-mesh supercell (0: off)
    void* chi_ws = nullptr;    // direct: [nk][nao][cchunk] chi~ of one chunk
    bool regfft = false;       // complex64 pair passes with register-resident transforms
    // conventional algorithms (AO-RI-K, MO-RI-K): workspaces allocated on first use
    int conv_kbatch = 0;       // (a, b) blocks per batch of the conventional pair passes
    int conv_nsum = 0;         // summed orbitals the X workspace is sized for
    void* conv_psi = nullptr;  // [nk][nout][ng] occupied orbitals of the conventional call
    void* conv_psit = nullptr; // AO-RI-K: [nk][nao][ng] density-contracted AOs (eq. aointerm)
    void* conv_W = nullptr;    // [nao][ng] W of every AO of one output k-point
    void* conv_X = nullptr;    // [conv_kbatch * conv_nsum * kConvGroup][ng]
    void* conv_Wpart = nullptr;  // [splits][kConvGroup][ng]
    void* conv_kvals = nullptr;  // [conv_kbatch][ng]
    double2* conv_Kpart = nullptr;  // [nao][16][nchunks]
    double2* Kpart = nullptr;  // [nk][nao][nout][nchunks]
    double2* Kmi = nullptr;    // [nk][nao][nout]
    double2* Kij = nullptr;    // [nk][nout][nout]
    double2* L = nullptr;      // [nk][nout][nout]
    double2* Y = nullptr;      // [nk][nao][nout]
    double* eterm = nullptr;   // [nk]
    double* scal = nullptr;    // [4] device scalars
    int* flags = nullptr;      // [2 + nk]

    bool built = false;
    int last_err_k = -1;
    double plan_seconds = 0.0;

    int profiling = 0;
    std::vector<ProfileEvents> prof;
    occrik_profile prof_acc{};

    ~occrik_plan() {
        for (auto& p : prof) {
            for (auto& e : p.e) (void)hipEventDestroy(e);
            for (auto& e : p.pe) (void)hipEventDestroy(e);
        }
        for (void* p : allocations) (void)hipFree(p);
    }

    hipError_t alloc(void** p, size_t bytes) {
        if (params.mem_budget != 0 && bytes_alloc + bytes > params.mem_budget) return hipErrorOutOfMemory;
        hipError_t e = hipMalloc(p, bytes == 0 ? 16 : bytes);
        if (e == hipSuccess) {
            allocations.push_back(*p);
            sizes.push_back(bytes);
            bytes_alloc += bytes;
        }
        return e;
    }
    void release(void* p) {
        for (size_t i = 0; i < allocations.size(); ++i) {
            if (allocations[i] == p) {
                (void)hipFree(p);
                bytes_alloc -= sizes[i];
                allocations.erase(allocations.begin() + i);
                sizes.erase(sizes.begin() + i);
                return;
            }
        }
    }
};

namespace {

// ---------------------------------------------------------------------------
// geometry helpers (host)
// ---------------------------------------------------------------------------
bool invert3(const double* a, double* inv) {
    const double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                       a[2] * (a[3] * a[7] - a[4] * a[6]);
    if (!(std::fabs(det) > 1e-12) || !std::isfinite(det)) return false;
    const double id = 1.0 / det;
    inv[0] = (a[4] * a[8] - a[5] * a[7]) * id;
    inv[1] = (a[2] * a[7] - a[1] * a[8]) * id;
    inv[2] = (a[1] * a[5] - a[2] * a[4]) * id;
    inv[3] = (a[5] * a[6] - a[3] * a[8]) * id;
    inv[4] = (a[0] * a[8] - a[2] * a[6]) * id;
    inv[5] = (a[2] * a[3] - a[0] * a[5]) * id;
    inv[6] = (a[3] * a[7] - a[4] * a[6]) * id;
    inv[7] = (a[1] * a[6] - a[0] * a[7]) * id;
    inv[8] = (a[0] * a[4] - a[1] * a[3]) * id;
    return true;
}

double dfact(int n) {
    double r = 1.0;
    while (n > 1) {
        r *= n;
        n -= 2;
    }
    return r;
}

// radius beyond which N_s r^l exp(-alpha r^2) < tol, N_s the largest component norm
double shell_extent(double alpha, int l, double tol) {
    const double ln_n = 0.75 * std::log(2.0 * alpha / M_PI) + 0.5 * l * std::log(4.0 * alpha);
    const double ln_tol = std::log(tol);
    auto g = [&](double r) { return ln_n + (l > 0 ? l * std::log(r) : 0.0) - alpha * r * r - ln_tol; };
    double lo = l > 0 ? std::sqrt(l / (2.0 * alpha)) : 0.0;
    if (l > 0 && g(lo) < 0.0) return 0.0;
    if (l == 0 && ln_n - ln_tol < 0.0) return 0.0;
    double hi = std::max(lo, 1.0);
    while (g(hi) > 0.0) hi *= 2.0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (g(mid) > 0.0) lo = mid;
        else hi = mid;
    }
    return hi;
}

int pmod(long a, int m) {
    long r = a % m;
    return (int)(r < 0 ? r + m : r);
}

// Madelung constant M_s > 0 of the point-charge lattice with rows a (bohr) in a
// neutralising background, by Ewald summation with splitting eta = sqrt(pi) / V^(1/3):
// M_s = -[sum'_T erfc(eta|T|)/|T| + 4 pi/V sum'_G e^{-G^2/4 eta^2}/G^2 - 2 eta/sqrt(pi) - pi/(eta^2 V)]
double madelung_constant(const double* a) {
    const double vol = std::fabs(a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                                 a[2] * (a[3] * a[7] - a[4] * a[6]));
    double inv[9];
    invert3(a, inv);
    double g[9];                                   // reciprocal rows 2 pi (A^{-1})^T
    for (int d = 0; d < 3; ++d)
        for (int e = 0; e < 3; ++e) g[3 * d + e] = 2.0 * M_PI * inv[3 * e + d];
    const double eta = std::sqrt(M_PI) / std::cbrt(vol);
    const double rcut = 7.0 / eta, gcut = 14.0 * eta;
    // |t_d| <= cut |column d of rows^-1| covers every |t @ rows| <= cut
    auto range = [](const double* rows, double cut, int* n) {
        double ri[9];
        invert3(rows, ri);
        for (int d = 0; d < 3; ++d)
            n[d] = (int)std::ceil(cut * std::sqrt(ri[d] * ri[d] + ri[3 + d] * ri[3 + d] + ri[6 + d] * ri[6 + d])) + 1;
    };
    int nr[3], ng[3];
    range(a, rcut, nr);
    range(g, gcut, ng);
    double real = 0.0, rec = 0.0;
    for (int i = -nr[0]; i <= nr[0]; ++i)
        for (int j = -nr[1]; j <= nr[1]; ++j)
            for (int k = -nr[2]; k <= nr[2]; ++k) {
                if (i == 0 && j == 0 && k == 0) continue;
                double t2 = 0.0;
                for (int e = 0; e < 3; ++e) {
                    const double x = i * a[e] + j * a[3 + e] + k * a[6 + e];
                    t2 += x * x;
                }
                const double t = std::sqrt(t2);
                if (t <= rcut) real += std::erfc(eta * t) / t;
            }
    for (int i = -ng[0]; i <= ng[0]; ++i)
        for (int j = -ng[1]; j <= ng[1]; ++j)
            for (int k = -ng[2]; k <= ng[2]; ++k) {
                if (i == 0 && j == 0 && k == 0) continue;
                double q2 = 0.0;
                for (int e = 0; e < 3; ++e) {
                    const double x = i * g[e] + j * g[3 + e] + k * g[6 + e];
                    q2 += x * x;
                }
                if (q2 <= gcut * gcut) rec += std::exp(-q2 / (4.0 * eta * eta)) / q2;
            }
    rec *= 4.0 * M_PI / vol;
    return -(real + rec - 2.0 * eta / std::sqrt(M_PI) - M_PI / (eta * eta * vol));
}

// Image lists of every shell (host work, once per plan): the images T of shell
// sh kept by the truncation rule, bucketed by image cell L = t mod M, go to the
// device as one array with per-shell offsets, so that any range of grid points
// can be collocated later without host work.
occrik_status build_colloc_tables(occrik_plan* P) {
    const int nk = P->nk;
    // cell centre and circumradius
    double c[3], rho = 0.0;
    for (int d = 0; d < 3; ++d) c[d] = 0.5 * (P->lat[d] + P->lat[3 + d] + P->lat[6 + d]);
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int k = 0; k < 2; ++k) {
                double q = 0.0;
                for (int d = 0; d < 3; ++d) {
                    const double x = i * P->lat[d] + j * P->lat[3 + d] + k * P->lat[6 + d] - c[d];
                    q += x * x;
                }
                rho = std::max(rho, std::sqrt(q));
            }
    double inv[9];
    invert3(P->lat, inv);
    const int nshell = (int)P->shell_l.size();
    std::vector<double4> flat;
    std::vector<int> off((size_t)nshell * (nk + 1), 0);
    P->cshell.assign(nshell, ShellDev{});
    P->maxcomp = 1;
    for (int sh = 0; sh < nshell; ++sh) {
        const int l = P->shell_l[sh];
        const double alpha = P->shell_exp[sh];
        const double* R = &P->atom_cart[3 * P->shell_atom[sh]];
        const double rs = shell_extent(alpha, l, P->params.lattice_tol);
        const double reach = rho + rs;
        double rc = 0.0;
        for (int d = 0; d < 3; ++d) rc += (R[d] - c[d]) * (R[d] - c[d]);
        const double bound = reach + std::sqrt(rc);
        int nmax[3];
        for (int d = 0; d < 3; ++d) {
            const double cn = std::sqrt(inv[d] * inv[d] + inv[3 + d] * inv[3 + d] + inv[6 + d] * inv[6 + d]);
            nmax[d] = (int)std::ceil(bound * cn) + 1;
        }
        std::vector<std::vector<double4>> buckets(nk);
        for (int t1 = -nmax[0]; t1 <= nmax[0]; ++t1)
            for (int t2 = -nmax[1]; t2 <= nmax[1]; ++t2)
                for (int t3 = -nmax[2]; t3 <= nmax[2]; ++t3) {
                    double tv[3], q = 0.0;
                    for (int d = 0; d < 3; ++d) {
                        tv[d] = t1 * P->lat[d] + t2 * P->lat[3 + d] + t3 * P->lat[6 + d];
                        const double x = R[d] + tv[d] - c[d];
                        q += x * x;
                    }
                    if (q > reach * reach) continue;
                    const int L = (pmod(t1, P->M[0]) * P->M[1] + pmod(t2, P->M[1])) * P->M[2] + pmod(t3, P->M[2]);
                    buckets[L].push_back(make_double4(tv[0], tv[1], tv[2], 0.0));
                }
        for (int L = 0; L < nk; ++L) {
            off[(size_t)sh * (nk + 1) + L] = (int)flat.size();
            flat.insert(flat.end(), buckets[L].begin(), buckets[L].end());
        }
        off[(size_t)sh * (nk + 1) + nk] = (int)flat.size();

        ShellDev& sd = P->cshell[sh];
        for (int d = 0; d < 3; ++d) sd.R[d] = R[d];
        sd.alpha = alpha;
        sd.l = l;
        sd.ncomp = (l + 1) * (l + 2) / 2;
        P->maxcomp = std::max(P->maxcomp, sd.ncomp);
        int ic = 0;
        for (int a = l; a >= 0; --a)
            for (int b = l - a; b >= 0; --b) {
                const int cz = l - a - b;
                sd.norm[ic++] = std::pow(2.0 * alpha / M_PI, 0.75) * std::pow(4.0 * alpha, 0.5 * l) /
                                std::sqrt(dfact(2 * a - 1) * dfact(2 * b - 1) * dfact(2 * cz - 1));
            }
    }
    if (flat.empty()) flat.push_back(make_double4(0.0, 0.0, 0.0, 0.0));
    OCCRIK_HIP(P->alloc((void**)&P->cimg, sizeof(double4) * flat.size()));
    OCCRIK_HIP(P->alloc((void**)&P->cbucket, sizeof(int) * off.size()));
    OCCRIK_HIP(hipMemcpy(P->cimg, flat.data(), sizeof(double4) * flat.size(), hipMemcpyHostToDevice));
    OCCRIK_HIP(hipMemcpy(P->cbucket, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice));
    return OCCRIK_OK;
}

// chi~ of every AO and k at the grid points [n0, n0 + cnt) into
// dst[(k nao + mu) ldc + coff + t], t = n - n0; scratch sized for P->cchunk points
template <typename T>
occrik_status collocate_range(occrik_plan* P, int n0, int cnt, cplx<T>* dst, size_t ldc, size_t coff) {
    hipStream_t s = P->stream;
    CollocGeom g{};
    std::memcpy(g.lat, P->lat, sizeof(g.lat));
    for (int d = 0; d < 3; ++d) {
        g.N[d] = P->N[d];
        g.M[d] = P->M[d];
    }
    g.nk = P->nk;
    g.ng = P->ng;
    g.n0 = n0;
    g.cnt = cnt;
    int mu0 = 0;
    for (size_t sh = 0; sh < P->cshell.size(); ++sh) {
        const ShellDev& sd = P->cshell[sh];
        OCCRIK_HIP(launch_colloc_fold(P->cphi, P->cimg, P->cbucket + sh * (P->nk + 1), sd, g, s));
        for (int cc = 0; cc < sd.ncomp; ++cc) {
            double2* res = nullptr;
            OCCRIK_HIP(launch_colloc_kdft(P->cphi + (size_t)cc * P->nk * cnt, P->cw0, P->cw1, g, s, &res));
            OCCRIK_HIP(launch_colloc_store<T>(res, dst, mu0 + cc, P->nao, ldc, coff, g, s));
        }
        mu0 += sd.ncomp;
    }
    return OCCRIK_OK;
}

occrik_status alloc_colloc_scratch(occrik_plan* P) {
    OCCRIK_HIP(P->alloc((void**)&P->cphi, sizeof(double) * P->maxcomp * (size_t)P->nk * P->cchunk));
    OCCRIK_HIP(P->alloc((void**)&P->cw0, sizeof(double2) * (size_t)P->nk * P->cchunk));
    OCCRIK_HIP(P->alloc((void**)&P->cw1, sizeof(double2) * (size_t)P->nk * P->cchunk));
    return OCCRIK_OK;
}

// stored mode: collocate chi~ once, chunk by chunk, then drop the scratch.  The
// chunks here only bound the scratch (2 GiB), so they are larger than the direct
// mode's; every value is computed per point, so the chunking changes no result.
template <typename T>
occrik_status run_collocation(occrik_plan* P) {
    {
        const int cc = contract_chunk(P->ng, P->nchunks);
        const size_t per_point = (sizeof(double) * P->maxcomp + 2 * sizeof(double2)) * (size_t)P->nk;
        const size_t q = std::max<size_t>(1, ((size_t)2 << 30) / (per_point * cc));
        P->cchunk = (int)std::min<size_t>((size_t)P->ng, q * cc);
    }
    occrik_status st = alloc_colloc_scratch(P);
    for (int n0 = 0; st == OCCRIK_OK && n0 < P->ng; n0 += P->cchunk)
        st = collocate_range<T>(P, n0, std::min(P->cchunk, P->ng - n0), reinterpret_cast<cplx<T>*>(P->chi),
                                (size_t)P->ng, (size_t)n0);
    if (st != OCCRIK_OK) return st;
    OCCRIK_HIP(hipStreamSynchronize(P->stream));
    P->release(P->cphi);
    P->release(P->cw0);
    P->release(P->cw1);
    P->cphi = nullptr;
    P->cw0 = P->cw1 = nullptr;
    return OCCRIK_OK;
}

template <typename T>
occrik_status make_twiddles(occrik_plan* P) {
    std::vector<cplx<T>> h(3 * kMaxN);
    for (int d = 0; d < 3; ++d)
        for (int t = 0; t < kMaxN; ++t) {
            cplx<T> v;
            if (t < P->N[d]) {
                const double a = -2.0 * M_PI * double(t) / double(P->N[d]);
                v.x = T(std::cos(a));
                v.y = T(std::sin(a));
            } else {
                v.x = T(0);
                v.y = T(0);
            }
            h[d * kMaxN + t] = v;
        }
    OCCRIK_HIP(hipMemcpy(P->tw, h.data(), sizeof(cplx<T>) * h.size(), hipMemcpyHostToDevice));
    return OCCRIK_OK;
}

// conjugate-pair reuse needs exact conjugate pairs (symmetric Nyquist mode) and a square
// pair set: with conduction bands the mirror of an (occupied, virtual) pair is not summed
bool plan_reuses_pairs(const occrik_plan* P) {
    return P->params.nyquist == OCCRIK_NYQUIST_SYMMETRIC && P->nvir == 0;
}

int splits_for(const occrik_plan* P, int nb) {
    PairBatch B{};
    B.N1 = P->N[0];
    B.N2 = P->N[1];
    B.N3 = P->N[2];
    B.nocc = P->nocc;
    B.nout = P->nout;
    B.nb = nb;
    return pass3_splits(B, (int)P->elem);
}

// occ_only: pairs with occupied output orbitals only (the energy-derivative sweep)
PairBatch make_batch(const occrik_plan* P, int a, int b0, int nb, bool occ_only = false) {
    PairBatch B{};
    B.N1 = P->N[0];
    B.N2 = P->N[1];
    B.N3 = P->N[2];
    B.ng = P->ng;
    B.M1 = P->M[0];
    B.M2 = P->M[1];
    B.M3 = P->M[2];
    B.nocc = P->nocc;
    B.nout = occ_only ? P->nocc : P->nout;
    B.kstride = P->nout;
    B.a = a;
    B.b0 = b0;
    B.nb = nb;
    B.reuse = plan_reuses_pairs(P) ? 1 : 0;
    B.diag = (B.reuse && b0 == a) ? 1 : 0;
    B.ntri = P->nocc * (P->nocc + 1) / 2;
    const int nn = B.nocc * B.nout;
    B.nslots = B.diag ? B.ntri + (nb - 1) * nn : nb * nn;
    // stored pairs per pass-2 workgroup, complex64: up to 4 x nout (a workgroup's set-up,
    // its kernel values, twiddles and first slab load, is shared by more pairs) while the
    // launch keeps at least 2048 workgroups; never fewer pairs than the plan's own group (the
    // partial-sum buffer of the omega sweep is sized for that). Complex128 keeps the plan's
    // group: its pass 2 measured slower with the larger ones.
    B.group = P->group;
    for (int f = 4; f > 1 && !P->fp64; f /= 2) {
        if ((size_t)B.N2 * nb * nn / ((size_t)P->group * f) >= 2048) {
            B.group = P->group * f;
            break;
        }
    }
    B.kernel = P->params.kernel;
    B.nyquist = P->params.nyquist;
    B.omega = P->params.omega;
    B.rcut = std::cbrt(3.0 * double(P->nk) * P->volume / (4.0 * M_PI));
    B.madelung = P->madelung_g0 != 0.0 ? 1 : 0;
    B.g0 = P->madelung_g0;
    B.inv_ng = 1.0 / P->ng;
    std::memcpy(B.recip, P->recip, sizeof(B.recip));
    B.splits = splits_for(P, nb);
    B.parseval = 0;
    B.regfft = !P->regfft ? 0
               : (P->params.flags & OCCRIK_FLAG_REG_FFT_ALL) ? (REGFFT_PASS1 | REGFFT_PASS2 | REGFFT_PASS3)
                                                              : REGFFT_DEFAULT;
    B.kvals = P->kvals;
    if (P->kcache && !occ_only) {
        B.kvals = P->kcache;
        B.kcache = 1;
    }
    const char* psi = static_cast<const char*>(P->psi);
    B.outp = psi + (size_t)a * B.kstride * B.ng * P->elem;
    B.accp = psi;
    B.woff = (size_t)a * B.kstride * B.ng;
    return B;
}

// Stages of a build.  A batch recorded with fused rounds runs the prologue and the
// epilogue of each plan through build_impl and the pair loop of several plans at once.
enum : int { kStagePrologue = 1, kStagePairs = 2, kStageEpilogue = 4, kStageAll = 7 };

// the pair-pass launches of one build, in the order the pair loop issues them
std::vector<PairBatch> plan_launches(const occrik_plan* P) {
    std::vector<PairBatch> v;
    const bool reuse = plan_reuses_pairs(P);
    for (int a = 0; a < P->nk; ++a)
        for (int b0 = reuse ? a : 0; b0 < P->nk; b0 += P->kbatch)
            v.push_back(make_batch(P, a, b0, std::min(P->kbatch, P->nk - b0)));
    return v;
}

template <typename T>
occrik_status build_impl(occrik_plan* P, const double2* dC, double2* dK, double2* dKmi, double* dEx,
                         int stages = kStageAll) {
    if (stages != kStageAll && P->profiling) return fail(OCCRIK_ERR_INVALID_ARG, "profiling needs whole builds");
    hipStream_t s = P->stream;
    const int nk = P->nk, nao = P->nao, nocc = P->nout, ng = P->ng;   // nocc here: columns of C
    cplx<T>* chi = reinterpret_cast<cplx<T>*>(P->chi);
    cplx<T>* psi = reinterpret_cast<cplx<T>*>(P->psi);
    cplx<T>* W = reinterpret_cast<cplx<T>*>(P->W);
    cplx<T>* X = reinterpret_cast<cplx<T>*>(P->X);
    cplx<T>* Wp = reinterpret_cast<cplx<T>*>(P->Wpart);
    const cplx<T>* tw = reinterpret_cast<const cplx<T>*>(P->tw);
    ProfileEvents pe{};
    if (P->profiling) {
        for (auto& e : pe.e) OCCRIK_HIP(hipEventCreate(&e));
        OCCRIK_HIP(hipEventRecord(pe.e[0], s));
    }
    if (stages & kStagePrologue) {
        OCCRIK_HIP(launch_reset_flags_n(P->flags, 2 + nk, s));
        OCCRIK_HIP(launch_check_finite(dC, (size_t)nk * nao * nocc, P->flags, s));
        if (P->direct) {
            cplx<T>* ws = reinterpret_cast<cplx<T>*>(P->chi_ws);
            for (int n0 = 0; n0 < ng; n0 += P->cchunk) {
                const int cnt = std::min(P->cchunk, ng - n0);
                const occrik_status st = collocate_range<T>(P, n0, cnt, ws, (size_t)cnt, 0);
                if (st != OCCRIK_OK) return st;
                OCCRIK_HIP(launch_orbitals<T>(ws, (size_t)cnt, dC, psi, nk, nao, nocc, ng, n0, cnt,
                                              P->params.precision, s));
            }
        } else {
            OCCRIK_HIP(launch_orbitals<T>(chi, (size_t)ng, dC, psi, nk, nao, nocc, ng, 0, ng, P->params.precision, s));
        }
        if (P->profiling) OCCRIK_HIP(hipEventRecord(pe.e[1], s));
        OCCRIK_HIP(launch_fill_zero<T>(W, (size_t)nk * nocc * ng, s));
        // kernel values of every k-point difference, once per omega; under stream capture the
        // fill is recorded into the graph (and replayed with it) and the plan stays unfilled
        if (P->kcache && (!P->kcache_valid || P->kcache_omega != P->params.omega)) {
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            OCCRIK_HIP(hipStreamIsCapturing(s, &cs));
            OCCRIK_HIP(launch_kcache<T>(make_batch(P, 0, 0, 1), P->kcache, s));
            if (cs == hipStreamCaptureStatusNone) {
                P->kcache_valid = true;
                P->kcache_omega = P->params.omega;
            }
        }
    }
    int64_t launches = 1;
    const bool reuse = plan_reuses_pairs(P);
    for (int a = 0; a < nk && (stages & kStagePairs); ++a) {
        for (int b0 = reuse ? a : 0; b0 < nk; b0 += P->kbatch) {
            const int nb = std::min(P->kbatch, nk - b0);
            PairBatch B = make_batch(P, a, b0, nb);
            hipEvent_t ev[4] = {};
            if (P->profiling >= 2) {
                for (auto& e : ev) {
                    OCCRIK_HIP(hipEventCreate(&e));
                    pe.pe.push_back(e);
                }
                const double pb = double(B.nslots) * ng * sizeof(cplx<T>);
                pe.pbytes.push_back(pb);
                pe.pbytes.push_back(2.0 * pb);
                pe.pbytes.push_back(pb);
                OCCRIK_HIP(hipEventRecord(ev[0], s));
            }
            OCCRIK_HIP(launch_pass1<T>(B, psi, X, tw, s));
            if (P->profiling >= 2) OCCRIK_HIP(hipEventRecord(ev[1], s));
            OCCRIK_HIP(launch_pass2<T>(B, X, tw, P->parts, 0, s));
            if (P->profiling >= 2) OCCRIK_HIP(hipEventRecord(ev[2], s));
            OCCRIK_HIP(launch_pass3<T>(B, X, psi, Wp, W, tw, s));
            OCCRIK_HIP(launch_wreduce<T>(B, Wp, W, s));
            if (P->profiling >= 2) OCCRIK_HIP(hipEventRecord(ev[3], s));
            launches += 4;
        }
    }
    if (!(stages & kStageEpilogue)) return OCCRIK_OK;
    if (P->profiling) OCCRIK_HIP(hipEventRecord(pe.e[2], s));
    {
        const int chunk = contract_chunk(ng, P->nchunks);
        if (P->direct) {
            cplx<T>* ws = reinterpret_cast<cplx<T>*>(P->chi_ws);
            for (int n0 = 0; n0 < ng; n0 += P->cchunk) {
                const int cnt = std::min(P->cchunk, ng - n0);
                const occrik_status st = collocate_range<T>(P, n0, cnt, ws, (size_t)cnt, 0);
                if (st != OCCRIK_OK) return st;
                const int c0 = n0 / chunk, c1 = std::min(P->nchunks, (n0 + cnt + chunk - 1) / chunk);
                OCCRIK_HIP(launch_contract_part<T>(ws, (size_t)cnt, n0, W, P->Kpart, nk, nao, nocc, ng, P->nchunks, c0,
                                                   c1 - c0, P->params.precision, s));
            }
        } else {
            OCCRIK_HIP(launch_contract_part<T>(chi, (size_t)ng, 0, W, P->Kpart, nk, nao, nocc, ng, P->nchunks, 0,
                                               P->nchunks, P->params.precision, s));
        }
        OCCRIK_HIP(launch_contract_reduce(P->Kpart, P->Kmi, (size_t)nk * nao * nocc, P->nchunks, -P->dv / nk, s));
    }
    if (P->profiling) OCCRIK_HIP(hipEventRecord(pe.e[3], s));
    // a copy kernel rather than a memcpy, so that a captured build holds kernel nodes only
    if (dKmi) OCCRIK_HIP(launch_scale_copy(P->Kmi, (double2*)dKmi, (size_t)nk * nao * nocc, 1.0, s));
    OCCRIK_HIP(launch_kij(dC, P->Kmi, P->Kij, P->L, P->eterm, P->flags, nk, nao, nocc, P->nocc, s));
    if (dK) {
        OCCRIK_HIP(launch_xi(P->Kmi, P->L, P->Y, P->flags, nk, nao, nocc, s));
        OCCRIK_HIP(launch_ktilde(P->Y, dK, P->flags, nk, nao, nocc, s));
    }
    if (dEx) OCCRIK_HIP(launch_energy(P->eterm, nk, dEx, s));
    if (P->profiling) {
        OCCRIK_HIP(hipEventRecord(pe.e[4], s));
        pe.pair_launches = launches;
        P->prof.push_back(std::move(pe));
    }
    P->built = true;
    return OCCRIK_OK;
}

template <typename T>
occrik_status domega_impl(occrik_plan* P, double* out_host) {
    hipStream_t s = P->stream;
    const int nk = P->nk;
    cplx<T>* psi = reinterpret_cast<cplx<T>*>(P->psi);
    cplx<T>* X = reinterpret_cast<cplx<T>*>(P->X);
    const cplx<T>* tw = reinterpret_cast<const cplx<T>*>(P->tw);
    OCCRIK_HIP(launch_fill_zero_f64(P->scal, 4, s));
    const double scale = -P->volume / (2.0 * double(nk) * nk * double(P->ng) * P->ng);
    const bool reuse = plan_reuses_pairs(P);
    for (int a = 0; a < nk; ++a)
        for (int b0 = reuse ? a : 0; b0 < nk; b0 += P->kbatch) {
            const int nb = std::min(P->kbatch, nk - b0);
            PairBatch B = make_batch(P, a, b0, nb, true);
            OCCRIK_HIP(launch_pass1<T>(B, psi, X, tw, s));
            OCCRIK_HIP(launch_pass2<T>(B, X, tw, P->parts, 1, s));
            OCCRIK_HIP(launch_sum_f64(P->parts, (size_t)pair_groups(B) * P->N[1], scale, P->scal, s));
        }
    OCCRIK_HIP(hipMemcpyAsync(out_host, P->scal, sizeof(double), hipMemcpyDeviceToHost, s));
    OCCRIK_HIP(hipStreamSynchronize(s));
    return OCCRIK_OK;
}

// ---------------------------------------------------------------------------
// conventional exchange: AO-RI-K (Sec. II.B, Alg. 1) and MO-RI-K (Sec. II.C, Alg. 2)
// ---------------------------------------------------------------------------
// Pair passes of output k-point a, output AOs [j0, j0 + g), summed k-points [b0, b0 + nb).
// MO-RI-K: densities conj(psi_{i b}) chi_{mu a}, W_mu += psi_{i b} V (eq. mointerm2).
// AO-RI-K: densities conj(chi_{sigma b}) chi_{mu a}, V~_mu += psi~_{sigma b} V (eq. aointerm2).
PairBatch make_conv_batch(const occrik_plan* P, int algo, int a, int j0, int g, int b0, int nb) {
    PairBatch B{};
    B.N1 = P->N[0];
    B.N2 = P->N[1];
    B.N3 = P->N[2];
    B.ng = P->ng;
    B.M1 = P->M[0];
    B.M2 = P->M[1];
    B.M3 = P->M[2];
    const bool ao = algo == OCCRIK_ALGO_AO_RI_K;
    B.nocc = ao ? P->nao : P->nocc;
    B.nout = g;
    B.kstride = ao ? P->nao : P->nout;
    B.a = a;
    B.b0 = b0;
    B.nb = nb;
    B.reuse = 0;
    B.diag = 0;
    B.ntri = B.nocc * (B.nocc + 1) / 2;
    B.nslots = nb * B.nocc * g;
    B.group = g;
    B.kernel = P->params.kernel;
    B.nyquist = P->params.nyquist;
    B.omega = P->params.omega;
    B.rcut = std::cbrt(3.0 * double(P->nk) * P->volume / (4.0 * M_PI));
    B.madelung = P->madelung_g0 != 0.0 ? 1 : 0;
    B.g0 = P->madelung_g0;
    B.inv_ng = 1.0 / P->ng;
    std::memcpy(B.recip, P->recip, sizeof(B.recip));
    B.splits = pass3_splits(B, (int)P->elem);
    B.parseval = 0;
    B.regfft = 0;
    B.kvals = P->conv_kvals;
    const size_t e = P->elem;
    B.outp = static_cast<const char*>(P->chi) + ((size_t)a * P->nao + j0) * P->ng * e;
    B.accp = ao ? P->conv_psit : P->conv_psi;
    B.woff = (size_t)j0 * P->ng;
    return B;
}

// workspaces of the conventional passes, grown on demand
occrik_status conv_workspace(occrik_plan* P, int algo) {
    const int nk = P->nk, nao = P->nao, ng = P->ng;
    const size_t e = P->elem;
    const int nsum = algo == OCCRIK_ALGO_AO_RI_K ? nao : P->nocc;
    hipError_t err = hipSuccess;
    auto A = [&](void** p, size_t bytes) {
        if (err == hipSuccess && *p == nullptr) err = P->alloc(p, bytes);
    };
    A(&P->conv_psi, (size_t)nk * P->nout * ng * e);
    A(&P->conv_W, (size_t)nao * ng * e);
    A((void**)&P->conv_Kpart, sizeof(double2) * (size_t)nao * 16 * P->nchunks);
    if (algo == OCCRIK_ALGO_AO_RI_K) A(&P->conv_psit, (size_t)nk * nao * ng * e);
    if (err != hipSuccess) return hip_fail(err, "conventional workspace");
    if (nsum > P->conv_nsum) {
        P->release(P->conv_X);
        P->release(P->conv_Wpart);
        P->release(P->conv_kvals);
        P->conv_X = P->conv_Wpart = P->conv_kvals = nullptr;
        const size_t per_block = (size_t)nsum * kConvGroup * ng * e;
        const size_t cap = (size_t)4 << 30;
        P->conv_kbatch = (int)std::max<size_t>(1, std::min<size_t>((size_t)nk, cap / per_block));
        PairBatch B = make_conv_batch(P, algo, 0, 0, kConvGroup, 0, P->conv_kbatch);
        A(&P->conv_X, (size_t)P->conv_kbatch * per_block);
        A(&P->conv_Wpart, (size_t)B.splits * kConvGroup * ng * e);
        A(&P->conv_kvals, e / 2 * (size_t)P->conv_kbatch * ng);
        if (err != hipSuccess) {
            P->conv_nsum = 0;
            return hip_fail(err, "conventional workspace");
        }
        P->conv_nsum = nsum;
    }
    return OCCRIK_OK;
}

template <typename T>
occrik_status conventional_impl(occrik_plan* P, int algo, const double2* dC, double2* dK, double* dEx) {
    hipStream_t s = P->stream;
    const int nk = P->nk, nao = P->nao, ng = P->ng, ncol = P->nout;
    occrik_status st = conv_workspace(P, algo);
    if (st != OCCRIK_OK) return st;
    const cplx<T>* chi = reinterpret_cast<const cplx<T>*>(P->chi);
    cplx<T>* psi = reinterpret_cast<cplx<T>*>(P->conv_psi);
    cplx<T>* Wa = reinterpret_cast<cplx<T>*>(P->conv_W);
    cplx<T>* X = reinterpret_cast<cplx<T>*>(P->conv_X);
    cplx<T>* Wp = reinterpret_cast<cplx<T>*>(P->conv_Wpart);
    const cplx<T>* tw = reinterpret_cast<const cplx<T>*>(P->tw);
    const bool ao = algo == OCCRIK_ALGO_AO_RI_K;
    // eq. occmo, then (AO-RI-K) eq. aointerm
    OCCRIK_HIP(launch_orbitals<T>(chi, (size_t)ng, dC, psi, nk, nao, ncol, ng, 0, ng, P->params.precision, s));
    if (ao)
        OCCRIK_HIP(launch_density_orbitals<T>(dC, psi, reinterpret_cast<cplx<T>*>(P->conv_psit), nk, nao, ncol,
                                              P->nocc, ng, s));
    // the summed side's densities: occupied orbitals (MO-RI-K) or AOs (AO-RI-K)
    const cplx<T>* dens = ao ? chi : psi;
    for (int a = 0; a < nk; ++a) {
        OCCRIK_HIP(launch_fill_zero<T>(Wa, (size_t)nao * ng, s));
        for (int j0 = 0; j0 < nao; j0 += kConvGroup) {
            const int g = std::min(kConvGroup, nao - j0);
            for (int b0 = 0; b0 < nk; b0 += P->conv_kbatch) {
                const int nb = std::min(P->conv_kbatch, nk - b0);
                const PairBatch B = make_conv_batch(P, algo, a, j0, g, b0, nb);
                OCCRIK_HIP(launch_pass1<T>(B, dens, X, tw, s));
                OCCRIK_HIP(launch_pass2<T>(B, X, tw, P->parts, 0, s));
                OCCRIK_HIP(launch_pass3<T>(B, X, dens, Wp, Wa, tw, s));
                OCCRIK_HIP(launch_wreduce<T>(B, Wp, Wa, s));
            }
        }
        // eq. aok: K_{nu mu}(k_a) = -(dV/N_k) sum_r conj(chi_{nu a}) W_mu, 16 columns per contraction
        const cplx<T>* chia = chi + (size_t)a * nao * ng;
        for (int j0 = 0; j0 < nao; j0 += 16) {
            const int g = std::min(16, nao - j0);
            OCCRIK_HIP(launch_contract_part<T>(chia, (size_t)ng, 0, Wa + (size_t)j0 * ng, P->conv_Kpart, 1, nao, g,
                                               ng, P->nchunks, 0, P->nchunks, P->params.precision, s));
            OCCRIK_HIP(launch_reduce_columns(P->conv_Kpart, dK + (size_t)a * nao * nao, nao, g, nao, j0,
                                             P->nchunks, -P->dv / nk, s));
        }
    }
    if (dEx) {
        OCCRIK_HIP(launch_conv_energy(dC, dK, P->eterm, nk, nao, ncol, P->nocc, s));
        OCCRIK_HIP(launch_energy(P->eterm, nk, dEx, s));
    }
    return OCCRIK_OK;
}

occrik_status validate(const occrik_cell* cell, const occrik_basis* basis, const occrik_params* pr) {
    if (!cell || !basis || !pr) return fail(OCCRIK_ERR_INVALID_ARG, "null cell, basis or params");
    double inv[9];
    for (double v : cell->lattice)
        if (!std::isfinite(v)) return fail(OCCRIK_ERR_INVALID_ARG, "non-finite lattice");
    if (!invert3(cell->lattice, inv)) return fail(OCCRIK_ERR_INVALID_ARG, "singular lattice");
    if (cell->natm < 1 || !cell->atom_frac) return fail(OCCRIK_ERR_INVALID_ARG, "no atoms");
    for (int i = 0; i < 3 * cell->natm; ++i)
        if (!std::isfinite(cell->atom_frac[i])) return fail(OCCRIK_ERR_INVALID_ARG, "non-finite atom position");
    if (basis->nshell < 1 || !basis->shell_atom || !basis->shell_l || !basis->shell_exp)
        return fail(OCCRIK_ERR_INVALID_ARG, "empty basis");
    for (int s = 0; s < basis->nshell; ++s) {
        if (basis->shell_atom[s] < 0 || basis->shell_atom[s] >= cell->natm)
            return fail(OCCRIK_ERR_INVALID_ARG, "shell_atom out of range");
        if (basis->shell_l[s] < 0) return fail(OCCRIK_ERR_INVALID_ARG, "negative shell_l");
        if (basis->shell_l[s] > 3) return fail(OCCRIK_ERR_UNSUPPORTED, "shell_l > 3");
        if (!(basis->shell_exp[s] > 0.0) || !std::isfinite(basis->shell_exp[s]))
            return fail(OCCRIK_ERR_INVALID_ARG, "shell exponent must be positive and finite");
    }
    for (int d = 0; d < 3; ++d) {
        if (pr->kmesh[d] < 1 || pr->kmesh[d] > 16) return fail(OCCRIK_ERR_INVALID_ARG, "kmesh entries must be 1..16");
        if (pr->grid[d] < 1) return fail(OCCRIK_ERR_INVALID_ARG, "grid entries must be >= 1");
        if (!grid_size_supported(pr->grid[d]))
            return fail(OCCRIK_ERR_UNSUPPORTED, "grid size " + std::to_string(pr->grid[d]) + " not supported");
    }
    if (pr->nocc < 1 || pr->nocc > 16) return fail(OCCRIK_ERR_INVALID_ARG, "nocc must be 1..16");
    if (pr->nvir < 0 || pr->nocc + pr->nvir > 16)
        return fail(OCCRIK_ERR_INVALID_ARG, "nvir must be >= 0 with nocc + nvir <= 16");
    if (pr->kernel < 0 || pr->kernel > 4) return fail(OCCRIK_ERR_INVALID_ARG, "unknown kernel");
    const bool range_separated = pr->kernel == OCCRIK_KERNEL_ERF_LR || pr->kernel == OCCRIK_KERNEL_ERFC_SR ||
                                 pr->kernel == OCCRIK_KERNEL_TRUNC_ERF_LR;
    if (range_separated && !(pr->omega > 0.0 && std::isfinite(pr->omega)))
        return fail(OCCRIK_ERR_INVALID_ARG, "omega must be positive for range-separated kernels");
    if (pr->nyquist < 0 || pr->nyquist > 1) return fail(OCCRIK_ERR_INVALID_ARG, "unknown nyquist mode");
    if (pr->precision < 0 || pr->precision > 2) return fail(OCCRIK_ERR_INVALID_ARG, "unknown precision");
    if (!(pr->lattice_tol > 0.0 && pr->lattice_tol <= 1e-3)) return fail(OCCRIK_ERR_INVALID_ARG, "lattice_tol");
    if (pr->flags & ~(OCCRIK_FLAG_LDS_FFT | OCCRIK_FLAG_REG_FFT_ALL | OCCRIK_FLAG_DIRECT | OCCRIK_FLAG_MADELUNG))
        return fail(OCCRIK_ERR_INVALID_ARG, "unknown bits in flags");
    if ((pr->flags & OCCRIK_FLAG_LDS_FFT) && (pr->flags & OCCRIK_FLAG_REG_FFT_ALL))
        return fail(OCCRIK_ERR_INVALID_ARG, "OCCRIK_FLAG_LDS_FFT and OCCRIK_FLAG_REG_FFT_ALL exclude each other");
    if (pr->kbatch < 0) return fail(OCCRIK_ERR_INVALID_ARG, "kbatch must be >= 0");
    if (pr->contract_chunks < 0 || pr->contract_chunks > kMaxContractChunks)
        return fail(OCCRIK_ERR_INVALID_ARG, "contract_chunks must be 0..64");
    return OCCRIK_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* occrik_status_string(occrik_status s) {
    switch (s) {
        case OCCRIK_OK: return "OCCRIK_OK";
        case OCCRIK_ERR_INVALID_ARG: return "OCCRIK_ERR_INVALID_ARG";
        case OCCRIK_ERR_UNSUPPORTED: return "OCCRIK_ERR_UNSUPPORTED";
        case OCCRIK_ERR_OOM: return "OCCRIK_ERR_OOM";
        case OCCRIK_ERR_NOT_PD: return "OCCRIK_ERR_NOT_PD";
        case OCCRIK_ERR_NONFINITE: return "OCCRIK_ERR_NONFINITE";
        case OCCRIK_ERR_DEVICE: return "OCCRIK_ERR_DEVICE";
        case OCCRIK_ERR_STATE: return "OCCRIK_ERR_STATE";
    }
    return "OCCRIK_UNKNOWN";
}

const char* occrik_last_error_message(void) { return g_last_error.c_str(); }

int32_t occrik_grid_size_supported(int32_t n) { return grid_size_supported(n) ? 1 : 0; }

occrik_status occrik_plan_create(const occrik_cell* cell, const occrik_basis* basis, const occrik_params* params,
                                 int device, void* stream, occrik_plan** out) {
    if (!out) return fail(OCCRIK_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    occrik_status st = validate(cell, basis, params);
    if (st != OCCRIK_OK) return st;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(OCCRIK_ERR_DEVICE, "no HIP device");
    if (device < 0 || device >= ndev) return fail(OCCRIK_ERR_INVALID_ARG, "device ordinal out of range");
    const auto t0 = std::chrono::steady_clock::now();
    DeviceGuard guard(device);
    auto* P = new occrik_plan();
    P->device = device;
    P->stream = reinterpret_cast<hipStream_t>(stream);
    P->params = *params;
    std::memcpy(P->lat, cell->lattice, sizeof(P->lat));
    double inv[9];
    invert3(P->lat, inv);
    // b_d = 2 pi (A^{-1})^T rows: recip[d][e] = 2 pi inv[e][d]
    for (int d = 0; d < 3; ++d)
        for (int e = 0; e < 3; ++e) P->recip[3 * d + e] = 2.0 * M_PI * inv[3 * e + d];
    const double det = P->lat[0] * (P->lat[4] * P->lat[8] - P->lat[5] * P->lat[7]) -
                       P->lat[1] * (P->lat[3] * P->lat[8] - P->lat[5] * P->lat[6]) +
                       P->lat[2] * (P->lat[3] * P->lat[7] - P->lat[4] * P->lat[6]);
    P->volume = std::fabs(det);
    for (int d = 0; d < 3; ++d) {
        P->N[d] = params->grid[d];
        P->M[d] = params->kmesh[d];
    }
    P->nk = P->M[0] * P->M[1] * P->M[2];
    P->ng = P->N[0] * P->N[1] * P->N[2];
    P->dv = P->volume / P->ng;
    if (params->flags & OCCRIK_FLAG_MADELUNG) {
        double sup[9];
        for (int d = 0; d < 3; ++d)
            for (int e = 0; e < 3; ++e) sup[3 * d + e] = P->M[d] * P->lat[3 * d + e];
        P->madelung_g0 = double(P->nk) * P->volume * madelung_constant(sup);
    }
    P->natm = cell->natm;
    P->atom_cart.resize(3 * P->natm);
    for (int a = 0; a < P->natm; ++a)
        for (int e = 0; e < 3; ++e) {
            double x = 0.0;
            for (int d = 0; d < 3; ++d) x += cell->atom_frac[3 * a + d] * P->lat[3 * d + e];
            P->atom_cart[3 * a + e] = x;
        }
    P->shell_atom.assign(basis->shell_atom, basis->shell_atom + basis->nshell);
    P->shell_l.assign(basis->shell_l, basis->shell_l + basis->nshell);
    P->shell_exp.assign(basis->shell_exp, basis->shell_exp + basis->nshell);
    P->nao = 0;
    for (int l : P->shell_l) {
        P->nao += (l + 1) * (l + 2) / 2;
        P->maxcomp = std::max(P->maxcomp, (l + 1) * (l + 2) / 2);
    }
    P->nocc = params->nocc;
    P->nvir = params->nvir;
    P->nout = P->nocc + P->nvir;
    if (P->nout > P->nao) {
        delete P;
        return fail(OCCRIK_ERR_INVALID_ARG, "nocc + nvir exceeds the number of AOs");
    }
    P->fp64 = params->precision == OCCRIK_PREC_FP64;
    P->elem = P->fp64 ? 16 : 8;
    P->regfft = !P->fp64 && !(params->flags & OCCRIK_FLAG_LDS_FFT) && params->nvir == 0 &&
                reg_fft_size(params->grid[0], params->grid[1], params->grid[2]);

    const int nk = P->nk, ng = P->ng, nao = P->nao, nocc = P->nocc, nout = P->nout;
    const size_t per_k = (size_t)nocc * nout * ng * P->elem;
    if (params->kbatch > 0) {
        P->kbatch = std::min(params->kbatch, nk);
    } else {
        const size_t cap = (size_t)32 << 30;   // exchange buffer of one batch: a whole k row at the paper size in FP64
        P->kbatch = (int)std::max<size_t>(1, std::min<size_t>((size_t)nk, cap / per_k));
    }
    P->kbatch_max = P->kbatch;
    P->splits = splits_for(P, P->kbatch);
    P->group = nout;
    // every chunk holds grid points: the integral-direct contraction launches only the
    // chunks a collocation chunk covers, so an empty trailing chunk would never be written.
    // By default one chunk per 4096 points, and more (up to 64) where that leaves the
    // contraction's launch (chunks x 64-AO blocks x k-points) below 2048 workgroups: a
    // small cell's few long-running workgroups would leave most of the chip idle.
    const int wg_per_chunk = nk * ((nao + 63) / 64);
    const int nchunks_default = std::max(1, std::min(64, std::max(ng / 4096, (2048 + wg_per_chunk - 1) / wg_per_chunk)));
    P->nchunks = contract_chunk_count(ng, params->contract_chunks > 0 ? params->contract_chunks : nchunks_default);
    const size_t max_groups = (size_t)P->kbatch * ((nocc * nout + P->group - 1) / P->group) +
                              (nocc * (nocc + 1) / 2 + P->group - 1) / P->group;

    hipError_t e = hipSuccess;
    auto A = [&](void** p, size_t bytes) {
        if (e == hipSuccess) e = P->alloc(p, bytes);
    };
    // Collocation chunk: whole partial-sum chunks of the contraction, with chi~ of a
    // chunk for every k and AO (the direct mode's workspace) within 2 GiB, or within
    // an eighth of mem_budget when that is smaller.
    {
        const int cc = contract_chunk(ng, P->nchunks);
        const size_t per_point = (size_t)nk * nao * P->elem;
        size_t cap = (size_t)2 << 30;
        if (params->mem_budget != 0) cap = std::min(cap, params->mem_budget / 8);
        const size_t q = std::max<size_t>(1, cap / (per_point * cc));
        P->cchunk = (int)std::min<size_t>((size_t)ng, q * cc);
    }
    // Integral-direct (Sec. II.E, Alg. 4) when asked for, or when the stored chi~
    // would not fit next to the other workspaces: within mem_budget when one is
    // set, else within the device memory free now.
    const size_t bytes_chi_stored = (size_t)nk * nao * ng * P->elem;
    const size_t bytes_other = (size_t)nk * nout * ng * P->elem * 2 + (size_t)P->kbatch * per_k +
                               (size_t)P->splits * nout * ng * P->elem + sizeof(double2) * (size_t)nk * nao * nout *
                               (P->nchunks + 2) + P->elem / 2 * (size_t)P->kbatch * ng;
    const size_t bytes_scratch = (sizeof(double) * P->maxcomp + 2 * sizeof(double2)) * (size_t)nk * P->cchunk;
    P->direct = (params->flags & OCCRIK_FLAG_DIRECT) != 0;
    if (!P->direct) {
        size_t avail = params->mem_budget;
        if (avail == 0) {
            size_t fr = 0, tot = 0;
            if (hipMemGetInfo(&fr, &tot) == hipSuccess) avail = fr;
        }
        if (avail != 0 && bytes_chi_stored + bytes_other + bytes_scratch > avail) P->direct = true;
    }
    if (P->direct) {
        P->bytes_chi = 0;
        A(&P->chi_ws, (size_t)nk * nao * P->cchunk * P->elem);
    } else {
        P->bytes_chi = bytes_chi_stored;
        A(&P->chi, P->bytes_chi);
    }
    A(&P->psi, (size_t)nk * nout * ng * P->elem);
    A(&P->W, (size_t)nk * nout * ng * P->elem);
    A(&P->X, (size_t)P->kbatch * per_k);
    A(&P->Wpart, (size_t)P->splits * nout * ng * P->elem);
    A(&P->tw, 3 * kMaxN * P->elem);
    A((void**)&P->parts, sizeof(double) * max_groups * P->N[1]);
    A(&P->kvals, P->elem / 2 * (size_t)P->kbatch * ng);
    // kernel values of every k-point difference when they take at most 2 GiB (at the paper
    // size 1331 tables, 0.59 GB in FP32); otherwise every batch evaluates its own
    {
        const size_t kc = P->elem / 2 * kcache_tables(P->M[0], P->M[1], P->M[2]) * ng;
        if (e == hipSuccess && kc <= ((size_t)2 << 30)) {
            if (P->alloc(&P->kcache, kc) != hipSuccess) {
                (void)hipGetLastError();
                P->kcache = nullptr;
            }
        }
    }
    A((void**)&P->Kpart, sizeof(double2) * (size_t)nk * nao * nout * P->nchunks);
    P->kpart_chunks = P->nchunks;
    A((void**)&P->Kmi, sizeof(double2) * (size_t)nk * nao * nout);
    A((void**)&P->Kij, sizeof(double2) * (size_t)nk * nout * nout);
    A((void**)&P->L, sizeof(double2) * (size_t)nk * nout * nout);
    A((void**)&P->Y, sizeof(double2) * (size_t)nk * nao * nout);
    A((void**)&P->eterm, sizeof(double) * nk);
    A((void**)&P->scal, sizeof(double) * 4);
    A((void**)&P->flags, sizeof(int) * (2 + nk));
    if (e != hipSuccess) {
        delete P;
        return hip_fail(e, "plan allocation");
    }
    e = launch_reset_flags_n(P->flags, 2 + nk, P->stream);
    if (e != hipSuccess) {
        delete P;
        return hip_fail(e, "flag initialisation");
    }
    st = P->fp64 ? make_twiddles<double>(P) : make_twiddles<float>(P);
    if (st == OCCRIK_OK) st = build_colloc_tables(P);
    if (st == OCCRIK_OK) {
        if (P->direct) st = alloc_colloc_scratch(P);
        else st = P->fp64 ? run_collocation<double>(P) : run_collocation<float>(P);
    }
    if (st != OCCRIK_OK) {
        delete P;
        return st;
    }
    P->plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = P;
    return OCCRIK_OK;
}

void occrik_plan_destroy(occrik_plan* plan) {
    if (!plan) return;
    DeviceGuard guard(plan->device);
    (void)hipStreamSynchronize(plan->stream);
    delete plan;
}

occrik_status occrik_plan_query(const occrik_plan* P, occrik_plan_info* info) {
    if (!P || !info) return fail(OCCRIK_ERR_INVALID_ARG, "null plan or info");
    info->nk = P->nk;
    info->nao = P->nao;
    info->nocc = P->nocc;
    info->nvir = P->nvir;
    info->ng = P->ng;
    for (int d = 0; d < 3; ++d) {
        info->grid[d] = P->N[d];
        info->kmesh[d] = P->M[d];
    }
    info->precision = P->params.precision;
    info->nyquist = P->params.nyquist;
    info->kernel = P->params.kernel;
    info->kbatch = P->kbatch;
    info->omega = P->params.omega;
    info->cell_volume = P->volume;
    info->bytes_chi = P->bytes_chi;
    info->integral_direct = P->direct ? 1 : 0;
    info->colloc_chunk = P->cchunk;
    info->reg_fft_passes = make_batch(P, 0, 0, 1).regfft & (P->nout <= 8 ? ~0 : ~REGFFT_PASS3);
    info->bytes_workspace = P->bytes_alloc - P->bytes_chi;
    info->pair_transforms = plan_reuses_pairs(P)
                                ? (int64_t)P->nk * (P->nk - 1) / 2 * P->nocc * P->nocc +
                                      (int64_t)P->nk * P->nocc * (P->nocc + 1) / 2
                                : (int64_t)P->nk * P->nk * P->nocc * P->nout;
    info->plan_seconds = P->plan_seconds;
    info->contract_chunks = P->nchunks;
    info->tuned = P->tuned ? 1 : 0;
    return OCCRIK_OK;
}

occrik_status occrik_set_stream(occrik_plan* P, void* stream) {
    if (!P) return fail(OCCRIK_ERR_INVALID_ARG, "null plan");
    P->stream = reinterpret_cast<hipStream_t>(stream);
    return OCCRIK_OK;
}

occrik_status occrik_set_omega(occrik_plan* P, double omega) {
    if (!P) return fail(OCCRIK_ERR_INVALID_ARG, "null plan");
    if (!(omega > 0.0) || !std::isfinite(omega)) return fail(OCCRIK_ERR_INVALID_ARG, "omega must be positive");
    P->params.omega = omega;
    return OCCRIK_OK;
}

occrik_status occrik_build_device(occrik_plan* P, const void* dC, void* dK, void* dKmi, double* dEx) {
    if (!P || !dC) return fail(OCCRIK_ERR_INVALID_ARG, "null plan or C");
    DeviceGuard guard(P->device);
    P->last_err_k = -1;
    return P->fp64 ? build_impl<double>(P, (const double2*)dC, (double2*)dK, (double2*)dKmi, dEx)
                   : build_impl<float>(P, (const double2*)dC, (double2*)dK, (double2*)dKmi, dEx);
}

occrik_status occrik_plan_autotune(occrik_plan* P, const void* dC, occrik_tune_info* out) {
    if (!P || !dC) return fail(OCCRIK_ERR_INVALID_ARG, "null plan or C");
    DeviceGuard guard(P->device);
    hipStream_t s = P->stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(OCCRIK_ERR_DEVICE, "autotune events");
    }
    // settings before tuning, restored if a tuning build fails
    const int kbatch0 = P->kbatch, nchunks0 = P->nchunks, flags0 = P->params.flags;
    const int saved_profiling = P->profiling;
    P->profiling = 0;
    int builds = 0;
    auto timed = [&](double& ms) -> occrik_status {
        occrik_status st = OCCRIK_OK;
        if (hipEventRecord(e0, s) != hipSuccess) return fail(OCCRIK_ERR_DEVICE, "autotune event");
        st = P->fp64 ? build_impl<double>(P, (const double2*)dC, nullptr, nullptr, nullptr)
                     : build_impl<float>(P, (const double2*)dC, nullptr, nullptr, nullptr);
        if (st != OCCRIK_OK) return st;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
            return fail(OCCRIK_ERR_DEVICE, "autotune event");
        float f = 0.f;
        if (hipEventElapsedTime(&f, e0, e1) != hipSuccess) return fail(OCCRIK_ERR_DEVICE, "autotune timing");
        ms = f;
        ++builds;
        return OCCRIK_OK;
    };
    auto set_reg = [&](bool on) {
        P->params.flags &= ~OCCRIK_FLAG_REG_FFT_ALL;
        if (on) P->params.flags |= OCCRIK_FLAG_REG_FFT_ALL;
    };
    // contraction chunks above the allocated count need a larger partial-sum buffer;
    // a candidate that does not fit (device memory or mem_budget) is skipped
    auto ensure_chunks = [&](int nc) -> bool {
        if (nc <= P->kpart_chunks) return true;
        if (hipStreamSynchronize(s) != hipSuccess) return false;
        double2* bigger = nullptr;
        if (P->alloc((void**)&bigger, sizeof(double2) * (size_t)P->nk * P->nao * P->nout * nc) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        P->release(P->Kpart);
        P->Kpart = bigger;
        P->kpart_chunks = nc;
        return true;
    };
    occrik_status st = OCCRIK_OK;
    double ms = 0.0, best = 0.0, initial = 0.0;
    const bool reg_open = P->regfft && !(P->params.flags & (OCCRIK_FLAG_LDS_FFT | OCCRIK_FLAG_REG_FFT_ALL));
    const bool reg_initial = (P->params.flags & OCCRIK_FLAG_REG_FFT_ALL) != 0;
    do {
        if ((st = timed(ms)) != OCCRIK_OK) break;   // untimed warm-up
        if ((st = timed(initial)) != OCCRIK_OK) break;
        best = initial;
        // k batch: the allocated one, a half, a quarter
        if (P->params.kbatch == 0) {
            const int k0 = P->kbatch_max;
            int chosen = P->kbatch;
            for (int div : {2, 4}) {
                const int kb = (k0 + div - 1) / div;
                if (kb < 1 || kb == chosen || kb == k0) continue;
                P->kbatch = kb;
                if ((st = timed(ms)) != OCCRIK_OK) break;
                if (ms < best) {
                    best = ms;
                    chosen = kb;
                }
            }
            if (st != OCCRIK_OK) break;
            P->kbatch = chosen;
        }
        // pair transforms: LDS two-stage or register-resident
        if (reg_open) {
            set_reg(!reg_initial);
            if ((st = timed(ms)) != OCCRIK_OK) break;
            if (ms < best) best = ms;
            else set_reg(reg_initial);
        }
        // contraction chunks
        if (!P->direct && P->params.contract_chunks == 0) {
            const int n0 = P->nchunks;
            int chosen = n0;
            for (int nc : {contract_chunk_count(P->ng, std::min(kMaxContractChunks, 2 * n0)),
                           contract_chunk_count(P->ng, std::max(1, n0 / 2))}) {
                if (nc == n0 || nc == chosen || !ensure_chunks(nc)) continue;
                P->nchunks = nc;
                if ((st = timed(ms)) != OCCRIK_OK) break;
                if (ms < best) {
                    best = ms;
                    chosen = nc;
                }
            }
            if (st != OCCRIK_OK) break;
            P->nchunks = chosen;
        }
    } while (false);
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    P->profiling = saved_profiling;
    P->built = false;
    if (st != OCCRIK_OK) {
        P->kbatch = kbatch0;
        P->nchunks = nchunks0;
        P->params.flags = flags0;
        return st;
    }
    P->tuned = true;
    if (out) {
        out->kbatch = P->kbatch;
        out->reg_fft = (P->params.flags & OCCRIK_FLAG_REG_FFT_ALL) ? 1 : 0;
        out->contract_chunks = P->nchunks;
        out->builds = builds;
        out->ms_initial = initial;
        out->ms_best = best;
    }
    return OCCRIK_OK;
}

occrik_status occrik_conventional_k(occrik_plan* P, int32_t algo, const void* dC, void* dK, double* dEx) {
    if (!P || !dC || !dK) return fail(OCCRIK_ERR_INVALID_ARG, "null plan, C or K");
    if (algo != OCCRIK_ALGO_AO_RI_K && algo != OCCRIK_ALGO_MO_RI_K)
        return fail(OCCRIK_ERR_INVALID_ARG, "algo must be OCCRIK_ALGO_AO_RI_K or OCCRIK_ALGO_MO_RI_K");
    if (P->direct) return fail(OCCRIK_ERR_UNSUPPORTED, "the conventional algorithms need the stored Bloch AOs");
    DeviceGuard guard(P->device);
    return P->fp64 ? conventional_impl<double>(P, algo, (const double2*)dC, (double2*)dK, dEx)
                   : conventional_impl<float>(P, algo, (const double2*)dC, (double2*)dK, dEx);
}

occrik_status occrik_plan_status(occrik_plan* P) {
    if (!P) return fail(OCCRIK_ERR_INVALID_ARG, "null plan");
    if (!P->built) return OCCRIK_OK;
    DeviceGuard guard(P->device);
    int h[2];
    OCCRIK_HIP(hipMemcpyAsync(h, P->flags, sizeof(h), hipMemcpyDeviceToHost, P->stream));
    OCCRIK_HIP(hipStreamSynchronize(P->stream));
    if (h[0]) return fail(OCCRIK_ERR_NONFINITE, "non-finite entries in C");
    if (h[1] != INT_MAX) {
        P->last_err_k = h[1];
        return fail(OCCRIK_ERR_NOT_PD, "-K_ij is not positive definite at k = " + std::to_string(h[1]));
    }
    return OCCRIK_OK;
}

int32_t occrik_last_error_k(const occrik_plan* P) { return P ? P->last_err_k : -1; }

occrik_status occrik_build(occrik_plan* P, const double* C, double* K, double* Kmi, double* Ex) {
    if (!P || !C) return fail(OCCRIK_ERR_INVALID_ARG, "null plan or C");
    DeviceGuard guard(P->device);
    const size_t nC = (size_t)P->nk * P->nao * P->nout * 2;
    for (size_t i = 0; i < nC; ++i)
        if (!std::isfinite(C[i])) return fail(OCCRIK_ERR_NONFINITE, "non-finite entries in C");
    const size_t bC = nC * sizeof(double);
    const size_t bK = (size_t)P->nk * P->nao * P->nao * 2 * sizeof(double);
    void *dC = nullptr, *dK = nullptr, *dKmi = nullptr, *dEx = nullptr;
    occrik_status st = OCCRIK_OK;
    hipError_t e = hipMalloc(&dC, bC);
    if (e == hipSuccess && K) e = hipMalloc(&dK, bK);
    if (e == hipSuccess && Kmi) e = hipMalloc(&dKmi, bC);
    if (e == hipSuccess && Ex) e = hipMalloc(&dEx, sizeof(double));
    if (e == hipSuccess) e = hipMemcpyAsync(dC, C, bC, hipMemcpyHostToDevice, P->stream);
    if (e != hipSuccess) st = hip_fail(e, "occrik_build staging");
    if (st == OCCRIK_OK) st = occrik_build_device(P, dC, dK, dKmi, (double*)dEx);
    if (st == OCCRIK_OK) st = occrik_plan_status(P);
    if (st == OCCRIK_OK) {
        if (K) e = hipMemcpyAsync(K, dK, bK, hipMemcpyDeviceToHost, P->stream);
        if (e == hipSuccess && Kmi) e = hipMemcpyAsync(Kmi, dKmi, bC, hipMemcpyDeviceToHost, P->stream);
        if (e == hipSuccess && Ex) e = hipMemcpyAsync(Ex, dEx, sizeof(double), hipMemcpyDeviceToHost, P->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
        if (e != hipSuccess) st = hip_fail(e, "occrik_build readback");
    }
    (void)hipStreamSynchronize(P->stream);
    if (dC) (void)hipFree(dC);
    if (dK) (void)hipFree(dK);
    if (dKmi) (void)hipFree(dKmi);
    if (dEx) (void)hipFree(dEx);
    return st;
}

occrik_status occrik_build_static(occrik_plan* P, const double* C, double* K, double* Kmi, double* Ex) {
    if (!P || !C) return fail(OCCRIK_ERR_INVALID_ARG, "null plan or C");
    if (P->profiling) return fail(OCCRIK_ERR_STATE, "occrik_build_static needs profiling off (it creates events)");
    if (P->device < 0 || P->device >= kMaxStaticDevices)
        return fail(OCCRIK_ERR_UNSUPPORTED, "occrik_build_static: device ordinal beyond the staging table");
    DeviceGuard guard(P->device);
    const size_t nC = (size_t)P->nk * P->nao * P->nout * 2;
    for (size_t i = 0; i < nC; ++i)
        if (!std::isfinite(C[i])) return fail(OCCRIK_ERR_NONFINITE, "non-finite entries in C");
    // staging layout: C | K_{mu j} | E_x | K~ of as many k-points as fit
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t bC = nC * sizeof(double);
    const size_t offKmi = up(bC), offEx = up(offKmi + bC), offK = up(offEx + sizeof(double));
    const size_t perK = (size_t)P->nao * P->nao * sizeof(double2);
    if (offK > kStaticScratchBytes || (K && offK + perK > kStaticScratchBytes))
        return fail(OCCRIK_ERR_INVALID_ARG,
                    "occrik_build_static: C, K_{mu j} and one k-point of K~ need " +
                        std::to_string(offK + (K ? perK : 0)) + " bytes of staging, more than the " +
                        std::to_string(kStaticScratchBytes) + " it holds (use occrik_build)");
    char* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_static_mu);
        if (!g_static_ptr[P->device]) {
            void* p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return hip_fail(e, "occrik_build_static: hipGetSymbolAddress");
            if (!p) return fail(OCCRIK_ERR_DEVICE, "occrik_build_static: no device address for the staging area");
            g_static_ptr[P->device] = p;
        }
        base = static_cast<char*>(g_static_ptr[P->device]);
    }
    hipStream_t s = P->stream;
    double2* sC = reinterpret_cast<double2*>(base);
    double2* sKmi = reinterpret_cast<double2*>(base + offKmi);
    double* sEx = reinterpret_cast<double*>(base + offEx);
    double2* sK = reinterpret_cast<double2*>(base + offK);
    OCCRIK_HIP(hipMemcpyAsync(sC, C, bC, hipMemcpyHostToDevice, s));
    occrik_status st = occrik_build_device(P, sC, nullptr, Kmi ? sKmi : nullptr, Ex ? sEx : nullptr);
    if (st == OCCRIK_OK) st = occrik_plan_status(P);
    if (st != OCCRIK_OK) return st;
    if (Kmi) OCCRIK_HIP(hipMemcpyAsync(Kmi, sKmi, bC, hipMemcpyDeviceToHost, s));
    if (Ex) OCCRIK_HIP(hipMemcpyAsync(Ex, sEx, sizeof(double), hipMemcpyDeviceToHost, s));
    if (K) {
        // K~ = -xi xi^H in groups of k-points that fit the staging area, each copied out
        // before the next group overwrites it (same stream)
        const int nkc = (int)std::min<size_t>((size_t)P->nk, (kStaticScratchBytes - offK) / perK);
        OCCRIK_HIP(launch_xi(P->Kmi, P->L, P->Y, P->flags, P->nk, P->nao, P->nout, s));
        for (int k0 = 0; k0 < P->nk; k0 += nkc) {
            const int n = std::min(nkc, P->nk - k0);
            OCCRIK_HIP(launch_ktilde(P->Y + (size_t)k0 * P->nao * P->nout, sK, P->flags, n, P->nao, P->nout, s));
            OCCRIK_HIP(hipMemcpyAsync(K + (size_t)k0 * P->nao * P->nao * 2, sK, (size_t)n * perK,
                                      hipMemcpyDeviceToHost, s));
        }
    }
    OCCRIK_HIP(hipStreamSynchronize(s));
    return OCCRIK_OK;
}

occrik_status occrik_grad(occrik_plan* P, double gEx, void* dgradC, double* dgradOmega) {
    if (!P) return fail(OCCRIK_ERR_INVALID_ARG, "null plan");
    if (!P->built) return fail(OCCRIK_ERR_STATE, "occrik_grad needs a build on this plan first");
    if (!std::isfinite(gEx)) return fail(OCCRIK_ERR_INVALID_ARG, "non-finite gEx");
    DeviceGuard guard(P->device);
    if (dgradC)
        // dE_x/dC = (2 / N_k) K_{mu j} on the occupied columns; E_x does not depend on the
        // conduction-band columns, whose gradient is zero
        OCCRIK_HIP(launch_grad_columns(P->Kmi, (double2*)dgradC, (size_t)P->nk * P->nao, P->nout, P->nocc,
                                       gEx * 2.0 / P->nk, P->stream));
    if (dgradOmega) {
        double d = 0.0;
        if (P->params.kernel != OCCRIK_KERNEL_COULOMB) {
            occrik_status st = P->fp64 ? domega_impl<double>(P, &d) : domega_impl<float>(P, &d);
            if (st != OCCRIK_OK) return st;
        }
        *dgradOmega = gEx * d;
    }
    return OCCRIK_OK;
}

// ---------------------------------------------------------------------------
// ragged batches: the builds of a batch spread over worker streams of the
// device (fork and join on the plans' stream), either enqueued directly or
// recorded once as a HIP graph and replayed with one launch
// ---------------------------------------------------------------------------
extern "C++" {
namespace {

constexpr int kBatchStreams = 4;

struct BatchStreams {
    hipStream_t s[kBatchStreams] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kBatchStreams] = {};
};

std::mutex g_batch_mu;
std::vector<BatchStreams*> g_batch_streams;   // per device ordinal; kept until the process ends

// the calling thread's current device must be `device`
hipError_t batch_streams(int device, BatchStreams** out) {
    std::lock_guard<std::mutex> lock(g_batch_mu);
    if ((int)g_batch_streams.size() <= device) g_batch_streams.resize(device + 1, nullptr);
    if (!g_batch_streams[device]) {
        auto* b = new BatchStreams();
        hipError_t e = hipSuccess;
        for (int w = 0; w < kBatchStreams && e == hipSuccess; ++w) {
            e = hipStreamCreateWithFlags(&b->s[w], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[w], hipEventDisableTiming);
        }
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
        if (e != hipSuccess) {
            delete b;
            return e;
        }
        g_batch_streams[device] = b;
    }
    *out = g_batch_streams[device];
    return hipSuccess;
}

// relative cost of one build: pair round trips (each ~ N_g log N_g) plus the two GEMMs
double build_cost(const occrik_plan* P) {
    const double pairs = plan_reuses_pairs(P)
                             ? double(P->nk) * (P->nk - 1) / 2 * P->nocc * P->nocc +
                                   double(P->nk) * P->nocc * (P->nocc + 1) / 2
                             : double(P->nk) * P->nk * P->nocc * P->nout;
    return pairs * P->ng * std::log2(double(P->ng)) + 2.0 * P->nk * P->nao * P->nout * double(P->ng);
}

occrik_status validate_batch(int32_t n, occrik_plan* const* plans, const void* const* dC) {
    if (n < 0 || (n > 0 && (!plans || !dC))) return fail(OCCRIK_ERR_INVALID_ARG, "bad batch arguments");
    for (int i = 0; i < n; ++i) {
        if (!plans[i] || !dC[i]) return fail(OCCRIK_ERR_INVALID_ARG, "null plan or C in batch");
        if (plans[i]->device != plans[0]->device || plans[i]->stream != plans[0]->stream)
            return fail(OCCRIK_ERR_INVALID_ARG, "batch plans must share device and stream");
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i]) return fail(OCCRIK_ERR_INVALID_ARG, "a plan appears twice in the batch");
    }
    return OCCRIK_OK;
}

// Enqueue every build of the batch: worker streams wait for the plans' stream, the
// builds go to the least-loaded worker (largest first), the plans' stream waits
// for every worker.  The caller has made the plans' device current.
occrik_status enqueue_batch(int32_t n, occrik_plan* const* plans, const void* const* dC, void* const* dK,
                            void* const* dKmi, double* const* dEx) {
    hipStream_t s0 = plans[0]->stream;
    BatchStreams* bs = nullptr;
    OCCRIK_HIP(batch_streams(plans[0]->device, &bs));
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::vector<double> cost(n);
    for (int i = 0; i < n; ++i) cost[i] = build_cost(plans[i]);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    double load[kBatchStreams] = {};
    OCCRIK_HIP(hipEventRecord(bs->fork, s0));
    for (int w = 0; w < kBatchStreams; ++w) OCCRIK_HIP(hipStreamWaitEvent(bs->s[w], bs->fork, 0));
    occrik_status st = OCCRIK_OK;
    for (int i : order) {
        const int w = int(std::min_element(load, load + kBatchStreams) - load);
        load[w] += cost[i];
        occrik_plan* P = plans[i];
        P->stream = bs->s[w];
        P->last_err_k = -1;
        st = P->fp64 ? build_impl<double>(P, (const double2*)dC[i], dK ? (double2*)dK[i] : nullptr,
                                          dKmi ? (double2*)dKmi[i] : nullptr, dEx ? dEx[i] : nullptr)
                     : build_impl<float>(P, (const double2*)dC[i], dK ? (double2*)dK[i] : nullptr,
                                         dKmi ? (double2*)dKmi[i] : nullptr, dEx ? dEx[i] : nullptr);
        P->stream = s0;
        if (st != OCCRIK_OK) break;
    }
    // join even after a failed enqueue, so that the plans' stream never runs ahead of the workers
    for (int w = 0; w < kBatchStreams; ++w) {
        OCCRIK_HIP(hipEventRecord(bs->join[w], bs->s[w]));
        OCCRIK_HIP(hipStreamWaitEvent(s0, bs->join[w], 0));
    }
    return st;
}

// Fused rounds of a recorded batch.  Plans that share the working precision, a compiled
// cubic grid and the pass-3 form (up to 8 or 9-16 output orbitals) form a group; round r
// of a group runs the r-th pair-pass launch of each of its plans as one launch per stage
// (pass 1, pass 2, pass 3, the W reduction).  Each plan's launches keep their order, so
// every result is the plan's own single build, bit for bit.
struct FusedGroup {
    bool fp64 = false;
    PairBatch B0{};                          // the first batch of the group (kernel forms)
    std::vector<int> plans;                  // indices into the batch
    std::vector<int> round_off, round_n;     // items of each round in the device table
    std::vector<std::array<unsigned, kFusedStages>> round_total;
};

struct FusedSchedule {
    std::vector<FusedGroup> groups;
    std::vector<FusedItem> items;            // every round of every group, in launch order
    std::vector<char> fused;                 // per plan: 1 if its pair passes run in a group
};

FusedSchedule plan_fused(int32_t n, occrik_plan* const* plans) {
    FusedSchedule f;
    f.fused.assign(n, 0);
    std::vector<std::vector<PairBatch>> launches(n);
    std::map<std::array<int, 3>, std::vector<int>> by_key;
    for (int i = 0; i < n; ++i) {
        launches[i] = plan_launches(plans[i]);
        bool ok = !launches[i].empty();
        for (const PairBatch& B : launches[i]) ok = ok && fusable(B);
        if (ok) by_key[{plans[i]->fp64 ? 1 : 0, launches[i][0].N1, launches[i][0].nout <= 8 ? 8 : 16}].push_back(i);
    }
    for (auto& kv : by_key) {
        if (kv.second.size() < 2) continue;                // a single plan gains nothing
        FusedGroup g;
        g.fp64 = kv.first[0] != 0;
        g.plans = kv.second;
        g.B0 = launches[g.plans[0]][0];
        size_t rounds = 0;
        for (int i : g.plans) rounds = std::max(rounds, launches[i].size());
        for (size_t r = 0; r < rounds; ++r) {
            std::array<size_t, kFusedStages> tot{};
            const int off = (int)f.items.size();
            for (int i : g.plans) {
                if (r >= launches[i].size()) continue;
                const occrik_plan* P = plans[i];
                FusedItem it{};
                it.B = launches[i][r];
                it.psi = P->psi;
                it.X = P->X;
                it.Wpart = P->Wpart;
                it.W = P->W;
                it.tw = P->tw;
                it.parts = P->parts;
                int wg[kFusedStages];
                fused_workgroups(it.B, (int)P->elem, wg);
                for (int st = 0; st < kFusedStages; ++st) {
                    it.wg0[st] = (int)tot[st];
                    tot[st] += (size_t)wg[st];
                }
                f.items.push_back(it);
            }
            std::array<unsigned, kFusedStages> t{};
            for (int st = 0; st < kFusedStages; ++st) t[st] = tot[st] <= (size_t)INT_MAX ? (unsigned)tot[st] : 0u;
            g.round_off.push_back(off);
            g.round_n.push_back((int)f.items.size() - off);
            g.round_total.push_back(t);
        }
        for (int i : g.plans) f.fused[i] = 1;
        f.groups.push_back(std::move(g));
    }
    return f;
}

template <typename T>
occrik_status build_stages(occrik_plan* P, const void* dC, void* dK, void* dKmi, double* dEx, int stages) {
    return build_impl<T>(P, (const double2*)dC, (double2*)dK, (double2*)dKmi, dEx, stages);
}

occrik_status build_plan_stages(occrik_plan* P, const void* dC, void* dK, void* dKmi, double* dEx, int stages) {
    return P->fp64 ? build_stages<double>(P, dC, dK, dKmi, dEx, stages)
                   : build_stages<float>(P, dC, dK, dKmi, dEx, stages);
}

// The fused form of enqueue_batch (inside the recording of a batch graph): the
// prologues (orbitals, W zero, kernel values) of the grouped plans spread over the
// worker streams; then each group's rounds on one worker, the groups assigned largest
// first to the least-loaded worker, beside the other plans' whole builds; then the
// grouped plans' epilogues (contraction, assembly, E_x) spread over the workers.  The
// plans' stream joins the workers between the phases.  ev holds 4 + 3 kBatchStreams
// events.
occrik_status enqueue_fused(int32_t n, occrik_plan* const* plans, const void* const* dC, void* const* dK,
                            void* const* dKmi, double* const* dEx, const FusedSchedule& f, const FusedItem* d_items,
                            const hipEvent_t* ev) {
    hipStream_t s0 = plans[0]->stream;
    BatchStreams* bs = nullptr;
    OCCRIK_HIP(batch_streams(plans[0]->device, &bs));
    const hipEvent_t* fork = ev;                          // [3] s0 -> workers before each phase
    const hipEvent_t* join = ev + 4;                      // [3][kBatchStreams] workers -> s0 after each phase
    auto arg = [](auto* const* a, int i) { return a ? a[i] : nullptr; };
    occrik_status st = OCCRIK_OK;
    auto phase_begin = [&](int k) -> occrik_status {
        OCCRIK_HIP(hipEventRecord(fork[k], s0));
        for (int w = 0; w < kBatchStreams; ++w) OCCRIK_HIP(hipStreamWaitEvent(bs->s[w], fork[k], 0));
        return OCCRIK_OK;
    };
    auto phase_end = [&](int k) -> occrik_status {
        for (int w = 0; w < kBatchStreams; ++w) {
            OCCRIK_HIP(hipEventRecord(join[k * kBatchStreams + w], bs->s[w]));
            OCCRIK_HIP(hipStreamWaitEvent(s0, join[k * kBatchStreams + w], 0));
        }
        return OCCRIK_OK;
    };
    auto on_worker = [&](int i, int w, int stages) {
        occrik_plan* P = plans[i];
        P->stream = bs->s[w];
        P->last_err_k = -1;
        const occrik_status r = build_plan_stages(P, dC[i], arg(dK, i), arg(dKmi, i), arg(dEx, i), stages);
        P->stream = s0;
        return r;
    };
    // phase 1: prologues of the grouped plans
    if ((st = phase_begin(0)) != OCCRIK_OK) return st;
    int w = 0;
    for (int i = 0; i < n && st == OCCRIK_OK; ++i)
        if (f.fused[i]) {
            st = on_worker(i, w, kStagePrologue);
            w = (w + 1) % kBatchStreams;
        }
    occrik_status e = phase_end(0);
    if (st == OCCRIK_OK) st = e;
    // phase 2: each group's rounds on one worker, the other plans whole, largest first
    // to the least-loaded worker
    if (st == OCCRIK_OK) st = phase_begin(1);
    struct Job {
        double cost;
        int group, plan;
    };
    std::vector<Job> jobs;
    for (size_t g = 0; g < f.groups.size(); ++g) {
        double c = 0.0;
        for (int i : f.groups[g].plans) c += build_cost(plans[i]);
        jobs.push_back({c, (int)g, -1});
    }
    for (int i = 0; i < n; ++i)
        if (!f.fused[i]) jobs.push_back({build_cost(plans[i]), -1, i});
    std::stable_sort(jobs.begin(), jobs.end(), [](const Job& a, const Job& b) { return a.cost > b.cost; });
    double load[kBatchStreams] = {};
    for (const Job& j : jobs) {
        if (st != OCCRIK_OK) break;
        const int v = int(std::min_element(load, load + kBatchStreams) - load);
        load[v] += j.cost;
        if (j.plan >= 0) {
            st = on_worker(j.plan, v, kStageAll);
            continue;
        }
        const FusedGroup& g = f.groups[j.group];
        for (size_t r = 0; r < g.round_off.size() && st == OCCRIK_OK; ++r) {
            for (int stage = 0; stage < kFusedStages && st == OCCRIK_OK; ++stage) {
                const unsigned total = g.round_total[r][stage];
                const FusedItem* items = d_items + g.round_off[r];
                const hipError_t he = g.fp64
                                          ? launch_fused<double>(stage, g.B0, items, g.round_n[r], total, bs->s[v])
                                          : launch_fused<float>(stage, g.B0, items, g.round_n[r], total, bs->s[v]);
                if (he != hipSuccess) st = hip_fail(he, "launch_fused");
            }
        }
    }
    // join even after a failed enqueue, so that the plans' stream never runs ahead of the workers
    e = phase_end(1);
    if (st == OCCRIK_OK) st = e;
    // phase 3: epilogues of the grouped plans
    if (st == OCCRIK_OK) st = phase_begin(2);
    w = 0;
    for (int i = 0; i < n && st == OCCRIK_OK; ++i)
        if (f.fused[i]) {
            st = on_worker(i, w, kStageEpilogue);
            w = (w + 1) % kBatchStreams;
        }
    e = phase_end(2);
    return st != OCCRIK_OK ? st : e;
}

}  // namespace
}  // extern "C++"

struct occrik_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    FusedItem* d_items = nullptr;            // the fused rounds' item table (read by the graph)
    std::vector<hipEvent_t> events;          // fork and join events of the fused schedule
    int fused_plans = 0;
    ~occrik_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (d_items) (void)hipFree(d_items);
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
    }
};

occrik_status occrik_build_batch(int32_t n, occrik_plan* const* plans, const void* const* dC, void* const* dK,
                                 void* const* dKmi, double* const* dEx) {
    occrik_status st = validate_batch(n, plans, dC);
    if (st != OCCRIK_OK || n == 0) return st;
    DeviceGuard guard(plans[0]->device);
    return enqueue_batch(n, plans, dC, dK, dKmi, dEx);
}

}  // extern "C"

namespace {

occrik_status batch_create(int32_t n, occrik_plan* const* plans, const void* const* dC, void* const* dK,
                           void* const* dKmi, double* const* dEx, bool fuse, occrik_batch** out) {
    if (!out) return fail(OCCRIK_ERR_INVALID_ARG, "null out");
    *out = nullptr;
    occrik_status st = validate_batch(n, plans, dC);
    if (st != OCCRIK_OK) return st;
    if (n == 0) return fail(OCCRIK_ERR_INVALID_ARG, "empty batch");
    if (!plans[0]->stream) return fail(OCCRIK_ERR_INVALID_ARG, "recording a batch needs a non-default stream");
    for (int i = 0; i < n; ++i)
        if (plans[i]->profiling) return fail(OCCRIK_ERR_INVALID_ARG, "profiling must be off to record a batch");
    DeviceGuard guard(plans[0]->device);
    BatchStreams* bs = nullptr;
    OCCRIK_HIP(batch_streams(plans[0]->device, &bs));    // created before the capture starts
    auto* b = new occrik_batch();
    b->device = plans[0]->device;
    b->stream = plans[0]->stream;
    // fused rounds for the plans that share a kernel form: the item table is uploaded and
    // the events created before the recording starts
    const FusedSchedule f = fuse ? plan_fused(n, plans) : FusedSchedule{};
    hipError_t e = hipSuccess;
    if (!f.groups.empty()) {
        const size_t bytes = sizeof(FusedItem) * f.items.size();
        e = hipMalloc((void**)&b->d_items, bytes);
        if (e == hipSuccess) e = hipMemcpy(b->d_items, f.items.data(), bytes, hipMemcpyHostToDevice);
        for (int k = 0; k < 4 + 3 * kBatchStreams && e == hipSuccess; ++k) {
            hipEvent_t ev = nullptr;
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess) b->events.push_back(ev);
        }
        for (const FusedGroup& g : f.groups) b->fused_plans += (int)g.plans.size();
        if (e != hipSuccess) {
            delete b;
            return hip_fail(e, "fused batch set-up");
        }
    }
    e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "hipStreamBeginCapture");
    }
    st = f.groups.empty() ? enqueue_batch(n, plans, dC, dK, dKmi, dEx)
                          : enqueue_fused(n, plans, dC, dK, dKmi, dEx, f, b->d_items, b->events.data());
    e = hipStreamEndCapture(b->stream, &b->graph);
    if (st != OCCRIK_OK || e != hipSuccess) {
        delete b;
        return st != OCCRIK_OK ? st : hip_fail(e, "hipStreamEndCapture");
    }
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "hipGraphInstantiate");
    }
    *out = b;
    return OCCRIK_OK;
}

}  // namespace

extern "C" {

occrik_status occrik_batch_create(int32_t n, occrik_plan* const* plans, const void* const* dC, void* const* dK,
                                  void* const* dKmi, double* const* dEx, occrik_batch** out) {
    return batch_create(n, plans, dC, dK, dKmi, dEx, false, out);
}

occrik_status occrik_batch_create_fused(int32_t n, occrik_plan* const* plans, const void* const* dC,
                                        void* const* dK, void* const* dKmi, double* const* dEx, occrik_batch** out) {
    return batch_create(n, plans, dC, dK, dKmi, dEx, true, out);
}

occrik_status occrik_batch_launch(occrik_batch* b) {
    if (!b) return fail(OCCRIK_ERR_INVALID_ARG, "null batch");
    DeviceGuard guard(b->device);
    OCCRIK_HIP(hipGraphLaunch(b->exec, b->stream));
    return OCCRIK_OK;
}

occrik_status occrik_batch_fused(const occrik_batch* b, int32_t* nplans) {
    if (!b || !nplans) return fail(OCCRIK_ERR_INVALID_ARG, "null batch or out");
    *nplans = b->fused_plans;
    return OCCRIK_OK;
}

void occrik_batch_destroy(occrik_batch* b) {
    if (!b) return;
    DeviceGuard guard(b->device);
    (void)hipStreamSynchronize(b->stream);
    delete b;
}

occrik_status occrik_set_profiling(occrik_plan* P, int32_t on) {
    if (!P) return fail(OCCRIK_ERR_INVALID_ARG, "null plan");
    if (on < 0 || on > 2) return fail(OCCRIK_ERR_INVALID_ARG, "profiling level must be 0, 1 or 2");
    P->profiling = on;
    return OCCRIK_OK;
}

occrik_status occrik_get_profile(occrik_plan* P, occrik_profile* out, int32_t reset) {
    if (!P || !out) return fail(OCCRIK_ERR_INVALID_ARG, "null plan or out");
    DeviceGuard guard(P->device);
    for (auto& pe : P->prof) {
        OCCRIK_HIP(hipEventSynchronize(pe.e[4]));
        float t[4];
        for (int i = 0; i < 4; ++i) OCCRIK_HIP(hipEventElapsedTime(&t[i], pe.e[i], pe.e[i + 1]));
        P->prof_acc.ms_orbitals += t[0];
        P->prof_acc.ms_pairs += t[1];
        P->prof_acc.ms_contract += t[2];
        P->prof_acc.ms_assemble += t[3];
        P->prof_acc.launches_pairs += pe.pair_launches;
        P->prof_acc.builds += 1;
        for (size_t b = 0; b + 3 < pe.pe.size(); b += 4) {
            for (int q = 0; q < 3; ++q) {
                float ms = 0.f;
                OCCRIK_HIP(hipEventElapsedTime(&ms, pe.pe[b + q], pe.pe[b + q + 1]));
                P->prof_acc.ms_pass[q] += ms;
                P->prof_acc.launches_pass[q] += 1;
                P->prof_acc.bytes_pass[q] += pe.pbytes[3 * (b / 4) + q];
            }
        }
        for (auto& e : pe.e) (void)hipEventDestroy(e);
        for (auto& e : pe.pe) (void)hipEventDestroy(e);
    }
    P->prof.clear();
    *out = P->prof_acc;
    if (reset) P->prof_acc = occrik_profile{};
    return OCCRIK_OK;
}

occrik_status occrik_copy_intermediate(occrik_plan* P, int32_t which, void* dst, size_t bytes) {
    if (!P || !dst) return fail(OCCRIK_ERR_INVALID_ARG, "null plan or dst");
    DeviceGuard guard(P->device);
    const void* src = nullptr;
    size_t n = 0;
    if (which == 0) {
        if (P->direct) return fail(OCCRIK_ERR_STATE, "an integral-direct plan stores no chi");
        src = P->chi;
        n = (size_t)P->nk * P->nao * P->ng;
    } else if (which == 1 || which == 2) {
        if (!P->built) return fail(OCCRIK_ERR_STATE, "no build yet");
        src = which == 1 ? P->psi : P->W;
        n = (size_t)P->nk * P->nout * P->ng;
    } else {
        return fail(OCCRIK_ERR_INVALID_ARG, "which must be 0, 1 or 2");
    }
    if (bytes != n * sizeof(double2)) return fail(OCCRIK_ERR_INVALID_ARG, "bytes does not match the array size");
    if (P->fp64) OCCRIK_HIP(launch_convert_to_c128<double>((const cplx<double>*)src, (double2*)dst, n, P->stream));
    else OCCRIK_HIP(launch_convert_to_c128<float>((const cplx<float>*)src, (double2*)dst, n, P->stream));
    OCCRIK_HIP(hipStreamSynchronize(P->stream));
    return OCCRIK_OK;
}

}  // extern "C"
