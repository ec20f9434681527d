// FP64 tail of the build: the occupied block, its Cholesky factor, the
// assembled exchange matrix and the exchange energy (paper Sec. II.A energy
// expression, Sec. II.D eq. occrikop).
//
//   K_ij(k) = sum_mu conj(C_{mu i}(k)) K_{mu j}(k)
//   L L^H   = -(K_ij + K_ij^H)/2                 (Cholesky; failure -> NOT_PD)
//   y_mu    = L^{-1} conj(K_{mu .})              (y_mu is column mu of xi^H)
//   K~_{mu nu} = -sum_j conj(y_mu[j]) y_nu[j]    (K~ = -xi xi^H = K_mu K_ij^{-1} K_mu^H)
//   E_x     = sum_k Re tr K_ij(k) / (2 N_k)      (summed over k in a fixed order)
//
// Device status words: flags[0] = 1 when C holds NaN/Inf, flags[1] = smallest
// k whose Cholesky failed (INT_MAX when none), flags[2 + k] = 1 when k failed.
#include <climits>

#include "internal.hpp"

namespace occrik {

namespace {

constexpr int kMaxOccA = 16;

__global__ void check_finite_kernel(const double2* __restrict__ C, size_t n, int* flags) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (; i < n; i += stride) {
        const double2 v = C[i];
        if (!isfinite(v.x) || !isfinite(v.y)) bad = true;
    }
    if (bad) flags[0] = 1;
}

__global__ void reset_flags_kernel(int* flags, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 1) flags[1] = INT_MAX;
    else if (i < n) flags[i] = 0;
}

__global__ void __launch_bounds__(256) kij_kernel(const double2* __restrict__ C, const double2* __restrict__ Kmi,
                                                  double2* __restrict__ Kij, double2* __restrict__ L,
                                                  double* __restrict__ eterm, int* flags, int nk, int nao, int nocc,
                                                  int nocc_e) {
    __shared__ double2 kij[kMaxOccA * kMaxOccA];
    __shared__ double2 l[kMaxOccA * kMaxOccA];
    __shared__ double2 part[256];
    const int k = blockIdx.x;
    const int t = threadIdx.x;
    const double2* Ck = C + (size_t)k * nao * nocc;
    const double2* Kk = Kmi + (size_t)k * nao * nocc;
    // entry (i, j) = sum_mu conj(C_{mu i}) K_{mu j}: G threads per entry take every G-th
    // AO, and their G partial sums are added in a fixed order
    const int nn = nocc * nocc;
    const int G = nn > 0 ? 256 / nn : 1;
    if (t < nn * G) {
        const int e = t / G, g = t - e * G;
        const int i = e / nocc, j = e - i * nocc;
        double sx = 0.0, sy = 0.0;
        for (int mu = g; mu < nao; mu += G) {
            const double2 c = Ck[(size_t)mu * nocc + i];
            const double2 v = Kk[(size_t)mu * nocc + j];
            sx += c.x * v.x + c.y * v.y;
            sy += c.x * v.y - c.y * v.x;
        }
        part[t] = make_double2(sx, sy);
    }
    __syncthreads();
    if (t < nn) {
        double2 r = make_double2(0.0, 0.0);
        for (int g = 0; g < G; ++g) {
            r.x += part[t * G + g].x;
            r.y += part[t * G + g].y;
        }
        kij[t] = r;
        Kij[(size_t)k * nocc * nocc + t] = r;
    }
    __syncthreads();
    if (t == 0) {
        const int n = nocc;
        double tr = 0.0;
        for (int i = 0; i < nocc_e; ++i) tr += kij[i * n + i].x;      // occupied orbitals only
        eterm[k] = tr / (2.0 * nk);
        bool ok = true;
        for (int i = 0; i < n * n; ++i) l[i] = make_double2(0.0, 0.0);
        for (int c = 0; c < n && ok; ++c) {
            // A = -(K + K^H)/2
            double d = -kij[c * n + c].x;
            for (int q = 0; q < c; ++q) d -= l[c * n + q].x * l[c * n + q].x + l[c * n + q].y * l[c * n + q].y;
            if (!(d > 0.0) || !isfinite(d)) {
                ok = false;
                break;
            }
            const double lc = sqrt(d);
            l[c * n + c] = make_double2(lc, 0.0);
            for (int r = c + 1; r < n; ++r) {
                // A[r][c] = -(K[r][c] + conj(K[c][r]))/2
                double ax = -0.5 * (kij[r * n + c].x + kij[c * n + r].x);
                double ay = -0.5 * (kij[r * n + c].y - kij[c * n + r].y);
                for (int q = 0; q < c; ++q) {
                    const double2 a = l[r * n + q], b = l[c * n + q];   // a * conj(b)
                    ax -= a.x * b.x + a.y * b.y;
                    ay -= a.y * b.x - a.x * b.y;
                }
                l[r * n + c] = make_double2(ax / lc, ay / lc);
            }
        }
        if (!ok) {
            flags[2 + k] = 1;
            atomicMin(&flags[1], k);
        }
    }
    __syncthreads();
    if (t < nocc * nocc) L[(size_t)k * nocc * nocc + t] = l[t];
}

__global__ void xi_kernel(const double2* __restrict__ Kmi, const double2* __restrict__ L, double2* __restrict__ Y,
                          const int* __restrict__ flags, int nk, int nao, int nocc) {
    const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (size_t)nk * nao) return;
    const int k = (int)(g / nao);
    const double2* Lk = L + (size_t)k * nocc * nocc;
    const double2* b = Kmi + g * nocc;
    double2* y = Y + g * nocc;
    if (flags[2 + k]) {
        for (int r = 0; r < nocc; ++r) y[r] = make_double2(0.0, 0.0);
        return;
    }
    double2 yy[kMaxOccA];
    for (int r = 0; r < nocc; ++r) {
        double sx = b[r].x, sy = -b[r].y;                 // conj(K_{mu r})
        for (int c = 0; c < r; ++c) {
            const double2 a = Lk[r * nocc + c];
            sx -= a.x * yy[c].x - a.y * yy[c].y;
            sy -= a.x * yy[c].y + a.y * yy[c].x;
        }
        const double d = Lk[r * nocc + r].x;
        yy[r] = make_double2(sx / d, sy / d);
        y[r] = yy[r];
    }
}

__global__ void ktilde_kernel(const double2* __restrict__ Y, double2* __restrict__ K, const int* __restrict__ flags,
                              int nk, int nao, int nocc) {
    const int nu = blockIdx.x * 16 + threadIdx.x;
    const int mu = blockIdx.y * 16 + threadIdx.y;
    const int k = blockIdx.z;
    if (mu >= nao || nu >= nao) return;
    const double2* ym = Y + ((size_t)k * nao + mu) * nocc;
    const double2* yn = Y + ((size_t)k * nao + nu) * nocc;
    double sx = 0.0, sy = 0.0;
    for (int j = 0; j < nocc; ++j) {
        const double2 a = ym[j], b = yn[j];               // conj(a) * b
        sx += a.x * b.x + a.y * b.y;
        sy += a.x * b.y - a.y * b.x;
    }
    K[((size_t)k * nao + mu) * nao + nu] = make_double2(-sx, -sy);
}

__global__ void energy_kernel(const double* __restrict__ eterm, int nk, double* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int k = 0; k < nk; ++k) s += eterm[k];
    *out = s;
}

__global__ void sum_f64_kernel(const double* __restrict__ parts, size_t n, double scale, double* out) {
    __shared__ double red[256];
    double s = 0.0;
    for (size_t i = threadIdx.x; i < n; i += 256) s += parts[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out += scale * red[0];
}

__global__ void grad_columns_kernel(const double2* __restrict__ src, double2* __restrict__ dst, size_t rows,
                                    int ncol, int nkeep, double scale) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * ncol) return;
    const int c = (int)(t % ncol);
    const double2 v = src[t];
    dst[t] = c < nkeep ? make_double2(scale * v.x, scale * v.y) : make_double2(0.0, 0.0);
}

__global__ void scale_copy_kernel(const double2* __restrict__ src, double2* __restrict__ dst, size_t n, double scale) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = make_double2(scale * src[i].x, scale * src[i].y);
}

template <typename T>
__global__ void to_c128_kernel(const cplx<T>* __restrict__ src, double2* __restrict__ dst, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = make_double2(double(src[i].x), double(src[i].y));
}

}  // namespace

hipError_t launch_check_finite(const double2* C, size_t n, int* flags, hipStream_t s) {
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)blocks), dim3(256), 0, s, C, n, flags);
    return hipGetLastError();
}

hipError_t launch_reset_flags_n(int* flags, int n, hipStream_t s) {
    hipLaunchKernelGGL(reset_flags_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, flags, n);
    return hipGetLastError();
}

hipError_t launch_kij(const double2* C, const double2* Kmi, double2* Kij, double2* L, double* eterm, int* flags,
                      int nk, int nao, int ncol, int nocc, hipStream_t s) {
    hipLaunchKernelGGL(kij_kernel, dim3((unsigned)nk), dim3(256), 0, s, C, Kmi, Kij, L, eterm, flags, nk, nao, ncol,
                       nocc);
    return hipGetLastError();
}

hipError_t launch_xi(const double2* Kmi, const double2* L, double2* Y, const int* flags, int nk, int nao, int nocc,
                     hipStream_t s) {
    const size_t n = (size_t)nk * nao;
    hipLaunchKernelGGL(xi_kernel, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, Kmi, L, Y, flags, nk, nao, nocc);
    return hipGetLastError();
}

hipError_t launch_ktilde(const double2* Y, double2* K, const int* flags, int nk, int nao, int nocc, hipStream_t s) {
    dim3 grid((unsigned)((nao + 15) / 16), (unsigned)((nao + 15) / 16), (unsigned)nk);
    hipLaunchKernelGGL(ktilde_kernel, grid, dim3(16, 16), 0, s, Y, K, flags, nk, nao, nocc);
    return hipGetLastError();
}

hipError_t launch_energy(const double* eterm, int nk, double* out, hipStream_t s) {
    hipLaunchKernelGGL(energy_kernel, dim3(1), dim3(64), 0, s, eterm, nk, out);
    return hipGetLastError();
}

hipError_t launch_sum_f64(const double* parts, size_t n, double scale, double* out, hipStream_t s) {
    hipLaunchKernelGGL(sum_f64_kernel, dim3(1), dim3(256), 0, s, parts, n, scale, out);
    return hipGetLastError();
}

hipError_t launch_grad_columns(const double2* src, double2* dst, size_t rows, int ncol, int nkeep, double scale,
                               hipStream_t s) {
    const size_t n = rows * ncol;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(grad_columns_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, rows, ncol,
                       nkeep, scale);
    return hipGetLastError();
}

hipError_t launch_scale_copy(const double2* src, double2* dst, size_t n, double scale, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(scale_copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n, scale);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_convert_to_c128(const cplx<T>* src, double2* dst, size_t n, hipStream_t s) {
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(to_c128_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}
template hipError_t launch_convert_to_c128<float>(const cplx<float>*, double2*, size_t, hipStream_t);
template hipError_t launch_convert_to_c128<double>(const cplx<double>*, double2*, size_t, hipStream_t);

}  // namespace occrik
