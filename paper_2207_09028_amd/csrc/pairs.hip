// The occ-RI-K pair round trips (paper Alg. 3, inner loops; eqs. aodf, Vrao,
// VGao, occrikinterm) as three fused passes over a batch of pair densities.
//
// A 3D transform of N_1 x N_2 x N_3 points does not fit one CU's LDS, so each
// forward + inverse round trip exchanges the data through device memory twice:
//
//   pass 1  (one x-plane n1 of one pair per workgroup)
//           u = conj(psi~_{i b}) psi~_{j a} on the plane, FFT along n3 and n2,
//           store X[p][n1][m2][m3]
//   pass 2  (one m2-slab of one pair per workgroup, in place)
//           FFT along n1, multiply by f(|G+q|)/N_g (computed on the fly, with
//           the G+q=0 and Nyquist rules), inverse FFT along m1 and m3,
//           store X[p][n1][m2][n3]
//   pass 3  (one x-plane of one output orbital j, a slice of the (b, i) sum)
//           inverse FFT along m2, multiply by psi~_{i b}, accumulate over the
//           slice in registers: W~_j partial for this plane
//
// The potential Vt = IDFT(f DFT(u)) / N_g is the cell-periodic part of V;
// psi~_{i b} Vt is the cell-periodic part of psi_{i b} V, so W~ = e^{-ik_a.r} W.
#include "fft.hpp"
#include "internal.hpp"

namespace occrik {

namespace {

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

template <typename T>
__device__ inline T momentum_sq(const Recip<T>& rc, double q0, double q1, double q2, int m1, int m2, int m3) {
    const T a = T(m1 + q0), b = T(m2 + q1), c = T(m3 + q2);
    const T gx = a * rc.b[0] + b * rc.b[3] + c * rc.b[6];
    const T gy = a * rc.b[1] + b * rc.b[4] + c * rc.b[7];
    const T gz = a * rc.b[2] + b * rc.b[5] + c * rc.b[8];
    return gx * gx + gy * gy + gz * gz;
}

// ---------------------------------------------------------------------------
// pass 1
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kFftThreads) pass1_kernel(PairBatch B, const cplx<T>* __restrict__ psi,
                                                            cplx<T>* __restrict__ X, const cplx<T>* __restrict__ twg) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* plane = tw + 3 * kMaxN;
    const int N2 = B.N2, N3 = B.N3, S = N3 + 1;
    const int plane_sz = N2 * N3;
    const int n1 = blockIdx.x % B.N1;
    const int p = blockIdx.x / B.N1;
    const int j = p % B.nocc;
    const int i = (p / B.nocc) % B.nocc;
    const int b = B.b0 + p / (B.nocc * B.nocc);
    load_twiddles<T>(tw, twg);
    const cplx<T>* pj = psi + ((size_t)B.a * B.nocc + j) * B.ng + (size_t)n1 * plane_sz;
    const cplx<T>* pi = psi + ((size_t)b * B.nocc + i) * B.ng + (size_t)n1 * plane_sz;
    for (int e = threadIdx.x; e < plane_sz; e += kFftThreads) {
        const int n2 = e / N3, n3 = e - n2 * N3;
        plane[n2 * S + n3] = cjmul<T>(pi[e], pj[e]);
    }
    __syncthreads();
    fft_lines_n<T, -1>(N3, plane, N2, 1, S, tw + 2 * kMaxN);
    fft_lines_n<T, -1>(N2, plane, N3, S, 1, tw + kMaxN);
    cplx<T>* out = X + (size_t)p * B.ng + (size_t)n1 * plane_sz;
    for (int e = threadIdx.x; e < plane_sz; e += kFftThreads) {
        const int m2 = e / N3, m3 = e - m2 * N3;
        out[e] = plane[m2 * S + m3];
    }
}

// ---------------------------------------------------------------------------
// pass 2
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kFftThreads) pass2_kernel(PairBatch B, cplx<T>* __restrict__ X,
                                                            const cplx<T>* __restrict__ twg,
                                                            double* __restrict__ parts, int deriv_only) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
    double* red = reinterpret_cast<double*>(tw + 3 * kMaxN);
    cplx<T>* tile = reinterpret_cast<cplx<T>*>(red + kFftThreads);
    const int N1 = B.N1, N2 = B.N2, N3 = B.N3, S = N3 + 1;
    const int m2i = blockIdx.x % N2;
    const int p = blockIdx.x / N2;
    const int b = B.b0 + p / (B.nocc * B.nocc);
    load_twiddles<T>(tw, twg);
    cplx<T>* base = X + (size_t)p * B.ng + (size_t)m2i * N3;
    const size_t rs = (size_t)N2 * N3;
    const int tile_sz = N1 * N3;
    for (int e = threadIdx.x; e < tile_sz; e += kFftThreads) {
        const int n1 = e / N3, m3 = e - n1 * N3;
        tile[n1 * S + m3] = base[n1 * rs + m3];
    }
    __syncthreads();
    fft_lines_n<T, -1>(N1, tile, N3, S, 1, tw);

    double qa[3], qb[3];
    kfrac_of(B.a, B.M1, B.M2, B.M3, qa);
    kfrac_of(b, B.M1, B.M2, B.M3, qb);
    const double q0 = qa[0] - qb[0], q1 = qa[1] - qb[1], q2 = qa[2] - qb[2];
    const T om = T(B.omega);
    Recip<T> rc;
#pragma unroll
    for (int d = 0; d < 9; ++d) rc.b[d] = T(B.recip[d]);
    const int m2 = freq(m2i, N2);
    const bool sym = B.nyquist == OCCRIK_NYQUIST_SYMMETRIC;
    const T scale = T(B.inv_ng);
    double acc = 0.0;
    for (int e = threadIdx.x; e < tile_sz; e += kFftThreads) {
        const int t1 = e / N3, t3 = e - t1 * N3;
        const int m1 = freq(t1, N1), m3 = freq(t3, N3);
        const T x2 = momentum_sq<T>(rc, q0, q1, q2, m1, m2, m3);
        const bool nyq = sym && ((2 * m1 == -N1) || (2 * m2 == -N2) || (2 * m3 == -N3));
        T x2m = x2;
        if (nyq) {
            const int mm1 = (2 * m1 == -N1) ? -m1 : m1;
            const int mm2 = (2 * m2 == -N2) ? -m2 : m2;
            const int mm3 = (2 * m3 == -N3) ? -m3 : m3;
            x2m = momentum_sq<T>(rc, q0, q1, q2, mm1, mm2, mm3);
        }
        cplx<T> u = tile[t1 * S + t3];
        if (deriv_only) {
            T d = kernel_dfdw<T>(x2, B.kernel, om);
            if (nyq) d = T(0.5) * (d + kernel_dfdw<T>(x2m, B.kernel, om));
            acc += double(d) * (double(u.x) * double(u.x) + double(u.y) * double(u.y));
            continue;
        }
        T f = kernel_f<T>(x2, B.kernel, om);
        if (nyq) f = T(0.5) * (f + kernel_f<T>(x2m, B.kernel, om));
        if (B.parseval) acc += double(f) * (double(u.x) * double(u.x) + double(u.y) * double(u.y));
        tile[t1 * S + t3] = cscale<T>(u, f * scale);
    }
    if (B.parseval || deriv_only) {
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int w = kFftThreads / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) parts[blockIdx.x] = red[0];
    }
    if (deriv_only) return;
    __syncthreads();
    fft_lines_n<T, +1>(N1, tile, N3, S, 1, tw);
    fft_lines_n<T, +1>(N3, tile, N1, 1, S, tw + 2 * kMaxN);
    for (int e = threadIdx.x; e < tile_sz; e += kFftThreads) {
        const int n1 = e / N3, n3 = e - n1 * N3;
        base[n1 * rs + n3] = tile[n1 * S + n3];
    }
}

// ---------------------------------------------------------------------------
// pass 3
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kFftThreads) pass3_kernel(PairBatch B, const cplx<T>* __restrict__ X,
                                                            const cplx<T>* __restrict__ psi,
                                                            cplx<T>* __restrict__ Wpart,
                                                            const cplx<T>* __restrict__ twg) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* plane = tw + 3 * kMaxN;
    constexpr int ACC = (kMaxN * kMaxN + kFftThreads - 1) / kFftThreads;
    const int N2 = B.N2, N3 = B.N3, S = N3 + 1;
    const int plane_sz = N2 * N3;
    const int n1 = blockIdx.x % B.N1;
    const int j = (blockIdx.x / B.N1) % B.nocc;
    const int s = blockIdx.x / (B.N1 * B.nocc);
    const int total = B.nb * B.nocc;
    const int chunk = (total + B.splits - 1) / B.splits;
    const int q0 = s * chunk;
    const int q1 = min(total, q0 + chunk);
    load_twiddles<T>(tw, twg);
    cplx<T> acc[ACC];
#pragma unroll
    for (int t = 0; t < ACC; ++t) acc[t] = mk<T>(T(0), T(0));
    for (int q = q0; q < q1; ++q) {
        const int bb = q / B.nocc, i = q - bb * B.nocc;
        const int p = q * B.nocc + j;
        const cplx<T>* src = X + (size_t)p * B.ng + (size_t)n1 * plane_sz;
        for (int e = threadIdx.x; e < plane_sz; e += kFftThreads) {
            const int m2 = e / N3, n3 = e - m2 * N3;
            plane[m2 * S + n3] = src[e];
        }
        __syncthreads();
        fft_lines_n<T, +1>(N2, plane, N3, S, 1, tw + kMaxN);
        const cplx<T>* pi = psi + ((size_t)(B.b0 + bb) * B.nocc + i) * B.ng + (size_t)n1 * plane_sz;
#pragma unroll
        for (int t = 0; t < ACC; ++t) {
            const int e = threadIdx.x + t * kFftThreads;
            if (e < plane_sz) {
                const int n2 = e / N3, n3 = e - n2 * N3;
                const cplx<T> v = plane[n2 * S + n3];
                const cplx<T> w = pi[e];
                acc[t] = mk<T>(acc[t].x + w.x * v.x - w.y * v.y, acc[t].y + w.x * v.y + w.y * v.x);
            }
        }
        __syncthreads();
    }
    cplx<T>* out = Wpart + ((size_t)s * B.nocc + j) * B.ng + (size_t)n1 * plane_sz;
#pragma unroll
    for (int t = 0; t < ACC; ++t) {
        const int e = threadIdx.x + t * kFftThreads;
        if (e < plane_sz) out[e] = acc[t];
    }
}

template <typename T>
__global__ void wreduce_kernel(PairBatch B, const cplx<T>* __restrict__ Wpart, cplx<T>* __restrict__ W) {
    const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t tot = (size_t)B.nocc * B.ng;
    if (n >= tot) return;
    cplx<T> acc = W[(size_t)B.a * tot + n];
    for (int s = 0; s < B.splits; ++s) acc = cadd<T>(acc, Wpart[(size_t)s * tot + n]);
    W[(size_t)B.a * tot + n] = acc;
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

}  // namespace

template <typename T>
hipError_t launch_pass1(const PairBatch& B, const cplx<T>* psi, cplx<T>* X, const cplx<T>* tw, hipStream_t s) {
    const unsigned grid = (unsigned)((size_t)B.N1 * B.nb * B.nocc * B.nocc);
    hipLaunchKernelGGL(pass1_kernel<T>, dim3(grid), dim3(kFftThreads), lds_plane_bytes<T>(B.N2, B.N3), s, B, psi, X,
                       tw);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pass2(const PairBatch& B, cplx<T>* X, const cplx<T>* tw, double* parts, int deriv_only,
                        hipStream_t s) {
    const unsigned grid = (unsigned)((size_t)B.N2 * B.nb * B.nocc * B.nocc);
    const size_t lds = lds_plane_bytes<T>(B.N1, B.N3) + sizeof(double) * kFftThreads;
    hipLaunchKernelGGL(pass2_kernel<T>, dim3(grid), dim3(kFftThreads), lds, s, B, X, tw, parts, deriv_only);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pass3(const PairBatch& B, const cplx<T>* X, const cplx<T>* psi, cplx<T>* Wpart, const cplx<T>* tw,
                        hipStream_t s) {
    const unsigned grid = (unsigned)((size_t)B.N1 * B.nocc * B.splits);
    hipLaunchKernelGGL(pass3_kernel<T>, dim3(grid), dim3(kFftThreads), lds_plane_bytes<T>(B.N2, B.N3), s, B, X, psi,
                       Wpart, tw);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_wreduce(const PairBatch& B, const cplx<T>* Wpart, cplx<T>* W, hipStream_t s) {
    const size_t tot = (size_t)B.nocc * B.ng;
    hipLaunchKernelGGL(wreduce_kernel<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, B, Wpart, W);
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
    template hipError_t launch_pass3<T>(const PairBatch&, const cplx<T>*, const cplx<T>*, cplx<T>*,            \
                                        const cplx<T>*, hipStream_t);                                           \
    template hipError_t launch_wreduce<T>(const PairBatch&, const cplx<T>*, cplx<T>*, hipStream_t);            \
    template hipError_t launch_fill_zero<T>(cplx<T>*, size_t, hipStream_t);
OCCRIK_INST(float)
OCCRIK_INST(double)
#undef OCCRIK_INST

}  // namespace occrik
