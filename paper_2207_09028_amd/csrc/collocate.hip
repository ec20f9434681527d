// Bloch sums of cartesian Gaussians on the grid (paper Sec. II.A, Bloch AO;
// its 1/sqrt(N_k) dropped), stored as the cell-periodic parts
//
//   chi~_{mu k}(r_n) = e^{-ik.r_n} sum_T e^{ik.T} phi_mu(r_n - R_mu - T).
//
// The image sum is regrouped by image cell modulo the k-mesh: with T = t @ A
// and L = t mod M (componentwise), e^{ik.T} = e^{ik.L} exactly on a
// Gamma-centred mesh, so
//
//   fold   Phi_mu(r_n, L) = sum_{T in bucket L} phi_mu(r_n - R_mu - T)    (FP64, no k)
//   kdft   chi_{mu k}(r_n) = sum_L e^{2 pi i sum_d kappa_d L_d / M_d} Phi_mu(r_n, L)
//   store  chi~ = e^{-ik.r_n} chi, rounded once to the working precision.
//
// Every Gaussian is evaluated once instead of once per k-point.
#include "internal.hpp"

namespace occrik {

namespace {

template <int L>
__device__ inline void monomials(double x, double y, double z, double* m);
template <> __device__ inline void monomials<0>(double, double, double, double* m) { m[0] = 1.0; }
template <> __device__ inline void monomials<1>(double x, double y, double z, double* m) {
    m[0] = x; m[1] = y; m[2] = z;
}
template <> __device__ inline void monomials<2>(double x, double y, double z, double* m) {
    m[0] = x * x; m[1] = x * y; m[2] = x * z; m[3] = y * y; m[4] = y * z; m[5] = z * z;
}
template <> __device__ inline void monomials<3>(double x, double y, double z, double* m) {
    m[0] = x * x * x; m[1] = x * x * y; m[2] = x * x * z; m[3] = x * y * y; m[4] = x * y * z;
    m[5] = x * z * z; m[6] = y * y * y; m[7] = y * y * z; m[8] = y * z * z; m[9] = z * z * z;
}

template <int L>
__global__ void __launch_bounds__(256) fold_kernel(double* __restrict__ phi, const double4* __restrict__ img,
                                                   const int* __restrict__ bucket, ShellDev sh, CollocGeom g) {
    constexpr int NC = (L + 1) * (L + 2) / 2;
    const int nl = blockIdx.x * 256 + threadIdx.x;
    if (nl >= g.cnt) return;
    const int n = g.n0 + nl;
    const int n3 = n % g.N[2];
    const int n2 = (n / g.N[2]) % g.N[1];
    const int n1 = n / (g.N[1] * g.N[2]);
    const double f1 = double(n1) / g.N[0], f2 = double(n2) / g.N[1], f3 = double(n3) / g.N[2];
    const double rx = f1 * g.lat[0] + f2 * g.lat[3] + f3 * g.lat[6] - sh.R[0];
    const double ry = f1 * g.lat[1] + f2 * g.lat[4] + f3 * g.lat[7] - sh.R[1];
    const double rz = f1 * g.lat[2] + f2 * g.lat[5] + f3 * g.lat[8] - sh.R[2];
    for (int cell = 0; cell < g.nk; ++cell) {
        double acc[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = 0.0;
        const int t1 = bucket[cell + 1];
        for (int t = bucket[cell]; t < t1; ++t) {
            const double4 T = img[t];
            const double x = rx - T.x, y = ry - T.y, z = rz - T.z;
            const double e = exp(-sh.alpha * (x * x + y * y + z * z));
            double m[NC];
            monomials<L>(x, y, z, m);
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[c] += m[c] * e;
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) phi[((size_t)c * g.nk + cell) * g.cnt + nl] = sh.norm[c] * acc[c];
    }
}

// DFT along one k-mesh axis of a [M1][M2][M3][ng] array with e^{+2 pi i kappa l / M}.
// real_in: the input is real (first axis), else complex.
__global__ void __launch_bounds__(256) axis_dft_kernel(const double* __restrict__ in_real,
                                                       const double2* __restrict__ in_c, double2* __restrict__ out,
                                                       int M, int inner, int outer, int ng, int real_in) {
    // e^{2 pi i t / M}, t = kappa l mod M, once per workgroup
    __shared__ double2 tw[16];
    if (threadIdx.x < M) {
        double sn, cs;
        sincospi(2.0 * double(threadIdx.x) / double(M), &sn, &cs);
        tw[threadIdx.x] = make_double2(cs, sn);
    }
    __syncthreads();
    // thread over (outer index o, inner index q, grid point n); the axis has stride inner*ng
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t per = (size_t)inner * ng;
    if (gid >= (size_t)outer * per) return;
    const size_t o = gid / per;
    const size_t rem = gid - o * per;
    const size_t stride = per;
    const size_t base = o * (size_t)M * per + rem;
    double2 v[16];
    for (int l = 0; l < M; ++l) {
        if (real_in) v[l] = make_double2(in_real[base + l * stride], 0.0);
        else v[l] = in_c[base + l * stride];
    }
    for (int kap = 0; kap < M; ++kap) {
        double sx = 0.0, sy = 0.0;
        for (int l = 0; l < M; ++l) {
            const double2 w = tw[(kap * l) % M];
            sx += w.x * v[l].x - w.y * v[l].y;
            sy += w.x * v[l].y + w.y * v[l].x;
        }
        out[base + kap * stride] = make_double2(sx, sy);
    }
}

template <typename T>
__global__ void store_kernel(const double2* __restrict__ chik, cplx<T>* __restrict__ chi, int mu, int nao,
                             size_t ldc, size_t coff, CollocGeom g) {
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)g.nk * g.cnt) return;
    const int k = (int)(gid / g.cnt);
    const int nl = (int)(gid - (size_t)k * g.cnt);
    const int n = g.n0 + nl;
    const int k3 = k % g.M[2], k2 = (k / g.M[2]) % g.M[1], k1 = k / (g.M[1] * g.M[2]);
    const int n3 = n % g.N[2], n2 = (n / g.N[2]) % g.N[1], n1 = n / (g.N[1] * g.N[2]);
    // k.r_n = 2 pi sum_d kappa_d n_d / (M_d N_d), reduced exactly before the FP64 division
    const long d1 = (long)g.M[0] * g.N[0], d2 = (long)g.M[1] * g.N[1], d3 = (long)g.M[2] * g.N[2];
    const double fr = double(((long)k1 * n1) % d1) / double(d1) + double(((long)k2 * n2) % d2) / double(d2) +
                      double(((long)k3 * n3) % d3) / double(d3);
    double sn, cs;
    sincospi(-2.0 * fr, &sn, &cs);
    const double2 v = chik[gid];
    chi[((size_t)k * nao + mu) * ldc + coff + nl] = mk<T>(T(cs * v.x - sn * v.y), T(cs * v.y + sn * v.x));
}

}  // namespace

hipError_t launch_colloc_fold(double* phi, const double4* img, const int* bucket, const ShellDev& sh,
                              const CollocGeom& g, hipStream_t s) {
    dim3 grid((unsigned)((g.cnt + 255) / 256));
    switch (sh.l) {
        case 0: hipLaunchKernelGGL(fold_kernel<0>, grid, dim3(256), 0, s, phi, img, bucket, sh, g); break;
        case 1: hipLaunchKernelGGL(fold_kernel<1>, grid, dim3(256), 0, s, phi, img, bucket, sh, g); break;
        case 2: hipLaunchKernelGGL(fold_kernel<2>, grid, dim3(256), 0, s, phi, img, bucket, sh, g); break;
        case 3: hipLaunchKernelGGL(fold_kernel<3>, grid, dim3(256), 0, s, phi, img, bucket, sh, g); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_colloc_kdft(const double* phi_real, double2* work0, double2* work1, const CollocGeom& g,
                              hipStream_t s, double2** result) {
    // axes in the order 3, 2, 1; array layout [M1][M2][M3][cnt]
    const int M1 = g.M[0], M2 = g.M[1], M3 = g.M[2];
    const size_t total = (size_t)g.nk * g.cnt;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    // axis 3: inner = 1, outer = M1*M2
    hipLaunchKernelGGL(axis_dft_kernel, dim3(blocks), dim3(256), 0, s, phi_real, (const double2*)nullptr, work0, M3, 1,
                       M1 * M2, g.cnt, 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // axis 2: inner = M3, outer = M1
    hipLaunchKernelGGL(axis_dft_kernel, dim3(blocks), dim3(256), 0, s, (const double*)nullptr, work0, work1, M2, M3,
                       M1, g.cnt, 0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // axis 1: inner = M2*M3, outer = 1
    hipLaunchKernelGGL(axis_dft_kernel, dim3(blocks), dim3(256), 0, s, (const double*)nullptr, work1, work0, M1,
                       M2 * M3, 1, g.cnt, 0);
    *result = work0;
    return hipGetLastError();
}

template <typename T>
hipError_t launch_colloc_store(const double2* chik, cplx<T>* dst, int mu, int nao, size_t ldc, size_t coff,
                               const CollocGeom& g, hipStream_t s) {
    const size_t total = (size_t)g.nk * g.cnt;
    hipLaunchKernelGGL(store_kernel<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, chik, dst, mu, nao, ldc,
                       coff, g);
    return hipGetLastError();
}

template hipError_t launch_colloc_store<float>(const double2*, cplx<float>*, int, int, size_t, size_t,
                                               const CollocGeom&, hipStream_t);
template hipError_t launch_colloc_store<double>(const double2*, cplx<double>*, int, int, size_t, size_t,
                                                const CollocGeom&, hipStream_t);

}  // namespace occrik
