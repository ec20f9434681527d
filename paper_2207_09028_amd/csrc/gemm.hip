// The two grid contractions of the build.
//
//   orbitals   psi~_{j k}(r) = sum_mu C_{mu j}(k) chi~_{mu k}(r)           (paper eq. occmo)
//   contract   K_{mu j}(k)   = -(dV/N_k) sum_r conj(chi~_{mu k}(r)) W~_{j k}(r)
//                                                      (the contraction of Alg. 3)
//
// Both stream the Bloch AOs on the grid (N_k x N_ao x N_g) once and are
// bandwidth-bound for the few occupied columns involved.  The contraction
// splits the grid sum into fixed chunks, keeps each chunk's sum in the working
// precision, and adds the chunk partials in FP64 in a fixed order.
#include "internal.hpp"

namespace occrik {

namespace {

constexpr int kMaxOcc = 16;
constexpr int kCChunk = 128;     // AOs of C staged in LDS at a time

template <typename T>
__global__ void __launch_bounds__(256) orbitals_kernel(const cplx<T>* __restrict__ chi, const double2* __restrict__ C,
                                                       cplx<T>* __restrict__ psi, int nao, int nocc, int ng) {
    __shared__ cplx<T> cs[kCChunk * kMaxOcc];
    const int k = blockIdx.y;
    const int n = blockIdx.x * 256 + threadIdx.x;
    cplx<T> acc[kMaxOcc];
#pragma unroll
    for (int j = 0; j < kMaxOcc; ++j) acc[j] = mk<T>(T(0), T(0));
    const double2* Ck = C + (size_t)k * nao * nocc;
    const cplx<T>* ck = chi + (size_t)k * nao * ng;
    for (int m0 = 0; m0 < nao; m0 += kCChunk) {
        const int mc = min(kCChunk, nao - m0);
        __syncthreads();
        for (int t = threadIdx.x; t < mc * nocc; t += 256) {
            const double2 c = Ck[(size_t)m0 * nocc + t];
            cs[t] = mk<T>(T(c.x), T(c.y));
        }
        __syncthreads();
        if (n < ng) {
            for (int m = 0; m < mc; ++m) {
                const cplx<T> x = ck[(size_t)(m0 + m) * ng + n];
#pragma unroll
                for (int j = 0; j < kMaxOcc; ++j) {
                    if (j < nocc) {
                        const cplx<T> c = cs[m * nocc + j];
                        acc[j] = mk<T>(acc[j].x + c.x * x.x - c.y * x.y, acc[j].y + c.x * x.y + c.y * x.x);
                    }
                }
            }
        }
    }
    if (n < ng) {
#pragma unroll
        for (int j = 0; j < kMaxOcc; ++j)
            if (j < nocc) psi[((size_t)k * nocc + j) * ng + n] = acc[j];
    }
}

// One wave per AO, 4 AOs per workgroup, a chunk of grid points per workgroup.
template <typename T>
__global__ void __launch_bounds__(256) contract_kernel(const cplx<T>* __restrict__ chi, const cplx<T>* __restrict__ W,
                                                       double2* __restrict__ Kpart, int nao, int nocc, int ng,
                                                       int chunk) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = blockIdx.x;
    const int mu = blockIdx.y * 4 + wave;
    const int k = blockIdx.z;
    const int nchunks = gridDim.x;
    const int n0 = c * chunk;
    const int n1 = min(ng, n0 + chunk);
    cplx<T> acc[kMaxOcc];
#pragma unroll
    for (int j = 0; j < kMaxOcc; ++j) acc[j] = mk<T>(T(0), T(0));
    if (mu < nao) {
        const cplx<T>* x = chi + ((size_t)k * nao + mu) * ng;
        const cplx<T>* w = W + (size_t)k * nocc * ng;
        for (int n = n0 + lane; n < n1; n += 64) {
            const cplx<T> xv = x[n];
#pragma unroll
            for (int j = 0; j < kMaxOcc; ++j) {
                if (j < nocc) {
                    const cplx<T> wv = w[(size_t)j * ng + n];
                    acc[j] = mk<T>(acc[j].x + xv.x * wv.x + xv.y * wv.y, acc[j].y + xv.x * wv.y - xv.y * wv.x);
                }
            }
        }
    }
    // wave reduction in FP64 of the per-lane partials (fixed order)
    __shared__ double red[4][64][2];
#pragma unroll
    for (int j = 0; j < kMaxOcc; ++j) {
        if (j >= nocc) break;
        red[wave][lane][0] = double(acc[j].x);
        red[wave][lane][1] = double(acc[j].y);
        __syncthreads();
        for (int w2 = 32; w2 > 0; w2 >>= 1) {
            if (lane < w2) {
                red[wave][lane][0] += red[wave][lane + w2][0];
                red[wave][lane][1] += red[wave][lane + w2][1];
            }
            __syncthreads();
        }
        if (lane == 0 && mu < nao) {
            double2 r;
            r.x = red[wave][0][0];
            r.y = red[wave][0][1];
            Kpart[(((size_t)k * nao + mu) * nocc + j) * nchunks + c] = r;
        }
        __syncthreads();
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
hipError_t launch_orbitals(const cplx<T>* chi, const double2* C, cplx<T>* psi, int nk, int nao, int nocc, int ng,
                           hipStream_t s) {
    dim3 grid((unsigned)((ng + 255) / 256), (unsigned)nk);
    hipLaunchKernelGGL(orbitals_kernel<T>, grid, dim3(256), 0, s, chi, C, psi, nao, nocc, ng);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_contract(const cplx<T>* chi, const cplx<T>* W, double2* Kpart, double2* Kmi, int nk, int nao,
                           int nocc, int ng, int nchunks, double scale, hipStream_t s) {
    const int chunk = (ng + nchunks - 1) / nchunks;
    dim3 grid((unsigned)nchunks, (unsigned)((nao + 3) / 4), (unsigned)nk);
    hipLaunchKernelGGL(contract_kernel<T>, grid, dim3(256), 0, s, chi, W, Kpart, nao, nocc, ng, chunk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t n = (size_t)nk * nao * nocc;
    hipLaunchKernelGGL(contract_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Kpart, Kmi, n,
                       nchunks, scale);
    return hipGetLastError();
}

template hipError_t launch_orbitals<float>(const cplx<float>*, const double2*, cplx<float>*, int, int, int, int,
                                           hipStream_t);
template hipError_t launch_orbitals<double>(const cplx<double>*, const double2*, cplx<double>*, int, int, int, int,
                                            hipStream_t);
template hipError_t launch_contract<float>(const cplx<float>*, const cplx<float>*, double2*, double2*, int, int, int,
                                           int, int, double, hipStream_t);
template hipError_t launch_contract<double>(const cplx<double>*, const cplx<double>*, double2*, double2*, int, int,
                                            int, int, int, double, hipStream_t);

}  // namespace occrik
