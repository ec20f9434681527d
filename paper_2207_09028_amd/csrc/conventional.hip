// Kernels of the conventional GPW exchange algorithms (paper Sec. II.B, Alg. 1,
// AO-RI-K; Sec. II.C, Alg. 2, MO-RI-K) that the occ-RI-K build does not have.
// Their pair round trips run through the same three passes as occ-RI-K, with
// the Bloch AOs of the output k-point as the output orbitals.
//
//   density_orbitals  psi~_{sigma k}(r) = sum_lambda P_{lambda sigma}(k) chi_{lambda k}(r)
//                     (eq. aointerm), formed as sum_i conj(C_{sigma i}) psi_{i k}(r) since
//                     P_{lambda sigma} = sum_i C_{lambda i} conj(C_{sigma i})
//   reduce_columns    the FP64 chunk partials of one group of K columns, summed in
//                     chunk order and placed in the full AO x AO block (eq. aok)
//   conv_energy       e_k = Re tr(C^H K C) / (2 N_k) over the occupied columns
#include "internal.hpp"

namespace occrik {

namespace {

constexpr int kMaxSum = 16;   // occupied orbitals held per thread

template <typename T>
__global__ void __launch_bounds__(256) density_orbitals_kernel(const double2* __restrict__ C,
                                                               const cplx<T>* __restrict__ psi,
                                                               cplx<T>* __restrict__ psit, int nao, int ncol,
                                                               int nocc, int ng) {
    const int k = blockIdx.y;
    const size_t n = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= (size_t)ng) return;
    cplx<T> p[kMaxSum];
#pragma unroll
    for (int i = 0; i < kMaxSum; ++i)
        p[i] = i < nocc ? psi[((size_t)k * ncol + i) * ng + n] : mk<T>(T(0), T(0));
    const double2* Ck = C + (size_t)k * nao * ncol;
    cplx<T>* out = psit + (size_t)k * nao * ng + n;
    for (int s = 0; s < nao; ++s) {
        T re = T(0), im = T(0);
#pragma unroll
        for (int i = 0; i < kMaxSum; ++i) {
            if (i < nocc) {
                const double2 c = Ck[(size_t)s * ncol + i];
                const T cr = T(c.x), ci = T(c.y);
                // conj(c) p
                re += cr * p[i].x + ci * p[i].y;
                im += cr * p[i].y - ci * p[i].x;
            }
        }
        out[(size_t)s * ng] = mk<T>(re, im);
    }
}

__global__ void reduce_columns_kernel(const double2* __restrict__ Kpart, double2* __restrict__ dst, int rows,
                                      int ncols, int ld, int col0, int nchunks, double scale) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)rows * ncols) return;
    const int r = (int)(t / ncols), j = (int)(t - (size_t)r * ncols);
    double sx = 0.0, sy = 0.0;
    for (int c = 0; c < nchunks; ++c) {
        const double2 v = Kpart[t * nchunks + c];
        sx += v.x;
        sy += v.y;
    }
    dst[(size_t)r * ld + col0 + j] = make_double2(scale * sx, scale * sy);
}

// one workgroup per k: Re sum_{i < nocc} sum_mu conj(C_{mu i}) sum_nu K_{mu nu} C_{nu i}
__global__ void __launch_bounds__(256) conv_energy_kernel(const double2* __restrict__ C,
                                                          const double2* __restrict__ K, double* __restrict__ eterm,
                                                          int nk, int nao, int ncol, int nocc) {
    __shared__ double red[256];
    const int k = blockIdx.x;
    const double2* Ck = C + (size_t)k * nao * ncol;
    const double2* Kk = K + (size_t)k * nao * nao;
    double acc = 0.0;
    for (int e = threadIdx.x; e < nao * nocc; e += 256) {
        const int mu = e / nocc, i = e - mu * nocc;
        double tr = 0.0, ti = 0.0;
        for (int nu = 0; nu < nao; ++nu) {
            const double2 kv = Kk[(size_t)mu * nao + nu];
            const double2 c = Ck[(size_t)nu * ncol + i];
            tr += kv.x * c.x - kv.y * c.y;
            ti += kv.x * c.y + kv.y * c.x;
        }
        const double2 cm = Ck[(size_t)mu * ncol + i];
        acc += cm.x * tr + cm.y * ti;   // Re(conj(cm) t)
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) eterm[k] = red[0] / (2.0 * nk);
}

}  // namespace

template <typename T>
hipError_t launch_density_orbitals(const double2* C, const cplx<T>* psi, cplx<T>* psit, int nk, int nao, int ncol,
                                   int nocc, int ng, hipStream_t s) {
    if (nocc > kMaxSum || nocc > ncol) return hipErrorInvalidValue;
    dim3 grid((unsigned)((ng + 255) / 256), (unsigned)nk);
    hipLaunchKernelGGL((density_orbitals_kernel<T>), grid, dim3(256), 0, s, C, psi, psit, nao, ncol, nocc, ng);
    return hipGetLastError();
}

hipError_t launch_reduce_columns(const double2* Kpart, double2* dst, int rows, int ncols, int ld, int col0,
                                 int nchunks, double scale, hipStream_t s) {
    const size_t n = (size_t)rows * ncols;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_columns_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Kpart, dst, rows,
                       ncols, ld, col0, nchunks, scale);
    return hipGetLastError();
}

hipError_t launch_conv_energy(const double2* C, const double2* K, double* eterm, int nk, int nao, int ncol, int nocc,
                              hipStream_t s) {
    hipLaunchKernelGGL(conv_energy_kernel, dim3((unsigned)nk), dim3(256), 0, s, C, K, eterm, nk, nao, ncol, nocc);
    return hipGetLastError();
}

template hipError_t launch_density_orbitals<float>(const double2*, const cplx<float>*, cplx<float>*, int, int, int,
                                                   int, int, hipStream_t);
template hipError_t launch_density_orbitals<double>(const double2*, const cplx<double>*, cplx<double>*, int, int,
                                                    int, int, int, hipStream_t);

}  // namespace occrik
