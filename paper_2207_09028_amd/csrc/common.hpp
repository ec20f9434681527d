// Shared device/host helpers of the occ-RI-K library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

namespace occrik {

template <typename T> struct vec2;
template <> struct vec2<float> { using type = float2; };
template <> struct vec2<double> { using type = double2; };
template <typename T> using cplx = typename vec2<T>::type;

template <typename T> __host__ __device__ inline cplx<T> mk(T x, T y) { cplx<T> r; r.x = x; r.y = y; return r; }
template <typename T> __device__ inline cplx<T> cadd(cplx<T> a, cplx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ inline cplx<T> csub(cplx<T> a, cplx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ inline cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <typename T> __device__ inline cplx<T> cjmul(cplx<T> a, cplx<T> b) {
    return mk<T>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <typename T> __device__ inline cplx<T> cscale(cplx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
template <typename T> __device__ inline cplx<T> cconj(cplx<T> a) { return mk<T>(a.x, -a.y); }
// multiply by -i (forward) or +i (inverse): DIR = -1 gives -i
template <typename T, int DIR> __device__ inline cplx<T> mul_i(cplx<T> a) {
    return DIR < 0 ? mk<T>(a.y, -a.x) : mk<T>(-a.y, a.x);
}

// Largest grid extent along one dimension.
constexpr int kMaxN = 64;
// Threads of the FFT pass workgroups.
constexpr int kFftThreads = 256;

}  // namespace occrik
