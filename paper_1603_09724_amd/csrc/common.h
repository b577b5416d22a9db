// Shared device/host definitions of libpomm: complex arithmetic, error handling,
// launch helpers.  gfx950 only (64-wide wavefronts).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>

namespace pomm {

constexpr int kWave = 64;

// ----------------------------------------------------------------- device memory
// The library's buffers are stream-ordered allocations (on the stream of the API
// call, bound with AllocBind) from the device's default pool, whose release
// threshold is raised so that memory freed by one handle is reused by the next
// setup instead of being unmapped and mapped again (memory.cpp).
hipStream_t& alloc_stream();
hipError_t dev_alloc_raw(void** p, size_t bytes);
hipError_t dev_free(void* p);
template <typename P>
inline hipError_t dev_alloc(P** p, size_t bytes) {
    return dev_alloc_raw(reinterpret_cast<void**>(p), bytes);
}
struct AllocBind {
    hipStream_t prev;
    explicit AllocBind(hipStream_t s) : prev(alloc_stream()) { alloc_stream() = s; }
    ~AllocBind() { alloc_stream() = prev; }
};

// ----------------------------------------------------------------- complex
template <typename T>
struct cplx {
    T re, im;
};
using c64 = cplx<float>;
using c128 = cplx<double>;

template <typename T>
__host__ __device__ __forceinline__ cplx<T> mk(T r, T i) { return cplx<T>{r, i}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator*(T s, cplx<T> a) { return {s * a.re, s * a.im}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> conj(cplx<T> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T>
__host__ __device__ __forceinline__ T norm2(cplx<T> a) { return a.re * a.re + a.im * a.im; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cdiv(cplx<T> a, cplx<T> b) {
    T d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
template <typename To, typename Ti>
__host__ __device__ __forceinline__ cplx<To> ccast(cplx<Ti> a) { return {(To)a.re, (To)a.im}; }

// ----------------------------------------------------------------- errors
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& msg) : std::runtime_error(msg), code(c) {}
};

#define POMM_HIP(call)                                                                       \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            throw ::pomm::Error(5, std::string("HIP error at " __FILE__ ":") +               \
                                       std::to_string(__LINE__) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define POMM_CHECK(cond, code, msg)                                         \
    do {                                                                    \
        if (!(cond)) throw ::pomm::Error((code), std::string(msg));         \
    } while (0)

inline void check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        throw Error(5, std::string("kernel launch failed (") + what + "): " + hipGetErrorString(e));
}

inline unsigned cdiv_u(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

// ----------------------------------------------------------------- reductions
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Block-wide sum of one value per thread; every thread gets the result.
// `scratch` must hold blockDim/64 values.  Contains two barriers.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* scratch) {
    v = wave_sum(v);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int nw = (blockDim.x + kWave - 1) / kWave;
    __syncthreads();
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    T s = 0;
    for (int i = 0; i < nw; ++i) s += scratch[i];  // fixed order: deterministic
    return s;
}

// Block-wide sums of two values per thread at once (both results in every thread).
// `scratch` must hold 2 x blockDim/64 values.  Contains two barriers.
template <typename T>
__device__ __forceinline__ void block_sum2(T& a, T& b, T (*scratch)[16]) {
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int nw = (blockDim.x + kWave - 1) / kWave;
    __syncthreads();
    if (lane == 0) {
        scratch[0][wid] = a;
        scratch[1][wid] = b;
    }
    __syncthreads();
    T sa = 0, sb = 0;
    for (int i = 0; i < nw; ++i) {   // fixed order: deterministic
        sa += scratch[0][i];
        sb += scratch[1][i];
    }
    a = sa;
    b = sb;
}

}  // namespace pomm
