// Shared device/host helpers of the FSIB library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace fsib {

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
  T x, y;
};

template <typename T>
__host__ __device__ __forceinline__ cplx<T> mk(T a, T b) {
  cplx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator*(cplx<T> a, T s) { return mk(a.x * s, a.y * s); }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> conj(cplx<T> a) { return mk(a.x, -a.y); }
// multiply by i*s for s = +-1
template <typename T>
__host__ __device__ __forceinline__ cplx<T> mul_i(cplx<T> a, T s) { return mk(-a.y * s, a.x * s); }

constexpr int kMaxW = 16;       // largest kernel width (fine cells)
constexpr int kMaxDeg = 19;     // largest polynomial degree of the kernel pieces
constexpr int kMaxStages = 16;  // FFT stages

// Polynomial pieces of the spreading kernel: piece j (cell offset j of the support) is
// sum_i coef[i*w + j] * y^i, y in [-1, 1] the point's sub-cell position.
struct KernelPoly {
  int w;
  int deg;
  double beta;
};

// FFT pass description: a batch of 1-D transforms of length n along one axis of a
// [outer][len][inner] array; the input holds `nin` entries of that axis (zero-padded to n: entries
// i < pin sit at t = i, the rest at t = n - (nin - i)), the output keeps `nout` entries the same
// way (pout of them from the front).  fac_in/fac_out are per-entry real factors (nullable).
template <typename T>
struct FftArgs {
  int n;
  int nst;
  int radix[kMaxStages];
  const cplx<T>* tw;  // tw[t] = exp(-2 pi i t / n), t < n
  int sign;           // -1 forward, +1 inverse
  int64_t inner, outer;
  int nin, pin, nout, pout;
  const T* fac_in;
  const T* fac_out;
  T scale;
  int nb;             // transforms (columns) per workgroup
};

}  // namespace fsib
