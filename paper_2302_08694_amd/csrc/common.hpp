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

// Workgroup barrier for LDS traffic only: waits for this wave's LDS operations, then for every
// wave, but leaves global loads in flight (__syncthreads also waits for them), so loads issued
// for the next block of work overlap the current one.  The memory clobber keeps the compiler from
// moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Workgroups are dispatched to the chip's 8 XCDs in turn (workgroup i to XCD i mod 8) and each XCD
// has its own L2.  xcd_linear() renumbers a linear workgroup id so that each XCD receives one
// contiguous range of ids: neighbouring work (consecutive sorted points, adjacent tiles, FFT lines
// that share cache lines) then shares one L2 instead of being fetched into several.  It is a
// permutation of [0, n) whatever the dispatch order, so results never depend on it.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_linear(int64_t i, int64_t n) {
  const int64_t q = n / kXcds, r = n % kXcds;
  const int64_t x = i % kXcds, k = i / kXcds;
  return x * q + (x < r ? x : r) + k;
}

// The same in chunks: each XCD receives runs of C consecutive ids, the XCDs taking the runs in turn,
// which keeps most of the locality while spreading uneven work over all XCDs.  Ids past the last
// whole group of 8 C keep their number.
__device__ __forceinline__ int64_t xcd_chunked(int64_t i, int64_t n, int64_t C) {
  const int64_t g = kXcds * C;
  if (i >= n / g * g) return i;
  const int64_t s = i / g, r = i % g;
  return s * g + (r % kXcds) * C + r / kXcds;
}

// ---- launches over several plans ----
// One launch may carry the workgroups of several independent parts (the plans of a group), each with
// its own arguments and grid: part g owns workgroups [start[g], start[g+1]) of a one-dimensional
// launch.  Every part starts at a multiple of kXcds, so its workgroup i still lands on XCD i mod 8
// and the XCD-aware numbering inside its kernel works as in a launch of its own; the padding
// workgroups at the end of a part leave at once.  A kernel body sees its workgroup as a Blk: its
// coordinates and its grid, from the hardware registers in a launch of its own, from the part
// table in a launch over parts.
struct Blk {
  int64_t x, y;    // workgroup coordinates in the part's grid
  int64_t nx, ny;  // the part's grid
};
__device__ __forceinline__ Blk launch_blk() {
  return Blk{(int64_t)blockIdx.x, (int64_t)blockIdx.y, (int64_t)gridDim.x, (int64_t)gridDim.y};
}

constexpr int kMaxParts = 8;  // parts of one launch (the kernel arguments stay within 4 KiB)
template <class A>
struct Parts {
  A a[kMaxParts];
  uint32_t start[kMaxParts + 1];  // a launch has fewer than 2^32 workgroups
  uint32_t nx[kMaxParts], ny[kMaxParts];
  int n;
};

// Part of this workgroup (-1 for a padding workgroup) and its coordinates in the part's grid.  The
// coordinates are computed in 32 bits and widened, so the compiler knows their upper halves are zero
// and keeps the divisions that use them (the XCD renumbering) at 32-bit cost, as with the hardware
// registers.
template <class A>
__device__ __forceinline__ int part_blk(const Parts<A>& f, Blk& b) {
  const uint32_t w = blockIdx.x;
  int g = 0;
  while (g + 1 < f.n && w >= f.start[g + 1]) ++g;
  const uint32_t l = w - f.start[g], nx = f.nx[g], ny = f.ny[g];
  if (l >= nx * ny) return -1;
  if (ny == 1)
    b = Blk{(int64_t)l, 0, (int64_t)nx, 1};
  else
    b = Blk{(int64_t)(l % nx), (int64_t)(l / nx), (int64_t)nx, (int64_t)ny};
  return g;
}

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

// Occupancy masks of the fine grid (one byte per block of tile_y x tile_z grid lines along x):
// lines that no point's kernel support reaches are neither computed nor stored, and read as zero.
// For a strided pass the byte of entry i of line o is m[((o % omod) / odiv) * ostride + i / idiv]
// (idiv = 0: one byte per line).
struct StrideMask {
  const uint8_t* m;  // nullptr: no mask
  int omod, odiv, ostride, idiv;
};
// For a pass along x over rows r (= ((c * nz + z) * ny + y)): m[((r / ny) % nz / tbz) * nt1 + (r % ny) / tby],
// plus (r / rpi) * istride on multi-instance plans (rpi rows per instance, istride mask bytes per
// instance; rpi is huge and istride 0 otherwise).
struct RowMask {
  const uint8_t* m;  // nullptr: no mask
  int ny, nz, tby, tbz, nt1;
  int64_t rpi = INT64_MAX;
  int istride = 0;
};

__host__ __device__ __forceinline__ int mask_index(const StrideMask& k, int64_t o, int i) {
  return (int)(((o % k.omod) / k.odiv) * k.ostride) + (k.idiv > 0 ? i / k.idiv : 0);
}
__host__ __device__ __forceinline__ bool row_needed(const RowMask& k, int64_t r) {
  if (!k.m) return true;
  return k.m[(int)(r / k.rpi) * k.istride + (int)((r / k.ny) % k.nz / k.tbz) * k.nt1 + (int)(r % k.ny) / k.tby] != 0;
}

struct PassMasks {
  StrideMask line{nullptr, 1, 1, 0, 0};
  StrideMask ld{nullptr, 1, 1, 0, 0};
  StrideMask st{nullptr, 1, 1, 0, 0};
  RowMask rows{nullptr, 1, 1, 1, 1, 1};
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
  StrideMask line;    // strided passes: skip whole lines (masks on o only)
  StrideMask ld;      // strided passes: entries read as zero
  StrideMask st;      // strided passes: entries not stored
  RowMask rows;       // x passes: rows neither read nor stored
};

}  // namespace fsib
