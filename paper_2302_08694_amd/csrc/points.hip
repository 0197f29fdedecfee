// Point preparation for spreading/interpolation: fold positions into the periodic box, locate the
// first fine-grid cell of each point's kernel support, and counting-sort the points by tile (bin).
//
// Fold (periodicity, Sec. 2): x <- x - L floor(x/L) in double; the fine-grid coordinate
// g = x n_f / L; the support of width w starts at i0 = ceil(g - w/2) (mod n_f) and the point's
// sub-cell position y = 2 (i0 - g + w/2) - 1 in [-1, 1) selects the kernel values (see params.cpp).
// Only (i0, y) are kept: the integer cell is exact and y is rounded to the plan precision, so FP32
// plans keep full positional resolution within a cell.
#include <climits>

#include "plan.hpp"

namespace fsib {

struct Geo {
  int dim;
  int w;
  double L;
  int64_t nf[3];
  int64_t tb[3];
  int64_t nt[3];
  int ninst;                  // instances of the plan; their bins follow one another
  int64_t nbins;              // bins of one instance
  const int64_t* inst_off;    // ninst + 1 point offsets (ninst > 1)
};

// Instance owning point j: the last i with inst_off[i] <= j (binary search; inst_off[0] = 0 <= j).
__device__ __forceinline__ int point_instance(const int64_t* __restrict__ off, int ninst, int64_t j) {
  int lo = 0, hi = ninst;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= j) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ void locate(double x, double L, int64_t nf, int w, int& i0, double& y, bool& bad) {
  if (!isfinite(x)) {
    bad = true;
    x = 0.0;
  }
  double xf = x - L * floor(x / L);
  // rounding can leave xf at L (x just below a multiple of L) or, for huge |x|, anywhere; both
  // are multiples of L to within that rounding
  if (!(xf >= 0.0 && xf < L)) xf = 0.0;
  double g = xf * ((double)nf / L);
  if (!(g < (double)nf)) g = 0.0;
  const double start = g - 0.5 * w;
  int i = (int)ceil(start);
  double s = (double)i - start;  // in [0, 1)
  double yy = 2.0 * s - 1.0;
  yy = yy < -1.0 ? -1.0 : (yy > 1.0 ? 1.0 : yy);
  if (i < 0) i += (int)nf;
  if (i < 0 || i >= (int)nf) i = 0;  // unreachable for g in [0, nf) and 2 <= w <= nf; keeps indices in range
  i0 = i;
  y = yy;
}

// Bin of every point and its rank inside the bin.  Neighbouring points of a mesh usually share a
// bin, so the lanes of a wavefront form runs of equal bins and the first lane of each run claims
// the whole run with one atomic add.  (The order of the runs inside a bin follows the order of the
// atomics.)  Needs blockDim.x a multiple of 64.
__global__ void k_bin_count(int64_t M, const double* __restrict__ X, Geo g, int* __restrict__ counts,
                            int* __restrict__ pt_bin, int* __restrict__ pt_rank, int* __restrict__ flag) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = j < M;
  int bin = -1;
  if (valid) {
    bool bad = false;
    int64_t b = 0, stride = 1;
    for (int a = 0; a < g.dim; ++a) {
      int i0;
      double y;
      locate(X[j * g.dim + a], g.L, g.nf[a], g.w, i0, y, bad);
      b += (i0 / g.tb[a]) * stride;
      stride *= g.nt[a];
    }
    if (bad) flag[0] = 1;
    if (g.ninst > 1) b += (int64_t)point_instance(g.inst_off, g.ninst, j) * g.nbins;
    bin = (int)b;
  }
  const int lane = threadIdx.x & 63;
  const int prev = __shfl_up(bin, 1, 64);
  const bool head = lane == 0 || prev != bin;
  const unsigned long long heads = __ballot(head);
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);  // lanes <= lane
  const int h = 63 - __clzll(heads & upto);                                       // head of my run
  const unsigned long long after = heads & ~upto;
  const int end = after ? __ffsll((long long)after) - 1 : 64;                     // next run's head
  int base = 0;
  if (valid && head) base = atomicAdd(&counts[bin], end - lane);
  base = __shfl(base, h, 64);
  if (valid) {
    pt_bin[j] = bin;
    pt_rank[j] = base + (lane - h);
  }
}

// Exclusive scan of counts[0..n) into offsets[0..n] (offsets[n] = total).  Segments of
// kScanSeg = 1024 threads x kScanEpt (4) consecutive entries: each thread loads its run of kScanEpt
// entries at once (one 16-byte load per lane, consecutive lanes on consecutive runs), the runs' sums
// are scanned across the workgroup (wavefront shuffles, then the wavefront totals), and each thread
// writes its run.  With more than one segment, a first launch stores the segment sums and a second
// one scans every segment after the sum of the segments before it (summed by the whole workgroup).
// Short segments give the bin counts of a plan (10^4-10^6) several workgroups: with 32 entries per
// thread a 65k-bin scan had 2 workgroups and lanes 128 bytes apart.
constexpr int kScanThreads = 1024;
constexpr int kScanEpt = 4;
constexpr int64_t kScanSeg = (int64_t)kScanThreads * kScanEpt;

// exclusive prefix of v over the workgroup; *total = sum over the workgroup
__device__ __forceinline__ int block_exclusive_scan(int v, int* wsum, int* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int u = __shfl_up(inc, off, 64);
    if (lane >= off) inc += u;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  if (wv == 0) {
    const int nw = blockDim.x >> 6;
    int x = lane < nw ? wsum[lane] : 0;
    int xi = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int u = __shfl_up(xi, off, 64);
      if (lane >= off) xi += u;
    }
    if (lane < nw) wsum[lane] = xi - x;  // exclusive prefix of the wavefront totals
    if (lane == nw - 1) wsum[64] = xi;
  }
  __syncthreads();
  *total = wsum[64];
  return wsum[wv] + inc - v;
}

template <bool FINAL>
__global__ __launch_bounds__(kScanThreads) void k_scan(int64_t n, const int* __restrict__ counts,
                                                       int* __restrict__ offsets, int* __restrict__ seg_sum) {
  __shared__ int wsum[65];
  __shared__ int seg_base;
  const int64_t first = (int64_t)blockIdx.x * kScanSeg + (int64_t)threadIdx.x * kScanEpt;
  int v[kScanEpt];
  int run = 0;
#pragma unroll
  for (int k = 0; k < kScanEpt; ++k) {
    v[k] = first + k < n ? counts[first + k] : 0;
    run += v[k];
  }
  int before = 0;  // this thread's share of the sums of the segments before this one
  if (FINAL)
    for (unsigned s = threadIdx.x; s < blockIdx.x; s += kScanThreads) before += seg_sum[s];
  int total;
  int excl = block_exclusive_scan(run, wsum, &total);
  if (FINAL) {
    int bt;
    __syncthreads();  // wsum is reused
    (void)block_exclusive_scan(before, wsum, &bt);
    if (threadIdx.x == 0) seg_base = bt;
    __syncthreads();
  }
  if (!FINAL) {
    if (threadIdx.x == 0) seg_sum[blockIdx.x] = total;
    return;
  }
  excl += seg_base;
#pragma unroll
  for (int k = 0; k < kScanEpt; ++k) {
    if (first + k <= n) offsets[first + k] = excl;
    excl += v[k];
  }
}

template <typename T>
__global__ void k_bin_scatter(int64_t M, const double* __restrict__ X, Geo g, const int* __restrict__ offsets,
                              const int* __restrict__ pt_bin, const int* __restrict__ pt_rank,
                              int* __restrict__ s_idx, uint32_t* __restrict__ s_i0, T* __restrict__ s_y) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const int64_t pos = (int64_t)offsets[pt_bin[j]] + pt_rank[j];
  bool bad = false;
  uint32_t packed = 0;
  const int bits = g.dim == 3 ? 10 : 16;
  for (int a = 0; a < g.dim; ++a) {
    int i0;
    double y;
    locate(X[j * g.dim + a], g.L, g.nf[a], g.w, i0, y, bad);
    packed |= (uint32_t)i0 << (bits * a);
    s_y[pos * g.dim + a] = (T)y;
  }
  s_idx[pos] = (int)j;
  s_i0[pos] = packed;
}

// Deterministic placement (plans created with deterministic = 1).  The run claims of k_bin_count give
// correct bin counts but an arrival-dependent order inside each bin, and with it the summation order
// of spreading.  Here every point's rank inside its bin becomes the number of points of the same bin
// with a smaller original index, so each bin lists its points in ascending index and the sums are
// bitwise reproducible.  The points are first placed by the claimed ranks (key[pos] = index); then one
// workgroup per bin sorts the bin's keys in LDS (bitonic network over the next power of two, padded
// with INT_MAX) and gives each point its position in the sorted order.  Bins of more than kRankLds
// points (far beyond the crowding of the workloads here) count, for every point, the smaller keys of
// the bin in global memory instead.
__global__ void k_bin_place(int64_t M, const int* __restrict__ offsets, const int* __restrict__ pt_bin,
                            const int* __restrict__ pt_rank, int* __restrict__ key) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  key[(int64_t)offsets[pt_bin[j]] + pt_rank[j]] = (int)j;
}

constexpr int kRankThreads = 256;
constexpr int kRankLds = 4096;  // keys sorted in LDS per bin

__global__ __launch_bounds__(kRankThreads) void k_bin_rank(const int* __restrict__ offsets,
                                                            const int* __restrict__ key, int* __restrict__ pt_rank) {
  __shared__ int sk[kRankLds];
  const int b = blockIdx.x;
  const int s = offsets[b], n = offsets[b + 1] - s;
  if (n <= 0) return;
  if (n == 1) {
    if (threadIdx.x == 0) pt_rank[key[s]] = 0;
    return;
  }
  if (n > kRankLds) {  // count smaller keys (quadratic; bins this crowded do not occur in the workloads)
    for (int i = threadIdx.x; i < n; i += kRankThreads) {
      const int k = key[s + i];
      int r = 0;
      for (int q = 0; q < n; ++q) r += key[s + q] < k ? 1 : 0;
      pt_rank[k] = r;
    }
    return;
  }
  int P = 2;
  while (P < n) P <<= 1;
  for (int i = threadIdx.x; i < P; i += kRankThreads) sk[i] = i < n ? key[s + i] : INT_MAX;
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += kRankThreads) {
        const int l = i ^ j;
        if (l > i) {
          const int a = sk[i], c = sk[l];
          const bool up = (i & k) == 0;
          if ((a > c) == up) {
            sk[i] = c;
            sk[l] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < n; i += kRankThreads) pt_rank[sk[i]] = i;
}

__global__ void k_fill_zero(uint32_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

template <typename T>
__global__ void k_axpy_pos(int64_t n, double* __restrict__ Y, const double* __restrict__ X, const T* __restrict__ U,
                           double a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) Y[i] = X[i] + a * (double)U[i];
}

static Geo make_geo(const Plan& p) {
  Geo g;
  g.dim = p.dim;
  g.w = p.w;
  g.L = p.L;
  for (int a = 0; a < 3; ++a) {
    g.nf[a] = p.nf[a];
    g.tb[a] = p.tb[a];
    g.nt[a] = p.nt[a];
  }
  g.ninst = p.ninst;
  g.nbins = p.nbins;
  g.inst_off = p.inst_off;
  return g;
}

hipError_t launch_fill_zero(void* ptr, int64_t bytes, hipStream_t st) {
  const int64_t n = bytes / 4;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (uint32_t*)ptr, n);
  return hipGetLastError();
}

// Block (yb, zb) of x lines is needed when a point of some bin (any bx, by in [yb-qy, yb],
// bz in [zb-qz, zb]) has a kernel support reaching it.
// rowmask[i * nt1 * nt2 + zb * nt1 + yb] for the blocks of instance i < ninst (bins of instance i
// follow those of instance i - 1)
__global__ void k_row_masks(int nt0, int nt1, int nt2, int qy, int qz, int ninst, const int* __restrict__ counts,
                            uint8_t* __restrict__ rowmask) {
  const int tg = blockIdx.x * blockDim.x + threadIdx.x;
  if (tg >= nt1 * nt2 * ninst) return;
  const int inst = tg / (nt1 * nt2), t = tg - inst * nt1 * nt2;
  const int yb = t % nt1, zb = t / nt1;
  const int* ci = counts + (int64_t)inst * nt0 * nt1 * nt2;
  int any = 0;
  for (int dz = 0; dz <= qz && !any; ++dz)
    for (int dy = 0; dy <= qy && !any; ++dy) {
      const int by = (yb - dy + nt1) % nt1, bz = (zb - dz + nt2) % nt2;
      const int* c = ci + (int64_t)(bz * nt1 + by) * nt0;
      for (int bx = 0; bx < nt0; ++bx) any |= c[bx];
    }
  rowmask[tg] = any ? 1 : 0;
}

__global__ void k_plane_masks(int nt1, int nt2, const uint8_t* __restrict__ rowmask, uint8_t* __restrict__ zmask) {
  const int zb = blockIdx.x * blockDim.x + threadIdx.x;
  if (zb >= nt2) return;
  uint8_t any = 0;
  for (int yb = 0; yb < nt1; ++yb) any |= rowmask[zb * nt1 + yb];
  zmask[zb] = any;
}

hipError_t launch_row_masks(Plan& p, hipStream_t st) {
  const int ni = p.dim == 2 ? p.ninst : 1;  // 3D multi-instance plans keep no masks
  const int nrb = (int)(p.nt[1] * p.nt[2]) * ni;
  hipLaunchKernelGGL(k_row_masks, dim3((nrb + 255) / 256), dim3(256), 0, st, (int)p.nt[0], (int)p.nt[1], (int)p.nt[2],
                     (int)p.qn[1], (int)p.qn[2], ni, (const int*)p.counts, p.rowmask);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_plane_masks, dim3((unsigned)((p.nt[2] + 255) / 256)), dim3(256), 0, st, (int)p.nt[1],
                     (int)p.nt[2], (const uint8_t*)p.rowmask, p.zmask);
  return hipGetLastError();
}

int64_t scan_segments(int64_t n) { return n / kScanSeg + 1; }

hipError_t launch_scan(int64_t n, const int* counts, int* offsets, int* seg_sum, hipStream_t st) {
  const int64_t nseg = scan_segments(n);
  if (nseg > 1) {
    hipLaunchKernelGGL(k_scan<false>, dim3((unsigned)nseg), dim3(kScanThreads), 0, st, n, counts, offsets, seg_sum);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_scan<true>, dim3((unsigned)nseg), dim3(kScanThreads), 0, st, n, counts, offsets, seg_sum);
  return hipGetLastError();
}

hipError_t launch_sort_points(Plan& p, int64_t M, const double* X, hipStream_t st) {
  Geo g = make_geo(p);
  hipError_t e = launch_fill_zero(p.counts, (p.nbt + 1) * (int64_t)sizeof(int), st);
  if (e != hipSuccess) return e;
  if (M > 0) {
    const unsigned nblk = (unsigned)((M + 255) / 256);
    hipLaunchKernelGGL(k_bin_count, dim3(nblk), dim3(256), 0, st, M, X, g, p.counts, p.pt_bin, p.pt_rank, p.flag);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = launch_scan(p.nbt, p.counts, p.offsets, p.scan_part, st)) != hipSuccess) return e;
  // masks: single-instance plans and 2D multi-instance plans
  if ((p.ninst == 1 || p.dim == 2) && (e = launch_row_masks(p, st)) != hipSuccess) return e;
  if (M > 0 && p.deterministic) {  // ranks by original index inside each bin
    const unsigned nblk = (unsigned)((M + 255) / 256);
    hipLaunchKernelGGL(k_bin_place, dim3(nblk), dim3(256), 0, st, M, (const int*)p.offsets, (const int*)p.pt_bin,
                       (const int*)p.pt_rank, p.det_key);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_rank, dim3((unsigned)p.nbt), dim3(kRankThreads), 0, st, (const int*)p.offsets,
                       (const int*)p.det_key, p.pt_rank);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (M > 0) {
    const unsigned nblk = (unsigned)((M + 255) / 256);
    if (p.prec == FSIB_F64)
      hipLaunchKernelGGL(k_bin_scatter<double>, dim3(nblk), dim3(256), 0, st, M, X, g, (const int*)p.offsets,
                         (const int*)p.pt_bin, (const int*)p.pt_rank, p.s_idx, p.s_i0, (double*)p.s_y);
    else
      hipLaunchKernelGGL(k_bin_scatter<float>, dim3(nblk), dim3(256), 0, st, M, X, g, (const int*)p.offsets,
                         (const int*)p.pt_bin, (const int*)p.pt_rank, p.s_idx, p.s_i0, (float*)p.s_y);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_axpy_positions(const Plan& p, int64_t M, double* Y, const double* X, const void* U, double a,
                                 hipStream_t st) {
  const int64_t n = M * p.dim;
  if (n <= 0) return hipSuccess;
  const unsigned nblk = (unsigned)((n + 255) / 256);
  if (p.prec == FSIB_F64)
    hipLaunchKernelGGL(k_axpy_pos<double>, dim3(nblk), dim3(256), 0, st, n, Y, X, (const double*)U, a);
  else
    hipLaunchKernelGGL(k_axpy_pos<float>, dim3(nblk), dim3(256), 0, st, n, Y, X, (const float*)U, a);
  return hipGetLastError();
}

}  // namespace fsib
