// Point preparation for spreading/interpolation: fold positions into the periodic box, locate the
// first fine-grid cell of each point's kernel support, and counting-sort the points by tile (bin).
//
// Fold (periodicity, Sec. 2): x <- x - L floor(x/L) in double; the fine-grid coordinate
// g = x n_f / L; the support of width w starts at i0 = ceil(g - w/2) (mod n_f) and the point's
// sub-cell position y = 2 (i0 - g + w/2) - 1 in [-1, 1) selects the kernel values (see params.cpp).
// Only (i0, y) are kept: the integer cell is exact and y is rounded to the plan precision, so FP32
// plans keep full positional resolution within a cell.
#include <climits>

#include "bins.hpp"
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
struct BinCountArgs {
  int64_t M;
  const double* X;
  Geo g;
  int* counts;
  int* pt_bin;
  int* pt_rank;
  int* flag;
  uint8_t* zclear;  // plane masks cleared by workgroup 0 before k_row_masks sets them (nullable)
  int nz;
  int* clear = nullptr;  // three counters zeroed by workgroup 0 (the spreading tiles' counters; nullable)
};

__device__ __forceinline__ void bin_count(const BinCountArgs& A, Blk blk) {
  const int64_t M = A.M;
  const double* __restrict__ X = A.X;
  const Geo& g = A.g;
  int* __restrict__ counts = A.counts;
  int* __restrict__ flag = A.flag;
  if (A.zclear && blk.x == 0)
    for (int k = threadIdx.x; k < A.nz; k += blockDim.x) A.zclear[k] = 0;
  if (A.clear && blk.x == 0 && threadIdx.x < 3) A.clear[threadIdx.x] = 0;
  const int64_t j = blk.x * blockDim.x + threadIdx.x;
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
    A.pt_bin[j] = bin;
    A.pt_rank[j] = base + (lane - h);
  }
}

__global__ void k_bin_count(BinCountArgs a) { bin_count(a, launch_blk()); }
__global__ void k_bin_count_parts(Parts<BinCountArgs> f) {
  Blk b;
  const int g = part_blk(f, b);
  if (g >= 0) bin_count(f.a[g], b);
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

struct ScanArgs {
  int64_t n;
  const int* counts;
  int* offsets;
  int* seg_sum;
  int* clear = nullptr;  // nullable: three counters zeroed by the final pass (the spreading tiles' counters)
};

template <bool FINAL, int EPT = kScanEpt>
__device__ __forceinline__ void scan_body(const ScanArgs& A, Blk blk) {
  constexpr int64_t SEG = (int64_t)kScanThreads * EPT;
  __shared__ int wsum[65];
  __shared__ int seg_base;
  const int64_t n = A.n;
  const int* __restrict__ counts = A.counts;
  int* __restrict__ offsets = A.offsets;
  int* __restrict__ seg_sum = A.seg_sum;
  const int64_t first = blk.x * SEG + (int64_t)threadIdx.x * EPT;
  int v[EPT];
  int run = 0;
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    v[k] = first + k < n ? counts[first + k] : 0;
    run += v[k];
  }
  int before = 0;  // this thread's share of the sums of the segments before this one
  if (FINAL)
    for (int64_t s = threadIdx.x; s < blk.x; s += kScanThreads) before += seg_sum[s];
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
    if (threadIdx.x == 0) seg_sum[blk.x] = total;
    return;
  }
  if (A.clear && blk.x == 0 && threadIdx.x < 3) A.clear[threadIdx.x] = 0;
  excl += seg_base;
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    if (first + k <= n) offsets[first + k] = excl;
    excl += v[k];
  }
}

template <bool FINAL, int EPT = kScanEpt>
__global__ __launch_bounds__(kScanThreads) void k_scan(ScanArgs a) {
  scan_body<FINAL, EPT>(a, launch_blk());
}
// One workgroup of 8 entries per thread covers up to 8191 entries in a single pass (the bins of a 3D
// plan), where the segmented scan would take two launches.
constexpr int64_t kScanOnePass = (int64_t)kScanThreads * 8;
template <bool FINAL>
__global__ __launch_bounds__(kScanThreads) void k_scan_parts(Parts<ScanArgs> f) {
  Blk b;
  const int g = part_blk(f, b);
  if (g >= 0) scan_body<FINAL>(f.a[g], b);
}

template <typename T>
struct ScatterArgs {
  int64_t M;
  const double* X;
  Geo g;
  const int* offsets;
  const int* pt_bin;
  const int* pt_rank;
  int* s_idx;
  uint32_t* s_i0;
  T* s_y;
  int* counts;     // the bin counts, cleared here for the next sort (nothing reads them after the masks)
  int64_t ncounts;
  const T* str;    // real strengths, nch per point, placed in sorted order into sstr (nullable)
  T* sstr;
  int nch;
};

template <typename T>
__device__ __forceinline__ void bin_scatter(const ScatterArgs<T>& A, Blk blk) {
  const Geo& g = A.g;
  const double* __restrict__ X = A.X;
  T* __restrict__ s_y = A.s_y;
  const int64_t j = blk.x * blockDim.x + threadIdx.x;
  for (int64_t k = j; k < A.ncounts; k += blk.nx * blockDim.x) A.counts[k] = 0;
  if (j >= A.M) return;
  const int64_t pos = (int64_t)A.offsets[A.pt_bin[j]] + A.pt_rank[j];
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
  A.s_idx[pos] = (int)j;
  A.s_i0[pos] = packed;
  if (A.str)
    for (int ch = 0; ch < A.nch; ++ch) A.sstr[pos * A.nch + ch] = A.str[j * A.nch + ch];
}

template <typename T>
__global__ void k_bin_scatter(ScatterArgs<T> a) { bin_scatter<T>(a, launch_blk()); }
template <typename T>
__global__ void k_bin_scatter_parts(Parts<ScatterArgs<T>> f) {
  Blk b;
  const int g = part_blk(f, b);
  if (g >= 0) bin_scatter<T>(f.a[g], b);
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

struct FillArgs {
  uint32_t* p;
  int64_t n;
};
__device__ __forceinline__ void fill_zero(const FillArgs& A, Blk blk) {
  const int64_t i = blk.x * blockDim.x + threadIdx.x;
  if (i < A.n) A.p[i] = 0u;
}
__global__ void k_fill_zero(uint32_t* __restrict__ p, int64_t n) { fill_zero(FillArgs{p, n}, launch_blk()); }
__global__ void k_fill_zero_parts_one(FillArgs a) { fill_zero(a, launch_blk()); }
__global__ void k_fill_zero_parts(Parts<FillArgs> f) {
  Blk b;
  const int g = part_blk(f, b);
  if (g >= 0) fill_zero(f.a[g], b);
}

template <typename T>
struct AxpyArgs {
  int64_t n;
  double* Y;
  const double* X;
  const T* U;
  double a;
};
template <typename T>
__device__ __forceinline__ void axpy_pos(const AxpyArgs<T>& A, Blk blk) {
  const int64_t i = blk.x * blockDim.x + threadIdx.x;
  // one rounding (fma), as the position updates folded into the force and interpolation passes
  if (i < A.n) A.Y[i] = fma(A.a, (double)A.U[i], A.X[i]);
}
template <typename T>
__global__ void k_axpy_pos(int64_t n, double* __restrict__ Y, const double* __restrict__ X, const T* __restrict__ U,
                           double a) {
  axpy_pos<T>(AxpyArgs<T>{n, Y, X, U, a}, launch_blk());
}
template <typename T>
__global__ void k_axpy_pos_one(AxpyArgs<T> a) { axpy_pos<T>(a, launch_blk()); }
template <typename T>
__global__ void k_axpy_pos_parts(Parts<AxpyArgs<T>> f) {
  Blk b;
  const int g = part_blk(f, b);
  if (g >= 0) axpy_pos<T>(f.a[g], b);
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
struct RowMaskArgs {
  int nt0, nt1, nt2, qy, qz, ninst;
  const int* counts;
  uint8_t* rowmask;
  uint8_t* zmask;  // nullable: plane masks of instance 0, zb set when any of its blocks is reached
  TilePartsArgs tp;  // the spreading tiles' parts, by the threads past the row blocks (ntp of them)
  int ntp;
};
__device__ __forceinline__ void row_masks(const RowMaskArgs& A, Blk blk) {
  const int nt0 = A.nt0, nt1 = A.nt1, nt2 = A.nt2, qy = A.qy, qz = A.qz, ninst = A.ninst;
  const int* __restrict__ counts = A.counts;
  const int tg = (int)(blk.x * blockDim.x + threadIdx.x);
  const int nrb = nt1 * nt2 * ninst;
  if (tg >= nrb) {
    if (tg - nrb < A.ntp) tile_parts_at(A.tp, tg - nrb);
    return;
  }
  const int inst = tg / (nt1 * nt2), t = tg - inst * nt1 * nt2;
  const int yb = t % nt1, zb = t / nt1;
  const int* ci = counts + (int64_t)inst * nt0 * nt1 * nt2;
  // every count of the reaching bins is read (no early exit), so the loads go out together
  int any = 0;
  for (int dz = 0; dz <= qz; ++dz)
    for (int dy = 0; dy <= qy; ++dy) {
      const int by = (yb - dy + nt1) % nt1, bz = (zb - dz + nt2) % nt2;
      const int* c = ci + (int64_t)(bz * nt1 + by) * nt0;
#pragma unroll 8
      for (int bx = 0; bx < nt0; ++bx) any |= c[bx];
    }
  A.rowmask[tg] = any ? 1 : 0;
  // the byte of plane block zb, set through its 4-byte word (the masks are 256-byte aligned)
  if (any && A.zmask && inst == 0)
    atomicOr(reinterpret_cast<unsigned*>(A.zmask + (zb & ~3)), 1u << (8 * (zb & 3)));
}
__global__ void k_row_masks(RowMaskArgs a) { row_masks(a, launch_blk()); }
__global__ void k_row_masks_parts(Parts<RowMaskArgs> f) {
  Blk b;
  const int g = part_blk(f, b);
  if (g >= 0) row_masks(f.a[g], b);
}


// Plane masks exist on 3D one-instance plans (the passes of 3D multi-instance plans run dense).
static uint8_t* plane_masks_of(const Plan& p) { return p.dim == 3 && p.ninst == 1 ? p.zmask : nullptr; }

// Row masks, plane masks and the spreading tiles' parts of a plan (sets p.parts_split).
static PartLaunch<RowMaskArgs> row_mask_launch(Plan& p) {
  const int ni = p.dim == 2 ? p.ninst : 1;  // 3D multi-instance plans keep no masks
  const int nrb = (int)(p.nt[1] * p.nt[2]) * ni;
  PartLaunch<RowMaskArgs> L;
  // the tiles' parts (from the bin counts, which the scatter clears only later) and, directly, the
  // spreading work list (counters cleared by the bin scan or the bin count)
  const TilePartsArgs tp{p.dim, (int)p.nt[0], (int)p.nt[1], (int)p.nt[2], (int)p.qn[0], (int)p.qn[1], (int)p.qn[2],
                         p.ninst, p.split, (const int*)p.offsets, p.tile_parts, p.slot_ctr, 1, (int2*)p.work,
                         p.tile_slot, p.split_list, (const int*)p.counts};
  L.a = RowMaskArgs{(int)p.nt[0], (int)p.nt[1], (int)p.nt[2], (int)p.qn[1], (int)p.qn[2], ni, (const int*)p.counts,
                    p.rowmask, plane_masks_of(p), tp, (int)p.nbt};
  L.nx = (nrb + p.nbt + 255) / 256;
  p.parts_split = p.split;
  return L;
}

// Row masks, and the plane masks with them (cleared beforehand by k_bin_count, or here when no point
// was counted).
hipError_t launch_row_masks(Plan& p, int64_t M, hipStream_t st) {
  hipError_t e;
  if (M <= 0 && plane_masks_of(p) && (e = launch_fill_zero(p.zmask, (p.nt[2] + 3) / 4 * 4, st)) != hipSuccess)
    return e;
  const PartLaunch<RowMaskArgs> r = row_mask_launch(p);
  hipLaunchKernelGGL(k_row_masks, dim3((unsigned)r.nx), dim3(256), 0, st, r.a);
  return hipGetLastError();
}

int64_t scan_segments(int64_t n) { return n / kScanSeg + 1; }

// The bin scan and the row-mask pass of one plan in one launch of 1024-thread workgroups: workgroup 0
// scans the bin counts (EPT per thread, at most kScanMaskBins bins) while the others compute the masks
// and the tiles' parts, which read the counts, not the offsets.  The spreading tiles' counters are then
// cleared by the bin count.  Both halves are latency-bound chains of a few microseconds; side by side
// they take one.
constexpr int kScanMaskThreads = kScanThreads;
constexpr int64_t kScanMaskBins = (int64_t)kScanMaskThreads * 24 - 1;  // n + 1 offsets at 24 per thread
struct ScanMaskArgs {
  ScanArgs s;
  RowMaskArgs m;
};
template <int EPT>
__global__ __launch_bounds__(kScanMaskThreads) void k_scan_row_masks(ScanMaskArgs a) {
  if (blockIdx.x == 0) {
    scan_body<true, EPT>(a.s, Blk{0, 0, 1, 1});
    return;
  }
  row_masks(a.m, Blk{(int64_t)blockIdx.x - 1, 0, (int64_t)gridDim.x - 1, 1});
}

// The scan of the tiles' part counts with the spreading work list: the final pass's workgroup for a
// segment, once it has written that segment's offsets, lists the further parts of the segment's tiles
// (one launch fewer on the spreading path; a tile's entries need only its own offset).
struct ScanFillArgs {
  ScanArgs s;
  FillWorkArgs f;
};
template <int EPT>
__device__ __forceinline__ void scan_fill_body(const ScanFillArgs& A, Blk blk) {
  constexpr int64_t SEG = (int64_t)kScanThreads * EPT;
  scan_body<true, EPT>(A.s, blk);
  __syncthreads();  // the segment's offsets are complete and visible to the workgroup
  const int64_t n = A.s.n;
  const int64_t t1 = (blk.x + 1) * SEG < (int64_t)A.f.nbins ? (blk.x + 1) * SEG : (int64_t)A.f.nbins;
  for (int64_t t = blk.x * SEG + threadIdx.x; t < t1; t += kScanThreads) fill_work_tile(A.f, (int)t);
  // the number of entries, from the segment holding the total
  if (threadIdx.x == 0 && blk.x * SEG <= n && n < (blk.x + 1) * SEG) A.f.slot_ctr[2] = A.s.offsets[n] - (int)n;
}
template <int EPT>
__global__ __launch_bounds__(kScanThreads) void k_scan_fill(ScanFillArgs a) {
  scan_fill_body<EPT>(a, launch_blk());
}
__global__ __launch_bounds__(kScanThreads) void k_scan_fill_parts(Parts<ScanFillArgs> f) {
  Blk b;
  const int g = part_blk(f, b);
  if (g >= 0) scan_fill_body<kScanEpt>(f.a[g], b);
}

hipError_t launch_scan_fill_work(int64_t n, const int* counts, int* offsets, int* seg_sum, const FillWorkArgs& f,
                                 hipStream_t st) {
  const ScanFillArgs a{ScanArgs{n, counts, offsets, seg_sum}, f};
  if (n < kScanOnePass) {  // one workgroup of 8 entries per thread
    hipLaunchKernelGGL(k_scan_fill<8>, dim3(1), dim3(kScanThreads), 0, st, a);
    return hipGetLastError();
  }
  const int64_t nseg = scan_segments(n);
  hipLaunchKernelGGL(k_scan<false>, dim3((unsigned)nseg), dim3(kScanThreads), 0, st, a.s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_fill<kScanEpt>, dim3((unsigned)nseg), dim3(kScanThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_scan_fill_work_group(const std::vector<int64_t>& n, const std::vector<const int*>& counts,
                                       const std::vector<int*>& offsets, const std::vector<int*>& seg_sum,
                                       const std::vector<FillWorkArgs>& f, hipStream_t st) {
  std::vector<PartLaunch<ScanArgs>> first;
  std::vector<PartLaunch<ScanFillArgs>> fin;
  for (size_t g = 0; g < n.size(); ++g) {
    const int64_t nseg = scan_segments(n[g]);
    PartLaunch<ScanFillArgs> L;
    L.a = ScanFillArgs{ScanArgs{n[g], counts[g], offsets[g], seg_sum[g]}, f[g]};
    L.nx = nseg;
    L.threads = kScanThreads;
    fin.push_back(L);
    if (nseg > 1) {
      PartLaunch<ScanArgs> F;
      F.a = L.a.s;
      F.nx = nseg;
      F.threads = kScanThreads;
      first.push_back(F);
    }
  }
  hipError_t e = launch_parts(
      first,
      [&](const PartLaunch<ScanArgs>& L) {
        hipLaunchKernelGGL(k_scan<false>, dim3((unsigned)L.nx), dim3(kScanThreads), 0, st, L.a);
        return hipGetLastError();
      },
      [&](const Parts<ScanArgs>& pf, int64_t nwg, size_t, int) {
        hipLaunchKernelGGL(k_scan_parts<false>, dim3((unsigned)nwg), dim3(kScanThreads), 0, st, pf);
        return hipGetLastError();
      });
  if (e != hipSuccess) return e;
  return launch_parts(
      fin,
      [&](const PartLaunch<ScanFillArgs>& L) {
        hipLaunchKernelGGL(k_scan_fill<kScanEpt>, dim3((unsigned)L.nx), dim3(kScanThreads), 0, st, L.a);
        return hipGetLastError();
      },
      [&](const Parts<ScanFillArgs>& pf, int64_t nwg, size_t, int) {
        hipLaunchKernelGGL(k_scan_fill_parts, dim3((unsigned)nwg), dim3(kScanThreads), 0, st, pf);
        return hipGetLastError();
      });
}

hipError_t launch_scan(int64_t n, const int* counts, int* offsets, int* seg_sum, hipStream_t st, int* clear) {
  const int64_t nseg = scan_segments(n);
  const ScanArgs a{n, counts, offsets, seg_sum, clear};
  if (n < kScanOnePass) {  // n + 1 outputs in one segment
    hipLaunchKernelGGL((k_scan<true, 8>), dim3(1), dim3(kScanThreads), 0, st, a);
    return hipGetLastError();
  }
  if (nseg > 1) {
    hipLaunchKernelGGL(k_scan<false>, dim3((unsigned)nseg), dim3(kScanThreads), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_scan<true>, dim3((unsigned)nseg), dim3(kScanThreads), 0, st, a);
  return hipGetLastError();
}

// The scans of several plans' arrays (scans[g] = {n, counts, offsets, seg_sum}), one launch per pass.
static hipError_t launch_scan_parts(const std::vector<ScanArgs>& scans, hipStream_t st) {
  std::vector<PartLaunch<ScanArgs>> first, fin;
  for (const ScanArgs& a : scans) {
    const int64_t nseg = scan_segments(a.n);
    PartLaunch<ScanArgs> L;
    L.a = a;
    L.nx = nseg;
    L.threads = kScanThreads;
    fin.push_back(L);
    if (nseg > 1) first.push_back(L);
  }
  auto one = [&](bool final_pass) {
    return [=](const PartLaunch<ScanArgs>& L) {
      if (final_pass)
        hipLaunchKernelGGL(k_scan<true>, dim3((unsigned)L.nx), dim3(kScanThreads), 0, st, L.a);
      else
        hipLaunchKernelGGL(k_scan<false>, dim3((unsigned)L.nx), dim3(kScanThreads), 0, st, L.a);
      return hipGetLastError();
    };
  };
  auto fused = [&](bool final_pass) {
    return [=](const Parts<ScanArgs>& f, int64_t nwg, size_t, int) {
      if (final_pass)
        hipLaunchKernelGGL(k_scan_parts<true>, dim3((unsigned)nwg), dim3(kScanThreads), 0, st, f);
      else
        hipLaunchKernelGGL(k_scan_parts<false>, dim3((unsigned)nwg), dim3(kScanThreads), 0, st, f);
      return hipGetLastError();
    };
  };
  hipError_t e = launch_parts(first, one(false), fused(false));
  if (e != hipSuccess) return e;
  return launch_parts(fin, one(true), fused(true));
}

template <typename T>
static ScatterArgs<T> scatter_args(const Plan& p, int64_t M, const double* X, const void* str) {
  return ScatterArgs<T>{M, X, make_geo(p), (const int*)p.offsets, (const int*)p.pt_bin, (const int*)p.pt_rank,
                        p.s_idx, p.s_i0, (T*)p.s_y, p.counts, p.nbt + 1, (const T*)str, (T*)p.s_str, p.dim};
}

hipError_t launch_sort_points(Plan& p, int64_t M, const double* X, hipStream_t st, const void* str) {
  Geo g = make_geo(p);
  hipError_t e = hipSuccess;
  p.parts_split = 0;  // set again where the row-mask pass computes the tiles' parts
  // the bin counts start at zero: cleared by the last sort's scatter, else here
  if (!p.counts_zero && (e = launch_fill_zero(p.counts, (p.nbt + 1) * (int64_t)sizeof(int), st)) != hipSuccess)
    return e;
  p.counts_zero = true;  // after this sort: zero again (its scatter clears them; with M = 0 nothing is counted)
  // masks: single-instance plans and 2D multi-instance plans; with points counted and few bins the
  // scan runs inside the row-mask launch
  const bool masks = p.ninst == 1 || p.dim == 2;
  const bool fused = masks && M > 0 && p.nbt <= kScanMaskBins;
  if (M > 0) {
    const unsigned nblk = (unsigned)((M + 255) / 256);
    hipLaunchKernelGGL(k_bin_count, dim3(nblk), dim3(256), 0, st,
                       BinCountArgs{M, X, g, p.counts, p.pt_bin, p.pt_rank, p.flag, plane_masks_of(p), (int)p.nt[2],
                                    fused ? p.slot_ctr : nullptr});
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (fused) {
    const PartLaunch<RowMaskArgs> r = row_mask_launch(p);
    const ScanMaskArgs a{ScanArgs{p.nbt, p.counts, p.offsets, p.scan_part, nullptr}, r.a};
    const int nrb = (int)(p.nt[1] * p.nt[2]) * (p.dim == 2 ? (int)p.ninst : 1);
    const dim3 grid((unsigned)((nrb + p.nbt + kScanMaskThreads - 1) / kScanMaskThreads + 1));
    if (p.nbt < (int64_t)kScanMaskThreads * 8)
      hipLaunchKernelGGL(k_scan_row_masks<8>, grid, dim3(kScanMaskThreads), 0, st, a);
    else
      hipLaunchKernelGGL(k_scan_row_masks<24>, grid, dim3(kScanMaskThreads), 0, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  } else {
    if ((e = launch_scan(p.nbt, p.counts, p.offsets, p.scan_part, st, p.slot_ctr)) != hipSuccess) return e;
    if (masks && (e = launch_row_masks(p, M, st)) != hipSuccess) return e;
  }
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
      hipLaunchKernelGGL(k_bin_scatter<double>, dim3(nblk), dim3(256), 0, st, scatter_args<double>(p, M, X, str));
    else
      hipLaunchKernelGGL(k_bin_scatter<float>, dim3(nblk), dim3(256), 0, st, scatter_args<float>(p, M, X, str));
    e = hipGetLastError();
  }
  p.sstr_src = str;
  return e;
}

// Launch over parts of a kernel whose single-launch form is `k1` and fused form `kp`, with 256 threads.
#define FSIB_PARTS_256(k1, kp, Args)                                                                          \
  [&](const PartLaunch<Args>& L) {                                                                           \
    hipLaunchKernelGGL(k1, dim3((unsigned)L.nx, (unsigned)L.ny), dim3(256), 0, st, L.a);                      \
    return hipGetLastError();                                                                                \
  },                                                                                                         \
      [&](const Parts<Args>& f, int64_t nwg, size_t, int) {                                                  \
        hipLaunchKernelGGL(kp, dim3((unsigned)nwg), dim3(256), 0, st, f);                                    \
        return hipGetLastError();                                                                            \
      }

template <typename T>
static hipError_t scatter_group(const std::vector<Plan*>& ps, const int64_t* M, const double* const* X,
                                const void* const* str, hipStream_t st) {
  std::vector<PartLaunch<ScatterArgs<T>>> v(ps.size());
  for (size_t g = 0; g < ps.size(); ++g) {
    v[g].a = scatter_args<T>(*ps[g], M[g], X[g], str ? str[g] : nullptr);
    ps[g]->sstr_src = str ? str[g] : nullptr;
    v[g].nx = (M[g] + 255) / 256;
  }
  return launch_parts(v, FSIB_PARTS_256(k_bin_scatter<T>, k_bin_scatter_parts<T>, ScatterArgs<T>));
}

hipError_t launch_scan_group(const std::vector<int64_t>& n, const std::vector<const int*>& counts,
                             const std::vector<int*>& offsets, const std::vector<int*>& seg_sum, hipStream_t st) {
  std::vector<ScanArgs> sc(n.size());
  for (size_t g = 0; g < n.size(); ++g) sc[g] = ScanArgs{n[g], counts[g], offsets[g], seg_sum[g]};
  return launch_scan_parts(sc, st);
}

// launch_sort_points for the plans of a group (plan g with M[g] points at X[g]), each stage one launch
// over all plans (the ranking passes of deterministic plans one launch per plan).
hipError_t launch_sort_points_group(const std::vector<Plan*>& ps, const int64_t* M, const double* const* X,
                                    hipStream_t st, const void* const* str) {
  const size_t n = ps.size();
  std::vector<PartLaunch<FillArgs>> fz(n);
  std::vector<PartLaunch<BinCountArgs>> bc(n);
  std::vector<ScanArgs> sc(n);
  std::vector<PartLaunch<RowMaskArgs>> rm;
  for (size_t g = 0; g < n; ++g) {
    Plan& p = *ps[g];
    p.parts_split = 0;
    const int64_t words = p.nbt + 1;
    fz[g].a = FillArgs{(uint32_t*)p.counts, words};
    fz[g].nx = p.counts_zero ? 0 : (words + 255) / 256;  // cleared by the last sort's scatter
    ps[g]->counts_zero = true;
    bc[g].a = BinCountArgs{M[g], X[g], make_geo(p), p.counts, p.pt_bin, p.pt_rank, p.flag, plane_masks_of(p),
                           (int)p.nt[2]};
    bc[g].nx = (M[g] + 255) / 256;
    sc[g] = ScanArgs{p.nbt, p.counts, p.offsets, p.scan_part, p.slot_ctr};
    if (p.ninst == 1 || p.dim == 2) rm.push_back(row_mask_launch(p));
  }
  hipError_t e = launch_parts(fz, FSIB_PARTS_256(k_fill_zero_parts_one, k_fill_zero_parts, FillArgs));
  if (e != hipSuccess) return e;
  if ((e = launch_parts(bc, FSIB_PARTS_256(k_bin_count, k_bin_count_parts, BinCountArgs))) != hipSuccess) return e;
  if ((e = launch_scan_parts(sc, st)) != hipSuccess) return e;
  for (size_t g = 0; g < n; ++g)  // plane masks of plans with no point counted (k_bin_count clears the others)
    if (M[g] <= 0 && plane_masks_of(*ps[g]) &&
        (e = launch_fill_zero(ps[g]->zmask, (ps[g]->nt[2] + 3) / 4 * 4, st)) != hipSuccess)
      return e;
  if ((e = launch_parts(rm, FSIB_PARTS_256(k_row_masks, k_row_masks_parts, RowMaskArgs))) != hipSuccess) return e;
  for (size_t g = 0; g < n; ++g) {  // deterministic plans: ranks by original index, each plan on its own
    const Plan& p = *ps[g];
    if (!p.deterministic || M[g] <= 0) continue;
    hipLaunchKernelGGL(k_bin_place, dim3((unsigned)((M[g] + 255) / 256)), dim3(256), 0, st, M[g],
                       (const int*)p.offsets, (const int*)p.pt_bin, (const int*)p.pt_rank, p.det_key);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_rank, dim3((unsigned)p.nbt), dim3(kRankThreads), 0, st, (const int*)p.offsets,
                       (const int*)p.det_key, p.pt_rank);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return ps[0]->prec == FSIB_F64 ? scatter_group<double>(ps, M, X, str, st) : scatter_group<float>(ps, M, X, str, st);
}

// Zeroing of several device ranges (ptr[g], bytes[g], whole 4-byte words) in one launch.
hipError_t launch_fill_zero_group(const std::vector<void*>& ptr, const std::vector<int64_t>& bytes, hipStream_t st) {
  std::vector<PartLaunch<FillArgs>> v(ptr.size());
  for (size_t g = 0; g < ptr.size(); ++g) {
    v[g].a = FillArgs{(uint32_t*)ptr[g], bytes[g] / 4};
    v[g].nx = (bytes[g] / 4 + 255) / 256;
  }
  return launch_parts(v, FSIB_PARTS_256(k_fill_zero_parts_one, k_fill_zero_parts, FillArgs));
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

template <typename T>
static hipError_t axpy_group(const std::vector<Plan*>& ps, const int64_t* M, double* const* Y,
                             const double* const* X, const void* const* U, const double* a, hipStream_t st) {
  std::vector<PartLaunch<AxpyArgs<T>>> v(ps.size());
  for (size_t g = 0; g < ps.size(); ++g) {
    const int64_t n = M[g] * ps[g]->dim;
    v[g].a = AxpyArgs<T>{n, Y[g], X[g], (const T*)U[g], a[g]};
    v[g].nx = (n + 255) / 256;
  }
  return launch_parts(v, FSIB_PARTS_256(k_axpy_pos_one<T>, k_axpy_pos_parts<T>, AxpyArgs<T>));
}

// Y[g] = X[g] + a[g] U[g] for the plans of a group, one launch.
hipError_t launch_axpy_positions_group(const std::vector<Plan*>& ps, const int64_t* M, double* const* Y,
                                       const double* const* X, const void* const* U, const double* a,
                                       hipStream_t st) {
  return ps[0]->prec == FSIB_F64 ? axpy_group<double>(ps, M, Y, X, U, a, st) : axpy_group<float>(ps, M, Y, X, U, a, st);
}

}  // namespace fsib
