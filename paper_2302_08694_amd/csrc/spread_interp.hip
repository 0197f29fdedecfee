// Spreading onto and interpolation from the fine grid (App. A, eqs. type1_conv and type2_conv).
//
// Spreading is output-stationary: one workgroup owns one tile of the fine grid, accumulates every
// point whose kernel support meets the tile (register rows, see k_spread), and writes the tile
// once with plain coalesced stores -- no atomics and no separate zeroing pass.  Points are counting-sorted by the tile holding their first support cell, so the points
// that reach a tile live in that tile's bin and in the Q bins before it along each axis,
// Q = ceil((w-1)/tile).  Kernel values are the piecewise polynomials of params.cpp evaluated in
// registers (Horner) from the point's sub-cell position.
//
// Interpolation gathers the w^d cells of each point from the grid (sorted order, so neighbouring
// threads read neighbouring cells) and writes the result at the point's original index.
#include "plan.hpp"

namespace fsib {

constexpr int kSpreadThreads = 256;
constexpr int kChunk = 64;           // points staged per round
constexpr int kMaxTileCells = 1024;  // cells of one tile
constexpr int kTileX = 16;           // tile extent along x (one register row per thread)

constexpr int kSplit = 1024;         // points per part of a heavy tile

template <typename T>
struct SpreadArgs {
  const T* coef;        // (deg+1)*w
  int deg;
  const int* offsets;   // nbins+1
  const int* s_idx;
  const uint32_t* s_i0;
  const T* s_y;
  const T* str;         // strengths: real (M, nch) or complex (ntrans, M)
  T* sstr;              // the strengths in sorted order, [ntrans][M][NCH]
  T* grid;              // real: nch planes; complex: ntrans interleaved complex grids
  int64_t M;
  int nf[3];
  int tb[3];
  int nt[3];
  int q[3];             // neighbour bins to visit per axis (0..q)
  // work list: part b of the launch spreads points [q*kSplit, (q+1)*kSplit) of tile t
  const int* part_off;  // nbins+1 (exclusive scan of tile_parts)
  const int2* work;     // (t, q) per part
  const int* tile_parts;
  const int* tile_slot; // first scratch slot of a split tile
  T* scratch;           // split tiles: [ntrans][slots][NCH][kMaxTileCells] partial tiles
  int64_t slots;        // scratch slots per transform
  const uint8_t* rowmask;  // blocks of x lines reached by some point (lines elsewhere stay unwritten)
};

template <typename T, int W>
__device__ __forceinline__ void kernel_values(const T* __restrict__ coef, int deg, T y, T* v) {
#pragma unroll
  for (int j = 0; j < W; ++j) v[j] = coef[deg * W + j];
  for (int i = deg - 1; i >= 0; --i) {
#pragma unroll
    for (int j = 0; j < W; ++j) v[j] = v[j] * y + coef[i * W + j];
  }
}

template <int DIM>
__device__ __forceinline__ int unpack_i0(uint32_t p, int a) {
  return DIM == 3 ? (int)((p >> (10 * a)) & 1023u) : (int)((p >> (16 * a)) & 65535u);
}

// NCH channels per point: real vector strengths (NCH = components, planar grids) or one complex
// strength (NCH = 2, interleaved complex grid, transform index = blockIdx.y).
//
// Inside a tile every thread owns one row of kTileX cells along x (rows = tile_y * tile_z) and
// accumulates it in registers for a 1/TPR share of the tile's points; the lanes of a wavefront
// hold different rows and visit the same point together, so point data are LDS broadcasts and no
// atomics are needed.  The TPR partial rows are then summed in a fixed order through LDS and the
// tile is written once.  Dense clusters (e.g. the poles of a lat-long mesh, where thousands of
// points share a few cells) cost the same per point as isolated points.
template <typename T, int DIM, int W, int NCH, bool CPLX>
__global__ __launch_bounds__(kSpreadThreads) void k_spread(SpreadArgs<T> a) {
  constexpr int RS = kTileX + 1;  // padded LDS row stride
  __shared__ T accs[NCH][kMaxTileCells / kTileX][RS];
  __shared__ T wts[kChunk][DIM][W];
  __shared__ T wxr[kChunk][kTileX];  // x weights of the point on this tile's 16 columns (0 outside)
  __shared__ T sv[kChunk][NCH];
  __shared__ int vstart[kChunk][DIM];
  __shared__ int rbeg[27], rlen[27];
  __shared__ int nrange;

  const int tid = threadIdx.x;
  const int tr = blockIdx.y;
  if ((int)blockIdx.x >= a.part_off[a.nt[0] * a.nt[1] * a.nt[2]]) return;  // beyond the work list
  const int2 wk = a.work[blockIdx.x];
  const int tile_id = wk.x, part = wk.y;
  const int nparts = a.tile_parts[tile_id];
  int tcoord[3];
  {
    int64_t tile = tile_id;
    tcoord[0] = (int)(tile % a.nt[0]);
    tile /= a.nt[0];
    tcoord[1] = (int)(tile % a.nt[1]);
    tcoord[2] = DIM == 3 ? (int)(tile / a.nt[1]) : 0;
  }
  // no point reaches this tile's block of x lines: those lines are neither read nor written
  if (!a.rowmask[tcoord[2] * a.nt[1] + tcoord[1]]) return;
  const int rows = a.tb[1] * (DIM == 3 ? a.tb[2] : 1);
  const int tcells = kTileX * rows;
  int base[3] = {0, 0, 0};
  for (int d = 0; d < DIM; ++d) base[d] = tcoord[d] * a.tb[d];
  const int64_t cells = (int64_t)a.nf[0] * a.nf[1] * (DIM == 3 ? a.nf[2] : 1);
  // bins that can reach this tile: this one and up to q before it along each axis, read in parallel
  {
    const int qx = a.q[0] + 1, qy = a.q[1] + 1, qz = DIM == 3 ? a.q[2] + 1 : 1;
    if (tid < qx * qy * qz) {
      const int dx = tid % qx, dy = (tid / qx) % qy, dz = tid / (qx * qy);
      const int bx = (tcoord[0] - dx + a.nt[0]) % a.nt[0];
      const int by = (tcoord[1] - dy + a.nt[1]) % a.nt[1];
      const int bz = DIM == 3 ? (tcoord[2] - dz + a.nt[2]) % a.nt[2] : 0;
      const int b = bx + a.nt[0] * (by + a.nt[1] * bz);
      const int s0 = a.offsets[b], e0 = a.offsets[b + 1];
      rbeg[tid] = s0;
      rlen[tid] = e0 - s0;
    }
    __syncthreads();
    if (tid == 0) {
      int nr = 0;
      for (int r = 0; r < qx * qy * qz; ++r)
        if (rlen[r] > 0) {
          rbeg[nr] = rbeg[r];
          rlen[nr] = rlen[r];
          ++nr;
        }
      nrange = nr;
    }
    __syncthreads();
  }
  int total = 0;
  for (int r = 0; r < nrange; ++r) total += rlen[r];
  const int cbeg = part * kSplit;
  const int cend = total < cbeg + kSplit ? total : cbeg + kSplit;
  if (total == 0) {  // no point reaches this tile, but some reach its lines: zeros
    for (int i = tid; i < tcells; i += kSpreadThreads) {
      const int lx = i % kTileX;
      const int ly = (i / kTileX) % a.tb[1];
      const int lz = DIM == 3 ? i / (kTileX * a.tb[1]) : 0;
      const int gz = DIM == 3 ? base[2] + lz : 0;
      const int64_t g = ((int64_t)gz * a.nf[1] + base[1] + ly) * a.nf[0] + base[0] + lx;
      if (CPLX) {
        reinterpret_cast<cplx<T>*>(a.grid)[(int64_t)tr * cells + g] = mk((T)0, (T)0);
      } else {
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) a.grid[ch * cells + g] = (T)0;
      }
    }
    return;
  }
  const int tpr = kSpreadThreads / rows;  // threads per row
  const int row = tid % rows, sub = tid / rows;
  const int ly = row % a.tb[1];
  const int lz = DIM == 3 ? row / a.tb[1] : 0;
  T acc[kTileX][NCH];
#pragma unroll
  for (int x = 0; x < kTileX; ++x)
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) acc[x][ch] = (T)0;

  for (int c0 = cbeg; c0 < cend; c0 += kChunk) {
    const int cnt = cend - c0 < kChunk ? cend - c0 : kChunk;
    // stage: kernel values per axis, start offset relative to the tile, strengths
    for (int it = tid; it < cnt * DIM; it += kSpreadThreads) {
      const int pl = it / DIM, d = it % DIM;
      int vi = c0 + pl, r = 0;
      while (vi >= rlen[r]) vi -= rlen[r++];
      const int64_t pos = (int64_t)rbeg[r] + vi;
      T v[W];
      kernel_values<T, W>(a.coef, a.deg, a.s_y[pos * DIM + d], v);
#pragma unroll
      for (int j = 0; j < W; ++j) wts[pl][d][j] = v[j];
      int s = unpack_i0<DIM>(a.s_i0[pos], d) - base[d];
      if (s < 0) s += a.nf[d];
      vstart[pl][d] = s;
      if (d == 0) {
        // strengths in sorted order (gathered after the sort)
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) sv[pl][ch] = a.sstr[((int64_t)tr * a.M + pos) * NCH + ch];
#pragma unroll
        for (int x = 0; x < kTileX; ++x) {
          int dx = x - s;
          if (dx < 0) dx += a.nf[0];
          T wv = (T)0;
#pragma unroll
          for (int j = 0; j < W; ++j) wv = dx == j ? v[j] : wv;
          wxr[pl][x] = wv;
        }
      }
    }
    __syncthreads();
    if (sub < tpr) {
      for (int pl = sub; pl < cnt; pl += tpr) {
        // offset of this thread's row inside the point's support (cells (v + j) mod n_f, j < w)
        int dy = ly - vstart[pl][1];
        if (dy < 0) dy += a.nf[1];
        if (dy >= W) continue;
        T wyz = wts[pl][1][dy];
        if (DIM == 3) {
          int dz = lz - vstart[pl][2];
          if (dz < 0) dz += a.nf[2];
          if (dz >= W) continue;
          wyz *= wts[pl][2][dz];
        }
        T s[NCH];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) s[ch] = wyz * sv[pl][ch];
#pragma unroll
        for (int x = 0; x < kTileX; ++x) {
          const T wx = wxr[pl][x];
#pragma unroll
          for (int ch = 0; ch < NCH; ++ch) acc[x][ch] += wx * s[ch];
        }
      }
    }
    __syncthreads();
  }
  // fixed-order sum of the partial rows through LDS
  for (int sidx = 0; sidx < tpr; ++sidx) {
    if (sub == sidx) {
#pragma unroll
      for (int x = 0; x < kTileX; ++x)
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) accs[ch][row][x] = (sidx == 0 ? (T)0 : accs[ch][row][x]) + acc[x][ch];
    }
    __syncthreads();
  }
  if (nparts > 1) {  // one part of a split tile: partial tile to scratch, summed by k_merge_tiles
    T* dst = a.scratch + ((int64_t)tr * a.slots + a.tile_slot[tile_id] + part) * NCH * kMaxTileCells;
    for (int i = tid; i < tcells; i += kSpreadThreads) {
      const int lx = i % kTileX;
      const int rw = i / kTileX;
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) dst[ch * kMaxTileCells + i] = accs[ch][rw][lx];
    }
    return;
  }
  // write the tile once
  for (int i = tid; i < tcells; i += kSpreadThreads) {
    const int lx = i % kTileX;
    const int rw = i / kTileX;
    const int lyy = rw % a.tb[1];
    const int lzz = DIM == 3 ? rw / a.tb[1] : 0;
    const int gz = DIM == 3 ? base[2] + lzz : 0;
    const int64_t g = ((int64_t)gz * a.nf[1] + base[1] + lyy) * a.nf[0] + base[0] + lx;
    if (CPLX) {
      reinterpret_cast<cplx<T>*>(a.grid)[(int64_t)tr * cells + g] = mk(accs[0][rw][lx], accs[1][rw][lx]);
    } else {
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) a.grid[ch * cells + g] = accs[ch][rw][lx];
    }
  }
}

// Strengths permuted into the sorted point order, so that the spreading stages read them contiguously.
template <typename T, int NCH, bool CPLX>
__global__ void k_sort_strengths(int64_t M, const int* __restrict__ s_idx, const T* __restrict__ str,
                                 T* __restrict__ sstr) {
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= M) return;
  const int tr = blockIdx.y;
  const int64_t j = s_idx[pos];
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch)
    sstr[((int64_t)tr * M + pos) * NCH + ch] = CPLX ? str[((int64_t)tr * M + j) * 2 + ch] : str[j * NCH + ch];
}

// Points reaching each tile (its bin and the q bins before it per axis) and the parts it splits into.
__global__ void k_tile_parts(int dim, int nt0, int nt1, int nt2, int q0, int q1, int q2, const int* __restrict__ offsets,
                             int* __restrict__ tile_parts) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt0 * nt1 * nt2) return;
  const int tx = t % nt0, ty = (t / nt0) % nt1, tz = t / (nt0 * nt1);
  int total = 0;
  for (int dz = 0; dz <= (dim == 3 ? q2 : 0); ++dz)
    for (int dy = 0; dy <= q1; ++dy)
      for (int dx = 0; dx <= q0; ++dx) {
        const int bx = (tx - dx + nt0) % nt0, by = (ty - dy + nt1) % nt1, bz = dim == 3 ? (tz - dz + nt2) % nt2 : 0;
        const int b = bx + nt0 * (by + nt1 * bz);
        total += offsets[b + 1] - offsets[b];
      }
  tile_parts[t] = total <= kSplit ? 1 : (total + kSplit - 1) / kSplit;
}

// Work list (tile, part) in tile order, and scratch slots for tiles split into several parts.
__global__ void k_fill_work(int nbins, const int* __restrict__ part_off, const int* __restrict__ tile_parts,
                            int2* __restrict__ work, int* __restrict__ tile_slot, int* __restrict__ slot_ctr) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nbins) return;
  const int np = tile_parts[t], off = part_off[t];
  for (int q = 0; q < np; ++q) work[off + q] = make_int2(t, q);
  tile_slot[t] = np > 1 ? atomicAdd(slot_ctr, np) : -1;
}

// Sum the partial tiles of every split tile in part order and write it to the grid.
template <typename T, int DIM, int NCH, bool CPLX>
__global__ __launch_bounds__(kSpreadThreads) void k_merge_tiles(SpreadArgs<T> a) {
  const int t = blockIdx.x;
  const int np = a.tile_parts[t];
  if (np <= 1) return;
  const int tr = blockIdx.y;
  const int tcoord[3] = {t % a.nt[0], (t / a.nt[0]) % a.nt[1], DIM == 3 ? t / (a.nt[0] * a.nt[1]) : 0};
  const int rows = a.tb[1] * (DIM == 3 ? a.tb[2] : 1);
  const int64_t cells = (int64_t)a.nf[0] * a.nf[1] * (DIM == 3 ? a.nf[2] : 1);
  const T* src = a.scratch + ((int64_t)tr * a.slots + a.tile_slot[t]) * NCH * kMaxTileCells;
  for (int i = threadIdx.x; i < kTileX * rows; i += kSpreadThreads) {
    T v[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) v[ch] = (T)0;
    for (int q = 0; q < np; ++q)
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) v[ch] += src[((int64_t)q * NCH + ch) * kMaxTileCells + i];
    const int lx = i % kTileX, rw = i / kTileX;
    const int ly = rw % a.tb[1], lz = DIM == 3 ? rw / a.tb[1] : 0;
    const int gz = DIM == 3 ? tcoord[2] * a.tb[2] + lz : 0;
    const int64_t g = ((int64_t)gz * a.nf[1] + tcoord[1] * a.tb[1] + ly) * a.nf[0] + tcoord[0] * kTileX + lx;
    if (CPLX) {
      reinterpret_cast<cplx<T>*>(a.grid)[(int64_t)tr * cells + g] = mk(v[0], v[1]);
    } else {
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) a.grid[ch * cells + g] = v[ch];
    }
  }
}

template <typename T>
struct InterpArgs {
  const T* coef;
  int deg;
  const int* s_idx;
  const uint32_t* s_i0;
  const T* s_y;
  const T* grid;
  T* out;   // real: (M, nch); complex: (ntrans, M)
  int64_t M;
  int nf[3];
};

// Several lanes per point (kInterpLanes): each lane gathers a share of the point's w^(d-1) grid
// lines along x and the partial sums are combined with cross-lane shuffles.
template <int DIM>
__host__ __device__ constexpr int interp_lanes() { return DIM == 3 ? 16 : 4; }

template <typename T, int DIM, int W, int NCH, bool CPLX>
__global__ __launch_bounds__(256) void k_interp(InterpArgs<T> a) {
  constexpr int TPP = interp_lanes<DIM>();
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t pos = gid / TPP;
  const int lane = (int)(gid % TPP);
  const bool valid = pos < a.M;
  const int tr = blockIdx.y;
  T acc[NCH];
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) acc[ch] = (T)0;
  if (valid) {
    const uint32_t pk = a.s_i0[pos];
    T wx[W], wy[W], wz[W];
    kernel_values<T, W>(a.coef, a.deg, a.s_y[pos * DIM + 0], wx);
    kernel_values<T, W>(a.coef, a.deg, a.s_y[pos * DIM + 1], wy);
    if (DIM == 3) kernel_values<T, W>(a.coef, a.deg, a.s_y[pos * DIM + 2], wz);
    const int ix = unpack_i0<DIM>(pk, 0), iy = unpack_i0<DIM>(pk, 1), iz = DIM == 3 ? unpack_i0<DIM>(pk, 2) : 0;
    const int64_t cells = (int64_t)a.nf[0] * a.nf[1] * (DIM == 3 ? a.nf[2] : 1);
    constexpr int LINES = DIM == 3 ? W * W : W;
    for (int l = lane; l < LINES; l += TPP) {
      const int jy = l % W, jz = DIM == 3 ? l / W : 0;
      int y = iy + jy;
      if (y >= a.nf[1]) y -= a.nf[1];
      int z = iz + jz;
      if (DIM == 3 && z >= a.nf[2]) z -= a.nf[2];
      T wyz = wy[0], wzz = DIM == 3 ? wz[0] : (T)1;
#pragma unroll
      for (int j = 1; j < W; ++j) {
        wyz = jy == j ? wy[j] : wyz;
        if (DIM == 3) wzz = jz == j ? wz[j] : wzz;
      }
      wyz *= wzz;
      const int64_t row = ((int64_t)z * a.nf[1] + y) * a.nf[0];
      T racc[NCH];
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) racc[ch] = (T)0;
#pragma unroll
      for (int jx = 0; jx < W; ++jx) {
        int x = ix + jx;
        if (x >= a.nf[0]) x -= a.nf[0];
        if (CPLX) {
          const cplx<T> v = reinterpret_cast<const cplx<T>*>(a.grid)[(int64_t)tr * cells + row + x];
          racc[0] += wx[jx] * v.x;
          racc[1] += wx[jx] * v.y;
        } else {
#pragma unroll
          for (int ch = 0; ch < NCH; ++ch) racc[ch] += wx[jx] * a.grid[ch * cells + row + x];
        }
      }
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) acc[ch] += wyz * racc[ch];
    }
  }
  // combine the lanes of each point (TPP consecutive lanes of one wavefront)
#pragma unroll
  for (int off = TPP / 2; off > 0; off >>= 1)
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) acc[ch] += __shfl_xor(acc[ch], off, TPP);
  if (valid && lane == 0) {
    const int64_t j = a.s_idx[pos];
    if (CPLX) {
      a.out[((int64_t)tr * a.M + j) * 2 + 0] = acc[0];
      a.out[((int64_t)tr * a.M + j) * 2 + 1] = acc[1];
    } else {
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) a.out[j * NCH + ch] = acc[ch];
    }
  }
}

// ---- dispatch over (precision, dim, w, channels) ----
template <typename T, int DIM, int NCH, bool CPLX, int W>
static hipError_t run_spread(Plan& p, int64_t M, const void* str, int ntr, hipStream_t st) {
  SpreadArgs<T> a;
  a.coef = (const T*)p.coef;
  a.deg = p.deg;
  a.offsets = p.offsets;
  a.s_idx = p.s_idx;
  a.s_i0 = p.s_i0;
  a.s_y = (const T*)p.s_y;
  a.str = (const T*)str;
  a.grid = (T*)p.grid;
  a.M = M;
  for (int d = 0; d < 3; ++d) {
    a.nf[d] = (int)p.nf[d];
    a.tb[d] = (int)p.tb[d];
    a.nt[d] = (int)p.nt[d];
    a.q[d] = (int)p.qn[d];
  }
  a.part_off = p.part_off;
  a.work = (const int2*)p.work;
  a.tile_parts = p.tile_parts;
  a.tile_slot = p.tile_slot;
  a.scratch = (T*)p.split_scratch;
  a.slots = p.split_slots;
  a.rowmask = p.rowmask;
  a.sstr = (T*)p.s_str;
  const unsigned nb = (unsigned)p.nbins;
  if (M > 0) {
    hipLaunchKernelGGL((k_sort_strengths<T, NCH, CPLX>), dim3((unsigned)((M + 255) / 256), (unsigned)ntr), dim3(256), 0,
                       st, M, (const int*)p.s_idx, (const T*)str, a.sstr);
    hipError_t e0 = hipGetLastError();
    if (e0 != hipSuccess) return e0;
  }
  hipLaunchKernelGGL(k_tile_parts, dim3((nb + 255) / 256), dim3(256), 0, st, DIM, a.nt[0], a.nt[1], a.nt[2], a.q[0],
                     a.q[1], a.q[2], (const int*)p.offsets, p.tile_parts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_scan(p.nbins, p.tile_parts, p.part_off, p.scan_part, st)) != hipSuccess) return e;
  if ((e = launch_fill_zero(p.slot_ctr, 4, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_fill_work, dim3((nb + 255) / 256), dim3(256), 0, st, (int)p.nbins, (const int*)p.part_off,
                     (const int*)p.tile_parts, (int2*)p.work, p.tile_slot, p.slot_ctr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const bool prof = prof_on(p, PROF_SPREAD);
  if (prof) prof_start(p, st);
  hipLaunchKernelGGL((k_spread<T, DIM, W, NCH, CPLX>), dim3((unsigned)p.work_blocks, (unsigned)ntr),
                     dim3(kSpreadThreads), 0, st, a);
  // algorithmic bytes: the grid written once, per point its sorted record and its strengths read
  if (prof)
    prof_stop(p, (double)ntr * p.fine_cells() * NCH * sizeof(T) + (double)M * (8 + DIM * sizeof(T)) +
                     (double)ntr * M * NCH * sizeof(T), st);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((k_merge_tiles<T, DIM, NCH, CPLX>), dim3(nb, (unsigned)ntr), dim3(kSpreadThreads), 0, st, a);
  return hipGetLastError();
}

template <typename T, int DIM, int NCH, bool CPLX, int W>
static hipError_t run_interp(Plan& p, int64_t M, void* out, int ntr, hipStream_t st) {
  InterpArgs<T> a;
  a.coef = (const T*)p.coef;
  a.deg = p.deg;
  a.s_idx = p.s_idx;
  a.s_i0 = p.s_i0;
  a.s_y = (const T*)p.s_y;
  a.grid = (const T*)p.grid;
  a.out = (T*)out;
  a.M = M;
  for (int d = 0; d < 3; ++d) a.nf[d] = (int)p.nf[d];
  if (M == 0) return hipSuccess;
  const bool prof = prof_on(p, PROF_INTERP);
  if (prof) prof_start(p, st);
  const int64_t threads = M * interp_lanes<DIM>();
  hipLaunchKernelGGL((k_interp<T, DIM, W, NCH, CPLX>), dim3((unsigned)((threads + 255) / 256), (unsigned)ntr),
                     dim3(256), 0, st, a);
  // algorithmic bytes: per point its sorted record, w^d grid cells per channel, the result
  if (prof) {
    double cellsper = 1;
    for (int d = 0; d < DIM; ++d) cellsper *= W;
    prof_stop(p, (double)M * (8 + DIM * sizeof(T)) + (double)ntr * M * (cellsper + 1) * NCH * sizeof(T), st);
  }
  return hipGetLastError();
}

#define FSIB_W_SWITCH(W_, CALL)                                     \
  switch (W_) {                                                     \
    case 2: return CALL(2);                                         \
    case 3: return CALL(3);                                         \
    case 4: return CALL(4);                                         \
    case 5: return CALL(5);                                         \
    case 6: return CALL(6);                                         \
    case 7: return CALL(7);                                         \
    case 8: return CALL(8);                                         \
    case 9: return CALL(9);                                         \
    case 10: return CALL(10);                                       \
    case 11: return CALL(11);                                       \
    case 12: return CALL(12);                                       \
    case 13: return CALL(13);                                       \
    case 14: return CALL(14);                                       \
    case 15: return CALL(15);                                       \
    case 16: return CALL(16);                                       \
    default: return hipErrorInvalidValue;                           \
  }

template <typename T, int DIM, int NCH, bool CPLX>
static hipError_t spread_dispatch(Plan& p, int64_t M, const void* str, int ntr, hipStream_t st) {
#define CALL_S(w) run_spread<T, DIM, NCH, CPLX, w>(p, M, str, ntr, st)
  FSIB_W_SWITCH(p.w, CALL_S)
#undef CALL_S
}

template <typename T, int DIM, int NCH, bool CPLX>
static hipError_t interp_dispatch(Plan& p, int64_t M, void* out, int ntr, hipStream_t st) {
#define CALL_I(w) run_interp<T, DIM, NCH, CPLX, w>(p, M, out, ntr, st)
  FSIB_W_SWITCH(p.w, CALL_I)
#undef CALL_I
}

// real_comps > 0: real vector strengths with dim components; 0: complex, p.ntrans transforms.
// The point set is the one last sorted by launch_sort_points.
hipError_t launch_spread(Plan& p, int64_t M, const void* str, int real_comps, hipStream_t st) {
  const bool f64 = p.prec == FSIB_F64;
  if (real_comps == 0) {
    if (p.dim == 2)
      return f64 ? spread_dispatch<double, 2, 2, true>(p, M, str, p.ntrans, st)
                 : spread_dispatch<float, 2, 2, true>(p, M, str, p.ntrans, st);
    return f64 ? spread_dispatch<double, 3, 2, true>(p, M, str, p.ntrans, st)
               : spread_dispatch<float, 3, 2, true>(p, M, str, p.ntrans, st);
  }
  if (p.dim == 2)
    return f64 ? spread_dispatch<double, 2, 2, false>(p, M, str, 1, st)
               : spread_dispatch<float, 2, 2, false>(p, M, str, 1, st);
  return f64 ? spread_dispatch<double, 3, 3, false>(p, M, str, 1, st)
             : spread_dispatch<float, 3, 3, false>(p, M, str, 1, st);
}

hipError_t launch_interp(Plan& p, int64_t M, void* out, int real_comps, hipStream_t st) {
  const bool f64 = p.prec == FSIB_F64;
  if (real_comps == 0) {
    if (p.dim == 2)
      return f64 ? interp_dispatch<double, 2, 2, true>(p, M, out, p.ntrans, st)
                 : interp_dispatch<float, 2, 2, true>(p, M, out, p.ntrans, st);
    return f64 ? interp_dispatch<double, 3, 2, true>(p, M, out, p.ntrans, st)
               : interp_dispatch<float, 3, 2, true>(p, M, out, p.ntrans, st);
  }
  if (p.dim == 2)
    return f64 ? interp_dispatch<double, 2, 2, false>(p, M, out, 1, st)
               : interp_dispatch<float, 2, 2, false>(p, M, out, 1, st);
  return f64 ? interp_dispatch<double, 3, 3, false>(p, M, out, 1, st)
             : interp_dispatch<float, 3, 3, false>(p, M, out, 1, st);
}

}  // namespace fsib
