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
#include "bins.hpp"
#include "plan.hpp"

namespace fsib {

constexpr int kSpreadThreads = 256;  // the most threads of a spreading workgroup
// Threads of a spreading workgroup: 256 for 3D tiles (16 x 8 x 8); for 2D tiles (16 x 16) 64 in FP32,
// so that a lane owns 4 cells of a row as in 3D (with 256 threads a 2D lane owns one cell and spends
// most of each point on the bit scan and addressing of the walk: 2D batch +8%), and 128 in FP64 (2
// cells per lane: 21 KiB of LDS per one-wave workgroup would leave too few waves per CU; +2% against
// 256).
template <int DIM, typename T>
__host__ __device__ constexpr int spread_threads() { return DIM == 3 ? 256 : (sizeof(T) == 8 ? 128 : 64); }
constexpr int kChunk = 64;           // points staged per round
constexpr int kMaxTileCells = 1024;  // cells of one tile
constexpr int kTileX = 16;           // tile extent along x (one register row per thread)


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
  // work list: entry e = (t, q), q >= 1: workgroup nbins + e spreads candidates [q*split, (q+1)*split) of tile t
  const int* nwork;     // the number of work list entries (the further parts)
  const int2* work;     // (t, q) per part
  const int* tile_parts;
  const int* tile_slot; // first scratch slot of a split tile
  T* scratch;           // split tiles: [ntrans][slots][NCH][kMaxTileCells] partial tiles
  int64_t slots;        // scratch slots per transform
  const int* split_list;  // the split tiles, split_cnt[0] of them (written with the work list)
  const int* split_cnt;
  const uint8_t* rowmask;  // blocks of x lines reached by some point (lines elsewhere stay unwritten)
  int xcd_chunk;           // > 0: workgroups renumbered in runs of this many per XCD (xcd_chunked)
  int split;               // candidates per part of a heavy tile
  int ninst;               // instances: tile t of the whole plan is tile t % nbins of instance t / nbins,
                           // whose real grids follow one another ([inst][ch][cells])
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

// Degree of the kernel pieces for width W (choose_degree), known at compile time: the Horner loops
// unroll, and interpolation lanes keep only the W + 3 coefficients of their column in registers.
template <int W>
__host__ __device__ constexpr int interp_degree() { return W + 2 < kMaxDeg ? W + 2 : kMaxDeg; }

template <int DIM>
__device__ __forceinline__ int unpack_i0(uint32_t p, int a) {
  return DIM == 3 ? (int)((p >> (10 * a)) & 1023u) : (int)((p >> (16 * a)) & 65535u);
}

// Coverage bits of tile coordinates [0, L) by the cells [a, a + W) (a may be negative or past L).
template <int W, int L>
__device__ __forceinline__ uint32_t run_bits(int a) {
  static_assert(W <= 16 && L <= 16, "coverage bits fit 32 bits");
  if (a >= L || a + W <= 0) return 0u;
  const uint32_t m = (1u << W) - 1u;
  const uint32_t r = a >= 0 ? (m << a) : (m >> (-a));
  return r & ((1u << L) - 1u);
}

// One staging lane per point along one axis: the point's W kernel values v expanded over the tile's
// L coordinates of the axis (zero outside the support; the support starts st cells after the tile,
// modulo nfd), and one 64-bit set per group of GW coordinates of the staged points covering it:
// coordinate c is covered when (c - st) mod nfd < W, i.e. it lies in [st, st + W) or in the wrapped
// run [st - nfd, st - nfd + W).  Lane 0 writes the sets.
template <typename T, int W, int L, int GW>
__device__ __forceinline__ void stage_axis(bool valid, int st, int nfd, const T* v, T* rowp,
                                           unsigned long long* mskp, int lane) {
  uint32_t bits = 0u;
  if (valid) {
    bits = run_bits<W, L>(st) | run_bits<W, L>(st - nfd);
#pragma unroll
    for (int c = 0; c < L; ++c) rowp[c] = (T)0;
#pragma unroll
    for (int j = 0; j < W; ++j) {
      int c = st + j;
      if (c >= nfd) c -= nfd;
      if (c < L) rowp[c] = v[j];
    }
  }
  constexpr int NG = L / GW;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const unsigned long long b = __ballot(((bits >> (g * GW)) & ((1u << GW) - 1u)) != 0u);
    if (lane == 0) mskp[g] = b;
  }
}

// NCH channels per point: real vector strengths (NCH = components, planar grids) or one complex
// strength (NCH = 2, interleaved complex grid, transform index = blockIdx.y).
//
// Inside a tile every lane owns CW consecutive cells of one row along x (3D: 64 rows x 4 groups of
// 4 cells; 2D FP32: 16 rows x 4 groups of 4 cells on 64 threads; 2D FP64: 16 rows x 8 groups of 2
// cells on 128 threads) and accumulates them in registers.  The tile's points are staged 64 at a time, the
// wavefronts taking the axes in turn with one lane per point: the lane evaluates the point's w
// kernel values along the axis (Horner), writes them expanded over the tile's coordinates of that
// axis (zero outside the support), and one ballot per coordinate group gives the 64-bit set of
// staged points whose support covers it.  A lane's points are the AND of the sets of
// its row's y and z and of its x group; every lane walks its own set, lowest point first, so lanes
// stay busy with different points and no lane visits a point that misses its cells.  Each cell is
// summed by one lane in point order (deterministic for a given sorted order), no atomics, and each
// lane writes its cells once.
//
// Workgroup b < nbins spreads (the first part of) tile b; workgroups past nbins take the further
// parts of heavy tiles from the work list.
template <typename T, int DIM, int NT_>
struct SpreadTile {
  static constexpr int TY = DIM == 3 ? 8 : 16;               // tile rows along y
  static constexpr int TZ = DIM == 3 ? 8 : 1;                // tile rows along z
  static constexpr int ROWS = TY * TZ;
  static constexpr int NT = NT_;                             // threads of the workgroup
  static constexpr int CW = kTileX * ROWS / NT;              // cells per lane along x
  static constexpr int NXG = kTileX / CW;                    // x groups
  static constexpr int XS = kTileX + (sizeof(T) == 4 ? 4 : 2);  // padded LDS strides
  static constexpr int YS = TY + 1;
  static constexpr int ZS = TZ + 1;
  static constexpr int NMASK = TY + (DIM == 3 ? TZ : 0) + NXG;
};

template <typename T, int DIM, int W, int NCH, bool CPLX, int NT>
__device__ __forceinline__ void spread_body(const SpreadArgs<T>& a, Blk wb) {
  using G = SpreadTile<T, DIM, NT>;
  static_assert(NT >= 64 && NT <= kSpreadThreads && kTileX * G::ROWS % NT == 0, "threads of a spreading tile");
  constexpr int TY = G::TY, TZ = G::TZ, ROWS = G::ROWS, CW = G::CW, NXG = G::NXG;
  __shared__ T wxr[kChunk][G::XS];
  __shared__ T wyr[kChunk][G::YS];
  __shared__ T wzr[DIM == 3 ? kChunk : 1][G::ZS];
  __shared__ T sv[kChunk][NCH];
  __shared__ T cf[(kMaxDeg + 1) * W];
  __shared__ unsigned long long msk[G::NMASK];
  __shared__ int rbeg[27], rlen[27];
  __shared__ int nrange;
  __shared__ int sel[kSpreadThreads];  // candidates of the current window whose support meets the tile
  __shared__ int wcnt[kSpreadThreads / 64 + 1];

  const int tid = threadIdx.x;
  const int tr = (int)wb.y;
  const int nbins = a.nt[0] * a.nt[1] * (DIM == 3 ? a.nt[2] : 1);
  const int nbt = nbins * a.ninst;  // tiles of all instances
  int tile_id, part;
  // tiles holding points cluster (surfaces): whole XCD-contiguous ranges of tiles would load the XCDs
  // unevenly, short runs keep neighbouring tiles (which stage the same points) on one L2
  const int blk = a.xcd_chunk > 0 ? (int)xcd_chunked(wb.x, wb.nx, a.xcd_chunk) : (int)wb.x;
  if (blk < nbt) {
    tile_id = blk;
    part = 0;
  } else {
    const int e = blk - nbt;
    if (e >= a.nwork[0]) return;  // beyond the further parts
    const int2 wk = a.work[e];
    tile_id = wk.x;
    part = wk.y;
  }
  const int inst = tile_id / nbins, lt = tile_id - inst * nbins;  // instance, tile within it
  int tcoord[3];
  tcoord[0] = lt % a.nt[0];
  tcoord[1] = (lt / a.nt[0]) % a.nt[1];
  tcoord[2] = DIM == 3 ? lt / (a.nt[0] * a.nt[1]) : 0;
  // no point reaches this tile's block of x lines: those lines are neither read nor written
  if (a.rowmask && !a.rowmask[(int64_t)inst * a.nt[1] * a.nt[2] + tcoord[2] * a.nt[1] + tcoord[1]]) return;
  const int nparts = a.tile_parts[tile_id];
  constexpr int tcells = kTileX * ROWS;
  int base[3] = {0, 0, 0};
  base[0] = tcoord[0] * kTileX;
  base[1] = tcoord[1] * TY;
  if (DIM == 3) base[2] = tcoord[2] * TZ;
  const int64_t cells = (int64_t)a.nf[0] * a.nf[1] * (DIM == 3 ? a.nf[2] : 1);
  // bins that can reach this tile: this one and up to q before it along each axis, read in parallel
  {
    const int qx = a.q[0] + 1, qy = a.q[1] + 1, qz = DIM == 3 ? a.q[2] + 1 : 1;
    if (tid < qx * qy * qz) {
      const int dx = tid % qx, dy = (tid / qx) % qy, dz = tid / (qx * qy);
      const int bx = (tcoord[0] - dx + a.nt[0]) % a.nt[0];
      const int by = (tcoord[1] - dy + a.nt[1]) % a.nt[1];
      const int bz = DIM == 3 ? (tcoord[2] - dz + a.nt[2]) % a.nt[2] : 0;
      const int b = bx + a.nt[0] * (by + a.nt[1] * bz) + inst * nbins;
      const int s0 = a.offsets[b], e0 = a.offsets[b + 1];
      rbeg[tid] = s0;
      rlen[tid] = e0 - s0;
    }
    for (int i = tid; i < (a.deg + 1) * W; i += G::NT) cf[i] = a.coef[i];
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
  const int cbeg = part * a.split;
  const int cend = total < cbeg + a.split ? total : cbeg + a.split;
  const int row = tid % ROWS, xg = tid / ROWS;
  const int ly = row % TY, lz = DIM == 3 ? row / TY : 0;
  const int lane = tid & 63, wave = tid >> 6;
  T acc[CW][NCH];
#pragma unroll
  for (int c = 0; c < CW; ++c)
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) acc[c][ch] = (T)0;

  // Candidates are taken G::NT at a time: each thread tests one (support meets the tile
  // along every axis, from the packed first cell alone) and the hits are compacted, in order, into
  // sel[]; only those are staged, kChunk at a time.  (With the reach of ceil((w-1)/tile) bins per
  // axis, about half of the candidates miss the tile.)
  for (int w0 = cbeg; w0 < cend; w0 += G::NT) {
  {
    const int ci = w0 + tid;
    bool hit = false;
    int cpos = 0;
    if (ci < cend) {
      int vi = ci, r = 0;
      while (vi >= rlen[r]) vi -= rlen[r++];
      cpos = rbeg[r] + vi;
      const uint32_t pk = a.s_i0[cpos];
      hit = true;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const int L = d == 0 ? kTileX : (d == 1 ? TY : TZ);
        int st = unpack_i0<DIM>(pk, d) - base[d];
        if (st < 0) st += a.nf[d];
        hit = hit && (st < L || st + W > a.nf[d]);  // starts inside, or wraps round into the tile
      }
    }
    const unsigned long long hb = __ballot(hit);
    const int before = __popcll(hb & ((1ull << lane) - 1ull));
    if (lane == 0) wcnt[wave] = __popcll(hb);
    __syncthreads();
    int wbase = 0, nsel = 0;
    for (int v = 0; v < G::NT / 64; ++v) {
      if (v < wave) wbase += wcnt[v];
      nsel += wcnt[v];
    }
    if (hit) sel[wbase + before] = cpos;
    if (tid == 0) wcnt[G::NT / 64] = nsel;
    __syncthreads();
  }
  const int nsel = wcnt[G::NT / 64];
  for (int c0 = 0; c0 < nsel; c0 += kChunk) {
    const int cnt = nsel - c0 < kChunk ? nsel - c0 : kChunk;
    // (1) the wavefronts take the axes d in turn (3D: one each), lane = point; then one wavefront (3D:
    // the fourth, 2D: the only one) the strengths
    {
      const int pl = lane;
      const bool valid = pl < cnt;
      const int64_t pos = valid ? (int64_t)sel[c0 + pl] : 0;
      constexpr int NW = G::NT / 64;
      for (int d = wave; d < DIM; d += NW) {
        const int nfd = a.nf[d];
        int st = 0;
        T v[W];
        if (valid) {
          const T y = a.s_y[pos * DIM + d];
          // runtime degree: a fully unrolled Horner loop here lifts the kernel's VGPRs (68 -> 105 in FP32)
#pragma unroll
          for (int j = 0; j < W; ++j) v[j] = cf[a.deg * W + j];
          for (int i = a.deg - 1; i >= 0; --i) {
#pragma unroll
            for (int j = 0; j < W; ++j) v[j] = v[j] * y + cf[i * W + j];
          }
          st = unpack_i0<DIM>(a.s_i0[pos], d) - base[d];  // support start relative to the tile
          if (st < 0) st += nfd;
        }
        // kernel values expanded over the tile's coordinates along d and the coverage sets
        if (d == 0)
          stage_axis<T, W, kTileX, CW>(valid, st, nfd, v, &wxr[pl][0], &msk[TY + (DIM == 3 ? TZ : 0)], lane);
        else if (d == 1)
          stage_axis<T, W, TY, 1>(valid, st, nfd, v, &wyr[pl][0], &msk[0], lane);
        else
          stage_axis<T, W, TZ, 1>(valid, st, nfd, v, &wzr[DIM == 3 ? pl : 0][0], &msk[TY], lane);
      }
      if (wave == (DIM < NW ? DIM : 0) && valid) {
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) sv[pl][ch] = a.sstr[((int64_t)tr * a.M + pos) * NCH + ch];
      }
    }
    __syncthreads();
    // (2) every lane walks the staged points that cover its cells
    unsigned long long m = msk[ly] & msk[TY + (DIM == 3 ? TZ : 0) + xg];
    if (DIM == 3) m &= msk[TY + lz];
    // the set in two 32-bit halves, lowest point first (32-bit bit scans are cheaper)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      uint32_t mm = (uint32_t)(m >> (32 * h));
      while (mm) {
        const int pl = 32 * h + __ffs(mm) - 1;
        mm &= mm - 1u;
        T wyz = wyr[pl][ly];
        if (DIM == 3) wyz *= wzr[DIM == 3 ? pl : 0][lz];
        T sw[NCH];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) sw[ch] = sv[pl][ch] * wyz;
#pragma unroll
        for (int c = 0; c < CW; ++c) {
          const T wx = wxr[pl][xg * CW + c];
#pragma unroll
          for (int ch = 0; ch < NCH; ++ch) acc[c][ch] += wx * sw[ch];
        }
      }
    }
    __syncthreads();
  }
  }
  // each lane writes its CW cells (zeros when no point reaches the tile but some reach its lines)
  if (nparts > 1) {  // one part of a split tile: partial tile to scratch, summed by k_merge_tiles
    T* dst = a.scratch + ((int64_t)tr * a.slots + a.tile_slot[tile_id] + part) * NCH * kMaxTileCells;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
      for (int c = 0; c < CW; ++c) dst[ch * kMaxTileCells + row * kTileX + xg * CW + c] = acc[c][ch];
    return;
  }
  const int gz = DIM == 3 ? base[2] + lz : 0;
  const int64_t g = ((int64_t)gz * a.nf[1] + base[1] + ly) * a.nf[0] + base[0] + xg * CW;
  if (CPLX) {
    cplx<T>* dst = reinterpret_cast<cplx<T>*>(a.grid) + (int64_t)tr * cells + g;
#pragma unroll
    for (int c = 0; c < CW; ++c) dst[c] = mk(acc[c][0], acc[c][1]);
  } else {
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
      for (int c = 0; c < CW; ++c) a.grid[((int64_t)inst * NCH + ch) * cells + g + c] = acc[c][ch];
  }
  (void)tcells;
}

template <typename T, int DIM, int W, int NCH, bool CPLX, int NT>
__global__ __launch_bounds__(kSpreadThreads) void k_spread(SpreadArgs<T> a) {
  spread_body<T, DIM, W, NCH, CPLX, NT>(a, launch_blk());
}
template <typename T, int DIM, int W, int NCH, bool CPLX, int NT>
__global__ __launch_bounds__(kSpreadThreads) void k_spread_parts(Parts<SpreadArgs<T>> f) {
  Blk b;
  const int g = part_blk(f, b);
  if (g >= 0) spread_body<T, DIM, W, NCH, CPLX, NT>(f.a[g], b);
}

// Threads per tile of a plan's spreading launches (its spread_threads knob, else the default).
template <int DIM, typename T>
static int plan_spread_threads(const Plan& p) {
  return DIM == 2 && p.spread_threads > 0 ? p.spread_threads : spread_threads<DIM, T>();
}

// Strengths permuted into the sorted point order, so that the spreading stages read them contiguously.
template <typename T>
struct SortStrArgs {
  int64_t M;
  const int* s_idx;
  const T* str;
  T* sstr;
};
template <typename T, int NCH, bool CPLX>
__device__ __forceinline__ void sort_strengths(const SortStrArgs<T>& A, Blk wb) {
  const int64_t M = A.M;
  const int64_t pos = wb.x * blockDim.x + threadIdx.x;
  if (pos >= M) return;
  const int64_t tr = wb.y;
  const int64_t j = A.s_idx[pos];
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch)
    A.sstr[(tr * M + pos) * NCH + ch] = CPLX ? A.str[(tr * M + j) * 2 + ch] : A.str[j * NCH + ch];
}
template <typename T, int NCH, bool CPLX>
__global__ void k_sort_strengths(SortStrArgs<T> a) { sort_strengths<T, NCH, CPLX>(a, launch_blk()); }
template <typename T, int NCH, bool CPLX>
__global__ void k_sort_strengths_parts(Parts<SortStrArgs<T>> f) {
  Blk b;
  const int g = part_blk(f, b);
  if (g >= 0) sort_strengths<T, NCH, CPLX>(f.a[g], b);
}

__device__ __forceinline__ void tile_parts_body(const TilePartsArgs& A, Blk wb) {
  tile_parts_at(A, (int)(wb.x * blockDim.x + threadIdx.x));
}
__global__ void k_tile_parts(TilePartsArgs a) { tile_parts_body(a, launch_blk()); }
__global__ void k_tile_parts_parts(Parts<TilePartsArgs> f) {
  Blk b;
  const int g = part_blk(f, b);
  if (g >= 0) tile_parts_body(f.a[g], b);
}



// Sum the partial tiles of every split tile in part order and write it to the grid: workgroup k takes
// entry k of the list of split tiles (launched over a bound on their number; the workgroups past the
// count leave at once).  The list's order does not matter: each tile is summed on its own.
// Workgroups per split tile: one per 256 cells (3D tiles have 1024), so that the sums over the parts
// of one crowded tile run in parallel.
template <int DIM>
__host__ __device__ constexpr int merge_chunks() { return DIM == 3 ? 4 : 1; }

template <typename T, int DIM, int NCH, bool CPLX>
__device__ __forceinline__ void merge_one_tile(const SpreadArgs<T>& a, int t, int np, int tr, int chunk);

template <typename T, int DIM, int NCH, bool CPLX>
__device__ __forceinline__ void merge_tiles(const SpreadArgs<T>& a, Blk wb) {
  constexpr int MC = merge_chunks<DIM>();
  const int64_t k = wb.x / MC;
  if (k >= a.split_cnt[0]) return;
  const int t = a.split_list[k];
  merge_one_tile<T, DIM, NCH, CPLX>(a, t, a.tile_parts[t], (int)wb.y, (int)(wb.x - k * MC));
}

template <typename T, int DIM, int NCH, bool CPLX>
__device__ __forceinline__ void merge_one_tile(const SpreadArgs<T>& a, int t, int np, int tr, int chunk) {
  constexpr int MC = merge_chunks<DIM>();
  const int nbins = a.nt[0] * a.nt[1] * (DIM == 3 ? a.nt[2] : 1);
  const int inst = t / nbins, lt = t - inst * nbins;
  const int tcoord[3] = {lt % a.nt[0], (lt / a.nt[0]) % a.nt[1], DIM == 3 ? lt / (a.nt[0] * a.nt[1]) : 0};
  const int rows = a.tb[1] * (DIM == 3 ? a.tb[2] : 1);
  const int64_t cells = (int64_t)a.nf[0] * a.nf[1] * (DIM == 3 ? a.nf[2] : 1);
  const T* src = a.scratch + ((int64_t)tr * a.slots + a.tile_slot[t]) * NCH * kMaxTileCells;
  const int per = kTileX * rows / MC;  // cells of this workgroup's chunk
  for (int i = chunk * per + threadIdx.x; i < (chunk + 1) * per; i += kSpreadThreads) {
    T v[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) v[ch] = (T)0;
    // the partial tiles in part order, eight loads in flight at a time (a crowded tile has tens of
    // parts, and one load after another left the merge waiting on memory)
    int q = 0;
    for (; q + 8 <= np; q += 8) {
      T l[8][NCH];
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) l[u][ch] = src[((int64_t)(q + u) * NCH + ch) * kMaxTileCells + i];
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) v[ch] += l[u][ch];
    }
    for (; q < np; ++q)
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
      for (int ch = 0; ch < NCH; ++ch) a.grid[((int64_t)inst * NCH + ch) * cells + g] = v[ch];
    }
  }
}
template <typename T, int DIM, int NCH, bool CPLX>
__global__ __launch_bounds__(kSpreadThreads) void k_merge_tiles(SpreadArgs<T> a) {
  merge_tiles<T, DIM, NCH, CPLX>(a, launch_blk());
}
template <typename T, int DIM, int NCH, bool CPLX>
__global__ __launch_bounds__(kSpreadThreads) void k_merge_tiles_parts(Parts<SpreadArgs<T>> f) {
  Blk b;
  const int g = part_blk(f, b);
  if (g >= 0) merge_tiles<T, DIM, NCH, CPLX>(f.a[g], b);
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
  int xcd_chunk;  // > 0: workgroups renumbered in runs of this many per XCD (xcd_chunked)
  int ppw;        // points per wavefront (a multiple of the points summed together)
  // instances (ninst > 1): sorted positions [offsets[i nbins], offsets[(i+1) nbins]) belong to
  // instance i, whose real grids start at channel i * NCH
  const int* offsets;
  int nbins;
  int ninst;
  // real strengths only, nullable: also move the points, move[j * NCH + c] = move_in[j * NCH + c] +
  // move_a * out[j * NCH + c] (the velocity as stored), so a position update needs no pass of its own
  double* move;
  const double* move_in;
  double move_a;
};

// Instance of sorted position pos: the last i with offsets[i * nbins] <= pos.
__device__ __forceinline__ int sorted_instance(const int* __restrict__ offsets, int nbins, int ninst, int64_t pos) {
  int lo = 0, hi = ninst;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (offsets[(int64_t)mid * nbins] <= pos) lo = mid;
    else hi = mid;
  }
  return lo;
}

// One wavefront per point (a few points at a time).  The lanes cover an XL x YL patch of the
// point's support in one z-plane (XL >= w lanes along x, YL = 64/XL along y), so one load
// instruction reads YL short runs of consecutive cells; the planes jz = 0..w-1 (and, when w > YL,
// the chunks of YL rows) are walked in turn.  Lanes 16a + j (axis a, j < w) evaluate the kernel value
// j along axis a (Horner, with the coefficient column j held in registers); every lane takes its x
// and y values by lane permute and the plane's z value by readlane.  The wavefront sum is a
// butterfly reduction.  Consecutive sorted points go to the same wavefront, so their shared cells
// hit in the L1 cache, and the next group of points' records is loaded one group ahead.

// Lane permutes and readlanes run with every lane of the wavefront active: the source lane of a
// permute must be active for its value to be read.
template <typename T>
__device__ __forceinline__ T lane_value(T v, int src) {
  if constexpr (sizeof(T) == 4) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
  } else {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(u & 0xffffffffll));
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(u >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
  }
}
template <typename T>
__device__ __forceinline__ T uniform_lane_value(T v, int src) {
  if constexpr (sizeof(T) == 4) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
  } else {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
  }
}

// x lanes per row: the power of two >= w, unless a narrower row (xl < 16) lets the 64 lanes cover the
// w rows of a plane in fewer chunks (w = 9, 10: rows of 9 or 10 lanes, 7 or 6 rows per chunk, two
// chunks instead of three).  Lanes past the last whole row (yl >= YL) stay idle.
template <int W>
__host__ __device__ constexpr int interp_xlanes() {
  constexpr int p2 = W <= 2 ? 2 : (W <= 4 ? 4 : (W <= 8 ? 8 : 16));
  int best = p2, cost = (W + 64 / p2 - 1) / (64 / p2);
  for (int xl = W; xl < p2; ++xl) {
    const int c = (W + 64 / xl - 1) / (64 / xl);
    if (c < cost) {
      cost = c;
      best = xl;
    }
  }
  return best;
}

// Points whose cells one wavefront sums together (by the registers one point's cells take).
template <typename T, int DIM, int W, int NCH, bool CPLX>
__host__ __device__ constexpr int interp_pb() {
  constexpr int YCH = (W + 64 / interp_xlanes<W>() - 1) / (64 / interp_xlanes<W>());
  constexpr int RPP = YCH * (DIM == 3 ? W : 1) * (CPLX ? 2 : NCH) * (int)sizeof(T) / 4;
  return RPP <= 16 ? 4 : (RPP <= 32 ? 2 : 1);
}

template <typename T, int DIM, int W, int NCH, bool CPLX>
__device__ __forceinline__ void interp_body(const InterpArgs<T>& a, Blk wb) {
  constexpr int XL = interp_xlanes<W>();
  constexpr int YL = 64 / XL;
  constexpr int YCH = (W + YL - 1) / YL;  // chunks of YL rows along y
  constexpr int NZ = DIM == 3 ? W : 1;
  constexpr int SC = CPLX ? 2 : NCH;
  constexpr int RPP = YCH * NZ * SC * (int)sizeof(T) / 4;  // registers of one point's cells
  constexpr int PB = interp_pb<T, DIM, W, NCH, CPLX>();       // points summed together
  static_assert(PB == (RPP <= 16 ? 4 : (RPP <= 32 ? 2 : 1)), "interp_pb matches the kernel");
  constexpr int GMAX = (PB == 1 ? 32 : 64) / (PB * SC * (int)sizeof(T) / 4);
  constexpr int G = NZ < GMAX ? NZ : GMAX;                  // planes loaded together
  const int lane = threadIdx.x & 63;
  const int xl = lane % XL, yl = lane / XL;
  const int axis = lane >> 4, jk = lane & 15;  // kernel value jk along axis (lanes 16a + j)
  const int tr = (int)wb.y;
  const int64_t cells = (int64_t)a.nf[0] * a.nf[1] * (DIM == 3 ? a.nf[2] : 1);
  // coefficient column jk of the kernel pieces
  constexpr int DEG = interp_degree<W>();  // the plan's degree for this width (checked on the host)
  T cfr[DEG + 1];
#pragma unroll
  for (int i = 0; i <= DEG; ++i) cfr[i] = jk < W ? a.coef[i * W + jk] : (T)0;
  const int64_t blk = a.xcd_chunk > 0 ? xcd_chunked(wb.x, wb.nx, a.xcd_chunk) : wb.x;
  const int64_t wave = (blk * blockDim.x + threadIdx.x) >> 6;
  const int64_t first = wave * a.ppw;
  uint32_t pkn[PB];
  T yn[PB];
  auto records = [&](int k0) {
#pragma unroll
    for (int b = 0; b < PB; ++b) {
      int64_t pq = first + k0 + b;
      if (pq >= a.M) pq = a.M - 1;
      pkn[b] = a.s_i0[pq];
      yn[b] = a.s_y[pq * DIM + (axis < DIM ? axis : 0)];
    }
  };
  if (first < a.M) records(0);
  for (int k0 = 0; k0 < a.ppw; k0 += PB) {
    if (first + k0 >= a.M) break;
    uint32_t pkc[PB];
    T yc[PB];
#pragma unroll
    for (int b = 0; b < PB; ++b) {
      pkc[b] = pkn[b];
      yc[b] = yn[b];
    }
    if (k0 + PB < a.ppw && first + k0 + PB < a.M) records(k0 + PB);
    T v[PB];
    int iz[PB], gxb[PB], gyb[PB][YCH];
    int64_t gin[PB];  // first grid channel of the point's instance
    T wxy[PB][YCH];
    bool ok[PB];
#pragma unroll
    for (int b = 0; b < PB; ++b) {
      ok[b] = first + k0 + b < a.M;
      gin[b] = a.ninst > 1 && ok[b] ? (int64_t)sorted_instance(a.offsets, a.nbins, a.ninst, first + k0 + b) * NCH : 0;
      T u = (T)0;
#pragma unroll
      for (int i = DEG; i >= 0; --i) u = u * yc[b] + cfr[i];
      v[b] = u;
      const int ix = unpack_i0<DIM>(pkc[b], 0), iy = unpack_i0<DIM>(pkc[b], 1);
      iz[b] = DIM == 3 ? unpack_i0<DIM>(pkc[b], 2) : 0;
      const T wxa = lane_value(v[b], xl < W ? xl : 0);
      const T wx = xl < W ? wxa : (T)0;
      gxb[b] = ix + xl;
      if (gxb[b] >= a.nf[0]) gxb[b] -= a.nf[0];
#pragma unroll
      for (int ch = 0; ch < YCH; ++ch) {
        const int jy = yl + YL * ch;
        const bool act = ok[b] && xl < W && jy < W && yl < YL;
        const T wya = lane_value(v[b], 16 + (jy < W ? jy : 0));
        wxy[b][ch] = act ? wx * wya : (T)0;
        int gy = iy + (jy < W ? jy : 0);
        if (gy >= a.nf[1]) gy -= a.nf[1];
        gyb[b][ch] = act ? gy : -1;
      }
    }
    T acc[PB][SC];
#pragma unroll
    for (int b = 0; b < PB; ++b)
#pragma unroll
      for (int c = 0; c < SC; ++c) acc[b][c] = (T)0;
#pragma unroll
    for (int ch = 0; ch < YCH; ++ch) {
      // planes jz0 .. jz0+G-1 of this chunk (a rolled loop when the support has more planes)
#pragma unroll 1
      for (int jz0 = 0; jz0 < NZ; jz0 += G) {
        T cv[PB][G][SC];
#pragma unroll
        for (int b = 0; b < PB; ++b)
#pragma unroll
          for (int t = 0; t < G; ++t) {
            const int jz = jz0 + t;
#pragma unroll
            for (int c = 0; c < SC; ++c) cv[b][t][c] = (T)0;
            int gz = iz[b] + jz;
            if (DIM == 3 && gz >= a.nf[2]) gz -= a.nf[2];
            if (jz < NZ && gyb[b][ch] >= 0) {
              const int64_t g = ((int64_t)gz * a.nf[1] + gyb[b][ch]) * a.nf[0] + gxb[b];
              if (CPLX) {
                const cplx<T> z = reinterpret_cast<const cplx<T>*>(a.grid)[(int64_t)tr * cells + g];
                cv[b][t][0] = z.x;
                cv[b][t][SC - 1] = z.y;
              } else {
#pragma unroll
                for (int c = 0; c < SC; ++c) cv[b][t][c] = a.grid[(gin[b] + c) * cells + g];
              }
            }
          }
#pragma unroll
        for (int b = 0; b < PB; ++b)
#pragma unroll
          for (int t = 0; t < G; ++t) {
            const int jz = jz0 + t;
            const T wz = DIM == 3 ? uniform_lane_value(v[b], 32 + (jz < NZ ? jz : 0)) : (T)1;
            if (jz < NZ) {
              const T w = wxy[b][ch] * wz;
#pragma unroll
              for (int c = 0; c < SC; ++c) acc[b][c] += w * cv[b][t][c];
            }
          }
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
      for (int b = 0; b < PB; ++b)
#pragma unroll
        for (int c = 0; c < SC; ++c) acc[b][c] += __shfl_xor(acc[b][c], off, 64);
    if (lane < PB) {  // lane b writes point b
      T res[SC];
#pragma unroll
      for (int c = 0; c < SC; ++c) res[c] = acc[0][c];
#pragma unroll
      for (int b = 1; b < PB; ++b)
        if (lane == b)
#pragma unroll
          for (int c = 0; c < SC; ++c) res[c] = acc[b][c];
      const int64_t pos = first + k0 + lane;
      if (pos < a.M) {
        const int64_t j = a.s_idx[pos];
        if (CPLX) {
          a.out[((int64_t)tr * a.M + j) * 2 + 0] = res[0];
          a.out[((int64_t)tr * a.M + j) * 2 + 1] = res[SC - 1];
        } else {
#pragma unroll
          for (int c = 0; c < SC; ++c) a.out[j * NCH + c] = res[c];
          if (a.move)
#pragma unroll
            for (int c = 0; c < SC; ++c) a.move[j * NCH + c] = fma(a.move_a, (double)res[c], a.move_in[j * NCH + c]);
        }
      }
    }
  }
}

template <typename T, int DIM, int W, int NCH, bool CPLX>
__global__ __launch_bounds__(256) void k_interp(InterpArgs<T> a) {
  interp_body<T, DIM, W, NCH, CPLX>(a, launch_blk());
}
template <typename T, int DIM, int W, int NCH, bool CPLX>
__global__ __launch_bounds__(256) void k_interp_parts(Parts<InterpArgs<T>> f) {
  Blk b;
  const int g = part_blk(f, b);
  if (g >= 0) interp_body<T, DIM, W, NCH, CPLX>(f.a[g], b);
}

// ---- dispatch over (precision, dim, w, channels) ----
template <typename T, int DIM>
static SpreadArgs<T> spread_args(const Plan& p, int64_t M, const void* str) {
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
  a.nwork = p.slot_ctr + 2;
  a.work = (const int2*)p.work;
  a.tile_parts = p.tile_parts;
  a.tile_slot = p.tile_slot;
  a.scratch = (T*)p.split_scratch;
  a.slots = p.split_slots;
  a.split_list = p.split_list;
  a.split_cnt = p.slot_ctr + 1;
  a.rowmask = p.ninst > 1 && DIM == 3 ? nullptr : p.rowmask;  // no masks on 3D multi-instance plans
  a.xcd_chunk = p.xcd_chunk_spread;
  a.ninst = p.ninst;
  a.split = p.split;
  a.sstr = (T*)p.s_str;
  return a;
}

template <int DIM>
static TilePartsArgs tile_parts_args(const Plan& p) {
  return TilePartsArgs{DIM, (int)p.nt[0], (int)p.nt[1], (int)p.nt[2], (int)p.qn[0], (int)p.qn[1], (int)p.qn[2],
                       p.ninst, p.split, (const int*)p.offsets, p.tile_parts, p.slot_ctr, 0, nullptr, nullptr,
                       nullptr};
}

static FillWorkArgs fill_work_args(const Plan& p) {
  return FillWorkArgs{(int)p.nbt, (const int*)p.part_off, (const int*)p.tile_parts, (int2*)p.work, p.tile_slot,
                      p.slot_ctr, p.split_list};
}

// Bound on the split tiles: each takes at least two of the split_slots scratch slots.
static int64_t merge_blocks(const Plan& p) {
  return (p.split_slots / 2 + 1) * (p.dim == 3 ? merge_chunks<3>() : merge_chunks<2>());
}

template <typename T, int DIM, int NCH, bool CPLX, int W>
static hipError_t run_spread(Plan& p, int64_t M, const void* str, int ntr, hipStream_t st) {
  const SpreadArgs<T> a = spread_args<T, DIM>(p, M, str);
  const unsigned nb = (unsigned)p.nbt;
  // real strengths the sort already placed in sorted order (its scatter) are not placed again
  if (M > 0 && !(!CPLX && ntr == 1 && p.sstr_src == str)) {
    hipLaunchKernelGGL((k_sort_strengths<T, NCH, CPLX>), dim3((unsigned)((M + 255) / 256), (unsigned)ntr), dim3(256), 0,
                       st, SortStrArgs<T>{M, (const int*)p.s_idx, (const T*)str, a.sstr});
    hipError_t e0 = hipGetLastError();
    if (e0 != hipSuccess) return e0;
  }
  hipError_t e;
  // the sort's row-mask pass built the tiles' parts and the work list with its split; else the parts
  // here, and their offsets and the work list from a scan
  if (p.parts_split != p.split) {
    hipLaunchKernelGGL(k_tile_parts, dim3((nb + 255) / 256), dim3(256), 0, st, tile_parts_args<DIM>(p));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_scan_fill_work(p.nbt, p.tile_parts, p.part_off, p.scan_part, fill_work_args(p), st)) != hipSuccess)
      return e;
  }
  const bool prof = prof_on(p, PROF_SPREAD);
  if (prof) prof_start(p, st);
  const dim3 sg((unsigned)p.work_blocks, (unsigned)ntr);
  const int nt = plan_spread_threads<DIM, T>(p);
  if constexpr (DIM == 3) {
    hipLaunchKernelGGL((k_spread<T, DIM, W, NCH, CPLX, 256>), sg, dim3(256), 0, st, a);
  } else {
    if (nt == 256)
      hipLaunchKernelGGL((k_spread<T, DIM, W, NCH, CPLX, 256>), sg, dim3(256), 0, st, a);
    else if (nt == 128)
      hipLaunchKernelGGL((k_spread<T, DIM, W, NCH, CPLX, 128>), sg, dim3(128), 0, st, a);
    else
      hipLaunchKernelGGL((k_spread<T, DIM, W, NCH, CPLX, 64>), sg, dim3(64), 0, st, a);
  }
  // algorithmic bytes: the grid written once, per point its sorted record and its strengths read
  if (prof)
    prof_stop(p, (double)ntr * p.ninst * p.fine_cells() * NCH * sizeof(T) + (double)M * (8 + DIM * sizeof(T)) +
                     (double)ntr * M * NCH * sizeof(T), st);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((k_merge_tiles<T, DIM, NCH, CPLX>), dim3((unsigned)merge_blocks(p), (unsigned)ntr),
                     dim3(kSpreadThreads), 0, st, a);
  return hipGetLastError();
}

// A launch over parts of a kernel with `nt` threads per workgroup: `k1` alone, `kp` over parts.
#define FSIB_PARTS(k1, kp, Args, nt)                                                                          \
  [&](const PartLaunch<Args>& L) {                                                                           \
    hipLaunchKernelGGL(k1, dim3((unsigned)L.nx, (unsigned)L.ny), dim3(nt), 0, st, L.a);                       \
    return hipGetLastError();                                                                                \
  },                                                                                                         \
      [&](const Parts<Args>& f, int64_t nwg, size_t, int) {                                                  \
        hipLaunchKernelGGL(kp, dim3((unsigned)nwg), dim3(nt), 0, st, f);                                     \
        return hipGetLastError();                                                                            \
      }

// run_spread (real strengths, one transform) for the plans of a group, each stage one launch.
template <typename T, int DIM, int W>
static hipError_t run_spread_group(const std::vector<Plan*>& ps, const int64_t* M, const void* const* str,
                                   hipStream_t st) {
  constexpr int NCH = DIM;
  const size_t n = ps.size();
  std::vector<PartLaunch<SortStrArgs<T>>> ss(n);
  std::vector<PartLaunch<TilePartsArgs>> tp(n);
  std::vector<FillWorkArgs> fw;  // the plans whose parts and work list the sort did not build
  std::vector<PartLaunch<SpreadArgs<T>>> sp(n), mg(n);
  std::vector<int64_t> nbt;
  std::vector<const int*> tparts;
  std::vector<int*> poff, spart;
  for (size_t g = 0; g < n; ++g) {
    Plan& p = *ps[g];
    const SpreadArgs<T> a = spread_args<T, DIM>(p, M[g], str[g]);
    ss[g].a = SortStrArgs<T>{M[g], (const int*)p.s_idx, (const T*)str[g], a.sstr};
    ss[g].nx = p.sstr_src == str[g] ? 0 : (M[g] + 255) / 256;  // placed by the sort's scatter
    tp[g].a = tile_parts_args<DIM>(p);
    tp[g].nx = p.parts_split == p.split ? 0 : (p.nbt + 255) / 256;  // computed by the sort
    if (p.parts_split != p.split) {
      fw.push_back(fill_work_args(p));
      nbt.push_back(p.nbt);
      tparts.push_back(p.tile_parts);
      poff.push_back(p.part_off);
      spart.push_back(p.scan_part);
    }
    sp[g].a = a;
    sp[g].nx = p.work_blocks;
    sp[g].threads = plan_spread_threads<DIM, T>(p);
    mg[g].a = a;
    mg[g].nx = merge_blocks(p);
  }
  hipError_t e = launch_parts(ss, FSIB_PARTS((k_sort_strengths<T, NCH, false>), (k_sort_strengths_parts<T, NCH, false>),
                                             SortStrArgs<T>, 256));
  if (e != hipSuccess) return e;
  if ((e = launch_parts(tp, FSIB_PARTS(k_tile_parts, k_tile_parts_parts, TilePartsArgs, 256))) != hipSuccess) return e;
  if (!fw.empty() && (e = launch_scan_fill_work_group(nbt, tparts, poff, spart, fw, st)) != hipSuccess) return e;
  // parts with different spreading variants run as launches of their own (launch_parts)
  const auto one = [&](const PartLaunch<SpreadArgs<T>>& L) {
    const dim3 g1((unsigned)L.nx);
    if constexpr (DIM == 3) {
      hipLaunchKernelGGL((k_spread<T, DIM, W, NCH, false, 256>), g1, dim3(256), 0, st, L.a);
    } else {
      if (L.threads == 256)
        hipLaunchKernelGGL((k_spread<T, DIM, W, NCH, false, 256>), g1, dim3(256), 0, st, L.a);
      else if (L.threads == 128)
        hipLaunchKernelGGL((k_spread<T, DIM, W, NCH, false, 128>), g1, dim3(128), 0, st, L.a);
      else
        hipLaunchKernelGGL((k_spread<T, DIM, W, NCH, false, 64>), g1, dim3(64), 0, st, L.a);
    }
    return hipGetLastError();
  };
  const auto fused = [&](const Parts<SpreadArgs<T>>& f, int64_t nwg, size_t, int thr) {
    const dim3 g1((unsigned)nwg);
    if constexpr (DIM == 3) {
      hipLaunchKernelGGL((k_spread_parts<T, DIM, W, NCH, false, 256>), g1, dim3(256), 0, st, f);
    } else {
      if (thr == 256)
        hipLaunchKernelGGL((k_spread_parts<T, DIM, W, NCH, false, 256>), g1, dim3(256), 0, st, f);
      else if (thr == 128)
        hipLaunchKernelGGL((k_spread_parts<T, DIM, W, NCH, false, 128>), g1, dim3(128), 0, st, f);
      else
        hipLaunchKernelGGL((k_spread_parts<T, DIM, W, NCH, false, 64>), g1, dim3(64), 0, st, f);
    }
    return hipGetLastError();
  };
  if ((e = launch_parts(sp, one, fused)) != hipSuccess) return e;
  return launch_parts(mg, FSIB_PARTS((k_merge_tiles<T, DIM, NCH, false>), (k_merge_tiles_parts<T, DIM, NCH, false>),
                                     SpreadArgs<T>, kSpreadThreads));
}

template <typename T, int DIM, int NCH, bool CPLX, int W>
static InterpArgs<T> interp_args(const Plan& p, int64_t M, void* out) {
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
  a.xcd_chunk = p.xcd_chunk_interp;
  // points per wavefront: the plan's knob rounded up to a multiple of the points summed together
  constexpr int PB = interp_pb<T, DIM, W, NCH, CPLX>();
  a.ppw = (p.interp_points + PB - 1) / PB * PB;
  a.offsets = p.offsets;
  a.nbins = (int)p.nbins;
  a.ninst = p.ninst;
  a.move = nullptr;
  a.move_in = nullptr;
  a.move_a = 0;
  return a;
}

template <typename T, int DIM, int NCH, bool CPLX, int W>
static hipError_t run_interp(Plan& p, int64_t M, void* out, int ntr, hipStream_t st, double* move, double move_a) {
  if (M == 0) return hipSuccess;
  if (p.deg != interp_degree<W>()) return hipErrorInvalidValue;  // the kernel's compile-time degree
  InterpArgs<T> a = interp_args<T, DIM, NCH, CPLX, W>(p, M, out);
  a.move = CPLX ? nullptr : move;
  a.move_in = move;
  a.move_a = move_a;
  const bool prof = prof_on(p, PROF_INTERP);
  if (prof) prof_start(p, st);
  const int64_t per_wg = 4 * (int64_t)a.ppw;  // four wavefronts per workgroup
  hipLaunchKernelGGL((k_interp<T, DIM, W, NCH, CPLX>), dim3((unsigned)((M + per_wg - 1) / per_wg), (unsigned)ntr),
                     dim3(256), 0, st, a);
  // algorithmic bytes: per point its sorted record, w^d grid cells per channel, the result
  if (prof) {
    double cellsper = 1;
    for (int d = 0; d < DIM; ++d) cellsper *= W;
    prof_stop(p, (double)M * (8 + DIM * sizeof(T)) + (double)ntr * M * (cellsper + 1) * NCH * sizeof(T), st);
  }
  return hipGetLastError();
}

template <typename T, int DIM, int W>
static hipError_t run_interp_group(const std::vector<Plan*>& ps, const int64_t* M, void* const* out, hipStream_t st,
                                   const GroupMove* mv) {
  constexpr int NCH = DIM;
  std::vector<PartLaunch<InterpArgs<T>>> v(ps.size());
  for (size_t g = 0; g < ps.size(); ++g) {
    if (ps[g]->deg != interp_degree<W>()) return hipErrorInvalidValue;
    v[g].a = interp_args<T, DIM, NCH, false, W>(*ps[g], M[g], out[g]);
    if (mv) {
      v[g].a.move = mv->out[g];
      v[g].a.move_in = mv->in[g];
      v[g].a.move_a = mv->a[g];
    }
    const int64_t per_wg = 4 * (int64_t)v[g].a.ppw;
    v[g].nx = (M[g] + per_wg - 1) / per_wg;
  }
  return launch_parts(v, FSIB_PARTS((k_interp<T, DIM, W, NCH, false>), (k_interp_parts<T, DIM, W, NCH, false>),
                                    InterpArgs<T>, 256));
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
static hipError_t interp_dispatch(Plan& p, int64_t M, void* out, int ntr, hipStream_t st, double* move = nullptr,
                                  double move_a = 0) {
#define CALL_I(w) run_interp<T, DIM, NCH, CPLX, w>(p, M, out, ntr, st, move, move_a)
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

hipError_t launch_interp(Plan& p, int64_t M, void* out, int real_comps, hipStream_t st, double* move, double move_a) {
  const bool f64 = p.prec == FSIB_F64;
  if (real_comps == 0) {
    if (p.dim == 2)
      return f64 ? interp_dispatch<double, 2, 2, true>(p, M, out, p.ntrans, st)
                 : interp_dispatch<float, 2, 2, true>(p, M, out, p.ntrans, st);
    return f64 ? interp_dispatch<double, 3, 2, true>(p, M, out, p.ntrans, st)
               : interp_dispatch<float, 3, 2, true>(p, M, out, p.ntrans, st);
  }
  if (p.dim == 2)
    return f64 ? interp_dispatch<double, 2, 2, false>(p, M, out, 1, st, move, move_a)
               : interp_dispatch<float, 2, 2, false>(p, M, out, 1, st, move, move_a);
  return f64 ? interp_dispatch<double, 3, 3, false>(p, M, out, 1, st, move, move_a)
             : interp_dispatch<float, 3, 3, false>(p, M, out, 1, st, move, move_a);
}

template <typename T, int DIM>
static hipError_t spread_group_dispatch(const std::vector<Plan*>& ps, const int64_t* M, const void* const* str,
                                        hipStream_t st) {
#define CALL_SG(w) run_spread_group<T, DIM, w>(ps, M, str, st)
  FSIB_W_SWITCH(ps[0]->w, CALL_SG)
#undef CALL_SG
}

template <typename T, int DIM>
static hipError_t interp_group_dispatch(const std::vector<Plan*>& ps, const int64_t* M, void* const* out,
                                        hipStream_t st, const GroupMove* mv) {
#define CALL_IG(w) run_interp_group<T, DIM, w>(ps, M, out, st, mv)
  FSIB_W_SWITCH(ps[0]->w, CALL_IG)
#undef CALL_IG
}

// The plans of a group share precision, dimension and kernel width (checked when the group is made).
hipError_t launch_spread_group(const std::vector<Plan*>& ps, const int64_t* M, const void* const* str, hipStream_t st) {
  const bool f64 = ps[0]->prec == FSIB_F64;
  if (ps[0]->dim == 2)
    return f64 ? spread_group_dispatch<double, 2>(ps, M, str, st) : spread_group_dispatch<float, 2>(ps, M, str, st);
  return f64 ? spread_group_dispatch<double, 3>(ps, M, str, st) : spread_group_dispatch<float, 3>(ps, M, str, st);
}

hipError_t launch_interp_group(const std::vector<Plan*>& ps, const int64_t* M, void* const* out, hipStream_t st,
                               const GroupMove* mv) {
  const bool f64 = ps[0]->prec == FSIB_F64;
  if (ps[0]->dim == 2)
    return f64 ? interp_group_dispatch<double, 2>(ps, M, out, st, mv)
               : interp_group_dispatch<float, 2>(ps, M, out, st, mv);
  return f64 ? interp_group_dispatch<double, 3>(ps, M, out, st, mv)
             : interp_group_dispatch<float, 3>(ps, M, out, st, mv);
}

}  // namespace fsib
