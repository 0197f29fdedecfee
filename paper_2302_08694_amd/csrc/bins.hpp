// Per-tile candidate counts of spreading, shared by the point sort (which computes them beside the row
// masks) and the spreading launcher (which computes them when the sort did not).
#pragma once

#include "common.hpp"

namespace fsib {

// Points reaching each tile (its bin and the q bins before it per axis) and the parts it splits into.
// slot_ctr: [0] scratch slots taken, [1] split tiles listed, [2] further parts (work list entries).
// direct = 0: tg = 0 clears the counters, and the work list comes from a scan of tile_parts afterwards;
// direct = 1 (the counters cleared by an earlier pass): each split tile also takes its work list
// entries, scratch slots and split-list entry here with atomics, so no scan is needed.  The entries
// land in arrival order; every part is spread the same whatever workgroup takes it and the merge sums
// a tile's parts in part order, so results do not depend on it.
struct TilePartsArgs {
  int dim, nt0, nt1, nt2, q0, q1, q2, ninst, split;
  const int* offsets;
  int* tile_parts;
  int* slot_ctr;
  int direct;
  int2* work;
  int* tile_slot;
  int* split_list;
  const int* counts = nullptr;  // the bin counts, read instead of offset differences when not null
};

// Tile tg of all instances (tg < nt0 nt1 nt2 ninst).
__device__ __forceinline__ void tile_parts_at(const TilePartsArgs& A, int tg) {
  const int dim = A.dim, nt0 = A.nt0, nt1 = A.nt1, nt2 = A.nt2, q0 = A.q0, q1 = A.q1, q2 = A.q2, ninst = A.ninst,
            split = A.split;
  const int* __restrict__ offsets = A.offsets;
  if (!A.direct && tg == 0) {
    A.slot_ctr[0] = 0;
    A.slot_ctr[1] = 0;
    A.slot_ctr[2] = 0;
  }
  const int nbins = nt0 * nt1 * nt2;
  if (tg >= nbins * ninst) return;
  const int inst = tg / nbins, t = tg - inst * nbins;
  const int tx = t % nt0, ty = (t / nt0) % nt1, tz = t / (nt0 * nt1);
  int total = 0;
  for (int dz = 0; dz <= (dim == 3 ? q2 : 0); ++dz)
    for (int dy = 0; dy <= q1; ++dy)
      for (int dx = 0; dx <= q0; ++dx) {
        const int bx = (tx - dx + nt0) % nt0, by = (ty - dy + nt1) % nt1, bz = dim == 3 ? (tz - dz + nt2) % nt2 : 0;
        const int b = bx + nt0 * (by + nt1 * bz) + inst * nbins;
        total += A.counts ? A.counts[b] : offsets[b + 1] - offsets[b];
      }
  const int np = total <= split ? 1 : (total + split - 1) / split;
  A.tile_parts[tg] = np;
  if (A.direct) {
    if (np > 1) {
      const int off = atomicAdd(A.slot_ctr + 2, np - 1);
      for (int q = 1; q < np; ++q) A.work[off + q - 1] = make_int2(tg, q);
      A.tile_slot[tg] = atomicAdd(A.slot_ctr, np);
      A.split_list[atomicAdd(A.slot_ctr + 1, 1)] = tg;
    } else {
      A.tile_slot[tg] = -1;
    }
  }
}

// Work list of the further parts (tile, part >= 1) in tile order, and scratch slots for tiles split
// into several parts.
struct FillWorkArgs {
  int nbins;
  const int* part_off;
  const int* tile_parts;
  int2* work;
  int* tile_slot;
  int* slot_ctr;  // [0] scratch slots, [1] split tiles (zero before the launch), [2] the entries (set here)
  int* split_list;
};
__device__ __forceinline__ void fill_work_tile(const FillWorkArgs& A, int t) {
  // parts 1.. of tile t: entries part_off[t] - t .. (parts before t, less one per tile)
  const int np = A.tile_parts[t], off = A.part_off[t] - t;
  for (int q = 1; q < np; ++q) A.work[off + q - 1] = make_int2(t, q);
  A.tile_slot[t] = np > 1 ? atomicAdd(A.slot_ctr, np) : -1;
  if (np > 1) A.split_list[atomicAdd(A.slot_ctr + 1, 1)] = t;
}

}  // namespace fsib
