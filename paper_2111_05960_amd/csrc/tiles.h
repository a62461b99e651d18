// Tile geometry and block scheduling shared by the fused kernels.
//
// x-aligned tiles: a tile owns TX x TY output nodes with TX a multiple of 64
// and tile origins at multiples of TX, so every output row is a run of whole
// 128-byte lines and its stores are full-line writes.  The block computes
// the tile grown by one node in x and y (the region, BX x BY): thread
// l < TX*BY takes region node (1 + l % TX, l / TX), one wavefront per region
// row when TX = 64, and the next 2*BY threads take the two halo columns.
//
// Persistent grid: one block per resident slot (occupancy x CUs); in each
// pass over the grid the slots of an XCD (block b runs on XCD b mod 8) take
// consecutive tiles, so that neighbouring tiles run at the same time and the
// lines of their shared halo are still in that XCD's L2 when the second tile
// reads them.
#pragma once

#include <hip/hip_runtime.h>

namespace gplbm {

constexpr int kNumXcd = 8;

__device__ __forceinline__ int wrap_coord(int u, int n) {
  int v = u % n;
  return v < 0 ? v + n : v;
}

template <int TX_, int TY_>
struct TileShape {
  static constexpr int TX = TX_, TY = TY_;
  static constexpr int BX = TX + 2, BY = TY + 2;
  static constexpr int kMain = TX * BY;
  static constexpr int kNodes = kMain + 2 * BY;
  static constexpr int NT = (kNodes + 63) / 64 * 64;
  static_assert(TX % 64 == 0, "output rows are whole wavefronts");
  static_assert(NT <= 1024, "block size");
  // region node (tx, ty) of thread l; threads past the region are not valid
  // and shadow node (0, 0)
  __device__ static void node(int l, int& tx, int& ty, bool& valid) {
    if (l < kMain) {
      tx = 1 + l % TX;
      ty = l / TX;
      valid = true;
    } else {
      const int j = l - kMain;
      valid = j < 2 * BY;
      const int jj = valid ? j : 0;
      tx = jj < BY ? 0 : BX - 1;
      ty = jj % BY;
    }
  }
};

// Resident grid of a persistent kernel: blocks per CU x CUs, a multiple of
// the XCD count, no more than the tiles need.  Cached per device in cache[].
template <class Kern>
inline int resident_grid(Kern kernel, int threads, int ntiles, int* cache) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return -1;
  if (cache[dev] == 0) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        per_cu < 1 || cus < 1)
      return -1;
    cache[dev] = max(kNumXcd, (per_cu * cus) / kNumXcd * kNumXcd);
  }
  return min(cache[dev], (ntiles + kNumXcd - 1) / kNumXcd * kNumXcd);
}

// First tile of this block in the first pass (the slots of an XCD take
// consecutive tiles); the block then strides by gridDim.x.
__device__ __forceinline__ int first_tile() {
  const int slots = gridDim.x / kNumXcd;
  return (blockIdx.x % kNumXcd) * slots + blockIdx.x / kNumXcd;
}

// x column of the tile txy (x fastest) of z chunk `chunk`.  A resident grid
// whose size is a multiple of the tiles per row keeps every block on one
// column; with walls the columns at an x wall are the slow ones, so the
// columns turn by one per chunk and every block takes its share of them.
__device__ __forceinline__ int tile_column(int txy, int tiles_x, int chunk, bool turn) {
  const int c = txy % tiles_x;
  return turn ? (c + chunk) % tiles_x : c;
}

}  // namespace gplbm
