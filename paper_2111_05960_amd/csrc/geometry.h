// Grid geometry, boundary rules and the buffers of the state.
//
// Layout in device memory: plane-major structure of arrays f[z][k][y][x],
// x fastest: each z-plane holds its Q population planes one after the other
// (for D2Q9, nz = 1, this is f[k][y][x]).  A wavefront of 64 consecutive x
// reads 64 consecutive elements of one population, and all Q populations of
// a plane lie within Q * nx * ny elements of each other, so a kernel addresses
// them from one per-plane base and a 32-bit offset.
//
// State invariant between steps (time level n):
//   G   = g~*^n      post-collision phi populations, not yet streamed
//   H   = h~*^{n-1}  post-collision c populations of the previous step
//   PHI = phi^n
// Streaming is a pull: the population k arriving at x comes from x - e_k
// (periodic wrap), or, when x - e_k lies beyond a zero-flux wall, is the
// opposite population leaving x (halfway bounce-back).  So g~^n and h~^n are
// never stored; they are read on the fly by the kernel that needs them.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gplbm {

struct Geo {
  int nx, ny, nz;
  int bcx, bcy, bcz;  // 0 periodic, 1 zero flux
  int64_t N;          // nx*ny*nz
};

__device__ __forceinline__ int64_t node_index(const Geo& g, int x, int y, int z) {
  return (int64_t)x + (int64_t)g.nx * ((int64_t)y + (int64_t)g.ny * z);
}

// Source coordinate of a pull along one axis; false when the source lies
// beyond a zero-flux wall.
__device__ __forceinline__ bool pull_axis(int& c, int e, int n, int bc) {
  c -= e;
  if (c < 0) {
    if (bc) return false;
    c += n;
  } else if (c >= n) {
    if (bc) return false;
    c -= n;
  }
  return true;
}

// Neighbour coordinate of the gradient stencil along one axis: periodic wrap
// or mirror ghost (phi(-1) = phi(0), phi(n) = phi(n-1)) at a zero-flux wall.
__device__ __forceinline__ int stencil_axis(int c, int n, int bc) {
  if (c < 0) return bc ? 0 : c + n;
  if (c >= n) return bc ? n - 1 : c - n;
  return c;
}

// Element index of population k at node (x, y, z).
template <class L>
__device__ __forceinline__ int64_t pop_index(const Geo& g, int k, int x, int y, int z) {
  const int64_t plane = (int64_t)g.nx * g.ny;
  return ((int64_t)z * L::Q + k) * plane + (int64_t)y * g.nx + x;
}

// Pull of population k at (x, y, z) from a post-collision array f.
template <class L, class S>
__device__ __forceinline__ S pull(const Geo& g, const S* __restrict__ f, int k, int x, int y,
                                  int z) {
  int sx = x, sy = y, sz = z;
  bool in = pull_axis(sx, L::ex[k], g.nx, g.bcx) && pull_axis(sy, L::ey[k], g.ny, g.bcy);
  if (L::D == 3) in = in && pull_axis(sz, L::ez[k], g.nz, g.bcz);
  if (!in) return f[pop_index<L>(g, L::opp[k], x, y, z)];
  return f[pop_index<L>(g, k, sx, sy, sz)];
}

}  // namespace gplbm
