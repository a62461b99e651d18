// Fused schedule for D3Q19: one kernel per time step n -> n+1, marching in z.
//
// A block owns an x-y output tile T of (BX-2) x (BY-2) nodes and a chunk of
// ZC planes, and runs one thread per node of the tile grown by one node in x
// and y (T+1).  It walks the planes p = z0-1 .. z1 (one halo plane below and
// above the chunk).  At plane p every thread
//   - pulls h~^n (-> c^n, mu^n) and g~^{n+1} (-> phi^{n+1}; the values stay in
//     registers for the g collision one plane later),
//   - takes phi^n of planes p-1, p, p+1 from a 3-plane LDS ring (T+2 in x-y)
//     for the gradient, writes phi^{n+1}(p) into a second ring,
//   - runs the h collision of step n.
// The post-collision h* are then streamed inside the block into a ring of
// three LDS accumulator planes: the e_z = +1 populations go to plane p+1, the
// in-plane ones to plane p, the e_z = -1 ones to plane p-1.  Because D3Q19 is
// numbered by layers of e_z (+1, 0, -1), every node's c^{n+1} receives its
// populations in index order across the three planes, the order of a pull.
// After plane p, c^{n+1}(p-1) is complete and the threads of T run the g
// collision of step n+1 at plane p-1.
//
// Only periodic domains take this path (a wall would bounce some +z
// populations into a plane one step later than the index order allows); the
// split schedule serves the others.
//
// HBM traffic per node and step is the algorithmic minimum (2Q reads, 2Q
// writes, phi read and write).  The x-y halo ring and the two halo planes are
// recomputed; their pulls hit the L2.
#pragma once

#include "kernels_fused2d.h"

namespace gplbm {

__device__ __forceinline__ int ring3(int q) { return (q + 6) % 3; }

template <int BX, int BY, int ZC, class S, class C>
__global__ void __launch_bounds__(BX* BY) k_fused3d(Geo g, Coef<C> K, StepBufs<S> b, int tiles_x,
                                                    int tiles_xy, int ntiles) {
  using L = D3Q19;
  constexpr int Q = L::Q;
  constexpr int TX = BX - 2, TY = BY - 2;
  constexpr int AX = BX + 2, AY = BY + 2;
  __shared__ C phiA[3][AY][AX];      // phi^n, planes p-1, p, p+1
  __shared__ C phiB[3][BY][BX];      // phi^{n+1}, planes p-2, p-1, p
  __shared__ double acc[3][BY][BX];  // c^{n+1} being accumulated

  const int tile = xcd_tile(blockIdx.x, ntiles);
  const int chunk = tile / tiles_xy, txy = tile % tiles_xy;
  const int X0 = (txy % tiles_x) * TX, Y0 = (txy / tiles_x) * TY;
  const int z0 = chunk * ZC, z1 = min(z0 + ZC, g.nz);
  const int tx = threadIdx.x % BX, ty = threadIdx.x / BX;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int plane = nx * ny;

  const int ux = X0 - 1 + tx, uy = Y0 - 1 + ty;
  const bool out = ux < nx && uy < ny && tx >= 1 && tx <= TX && ty >= 1 && ty <= TY;
  // wrapped neighbour coordinates along x and y (periodic)
  const int x = wrap_coord(ux, nx), y = wrap_coord(uy, ny);
  const int xo[3] = {x == 0 ? nx - 1 : x - 1, x, x == nx - 1 ? 0 : x + 1};
  const int yo[3] = {(y == 0 ? ny - 1 : y - 1) * nx, y * nx, (y == ny - 1 ? 0 : y + 1) * nx};

  auto load_phiA = [&](int p) {
    const int zp = wrap_coord(p, nz);
    const S* src = b.PHI + (int64_t)zp * plane;
    for (int l = threadIdx.x; l < AX * AY; l += BX * BY) {
      const int lx = l % AX, ly = l / AX;
      const int gx = wrap_coord(X0 - 2 + lx, nx), gy = wrap_coord(Y0 - 2 + ly, ny);
      phiA[ring3(p)][ly][lx] = C(src[gy * nx + gx]);
    }
  };

  load_phiA(z0 - 2);
  load_phiA(z0 - 1);

  C g_old[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) g_old[k] = C(0);

  for (int p = z0 - 1; p <= z1; ++p) {
    load_phiA(p + 1);
    __syncthreads();

    const int zp = wrap_coord(p, nz);
    const int zo[3] = {(zp == 0 ? nz - 1 : zp - 1), zp, (zp == nz - 1 ? 0 : zp + 1)};
    const int node = zp * plane + y * nx + x;

    // pulls: population k at (x,y,zp) comes from (x,y,zp) - e_k
    C h[Q], g_new[Q];
    double c = 0.0, sg = 0.0;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int src = zo[1 - L::ez[k]] * plane + yo[1 - L::ey[k]] + xo[1 - L::ex[k]];
      const S hv = b.H[(int64_t)k * g.N + src];
      h[k] = C(hv);
      c = k == 0 ? double(hv) : c + double(hv);
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int src = zo[1 - L::ez[k]] * plane + yo[1 - L::ey[k]] + xo[1 - L::ex[k]];
      const S gv = b.G[(int64_t)k * g.N + src];
      g_new[k] = C(gv);
      sg = k == 0 ? double(gv) : sg + double(gv);
    }
    const int sA = ring3(p);
    const C phi = phiA[sA][ty + 1][tx + 1];
    const C mu = C(closure(K.cl, K.cs, K.mueq, c, double(phi)));
    auto atA = [&](int dx, int dy, int dz) -> C {
      return phiA[ring3(p + dz)][ty + 1 + dy][tx + 1 + dx];
    };
    C gr[3], n[3];
    gradient_normal<L, C>(atA, K.eps2, gr, n);
    const C sbar = source_moment<C>(K, phi, mu);
    const double phin = sg + 0.5 * double(sbar);
    const C phin_c = C(phin);
    phiB[sA][ty][tx] = phin_c;
    const C dtphi = phin_c - phi;
    C F[3];
    h_flux<L, C>(K, mu, gr, n, dtphi, K.anti_trapping != 0, F);
    const C lam = h_lambda<C>(K, phi, mu);
    const C cc = C(c);
    C hs[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k)
      hs[k] = C(S(h_collide<L, C>(K, k, h[k], h_eq<L, C>(k, cc, lam), h_source<L, C>(K, k, F))));

    const bool own_p = p >= z0 && p < z1;
    if (out && own_p) {
#pragma unroll
      for (int k = 0; k < Q; ++k) b.Hn[(int64_t)k * g.N + node] = S(hs[k]);
      b.PHIn[node] = S(phin_c);
    }

    // in-block streaming of h* into the accumulator ring, 9 passes:
    // pass j carries population j (e_z=+1, to plane p+1), population 5+j
    // (e_z=0, to plane p) and population 14+j (e_z=-1, to plane p-1)
    const bool up_ok = p + 1 >= z0 && p + 1 < z1, dn_ok = p - 1 >= z0 && p - 1 < z1;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      if (j < 5 && up_ok) {
        const int k = j;
        const int tx2 = tx + L::ex[k], ty2 = ty + L::ey[k];
        if (tx2 >= 1 && tx2 <= TX && ty2 >= 1 && ty2 <= TY) {
          double& a = acc[ring3(p + 1)][ty2][tx2];
          a = k == 0 ? double(hs[k]) : a + double(hs[k]);
        }
      }
      if (own_p) {
        const int k = 5 + j;
        const int tx2 = tx + L::ex[k], ty2 = ty + L::ey[k];
        if (tx2 >= 1 && tx2 <= TX && ty2 >= 1 && ty2 <= TY) {
          double& a = acc[sA][ty2][tx2];
          a = a + double(hs[k]);
        }
      }
      if (j < 5 && dn_ok) {
        const int k = 14 + j;
        const int tx2 = tx + L::ex[k], ty2 = ty + L::ey[k];
        if (tx2 >= 1 && tx2 <= TX && ty2 >= 1 && ty2 <= TY) {
          double& a = acc[ring3(p - 1)][ty2][tx2];
          a = a + double(hs[k]);
        }
      }
      __syncthreads();
    }

    // g collision of step n+1 at plane p-1
    if (out && dn_ok) {
      const int zq = wrap_coord(p - 1, nz);
      const int qnode = zq * plane + y * nx + x;
      const int sB = ring3(p - 1);
      const double c1 = acc[sB][ty][tx];
      const C phi1 = phiB[sB][ty][tx];
      const C mu1 = C(closure(K.cl, K.cs, K.mueq, c1, double(phi1)));
      auto atB = [&](int dx, int dy, int dz) -> C {
        return phiB[ring3(p - 1 + dz)][ty + dy][tx + dx];
      };
      C gr1[3], n1[3];
      gradient_normal<L, C>(atB, K.eps2, gr1, n1);
      C G[Q];
      phi_sources<L, C>(K, phi1, mu1, n1, G);
#pragma unroll
      for (int k = 0; k < Q; ++k)
        b.Gn[(int64_t)k * g.N + qnode] = S(g_collide<L, C>(K, k, g_old[k], phi1, G[k]));
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) g_old[k] = g_new[k];
  }
}

constexpr int kF3BX = 64, kF3BY = 8, kF3ZC = 32;

inline bool fused3d_supported(int nx, int ny, int nz, const int* bc) {
  return bc[0] == 0 && bc[1] == 0 && bc[2] == 0 && (int64_t)nx * ny * nz < ((int64_t)1 << 31);
}

template <class S, class C>
struct Fused3D {
  static int launch(const Geo& g, const Coef<C>& K, const StepBufs<S>& b, hipStream_t st) {
    constexpr int BX = kF3BX, BY = kF3BY, ZC = kF3ZC;
    const int tiles_x = (g.nx + BX - 3) / (BX - 2);
    const int tiles_y = (g.ny + BY - 3) / (BY - 2);
    const int chunks = (g.nz + ZC - 1) / ZC;
    const int tiles_xy = tiles_x * tiles_y;
    const int ntiles = tiles_xy * chunks;
    hipLaunchKernelGGL((k_fused3d<BX, BY, ZC, S, C>), dim3(ntiles), dim3(BX * BY), 0, st, g, K,
                       b, tiles_x, tiles_xy, ntiles);
    return 0;
  }
};

template <class L, class S, class C>
struct FusedLaunch {
  static int launch(const Geo& g, const Coef<C>& K, const StepBufs<S>& b, hipStream_t st) {
    if constexpr (L::D == 2)
      return Fused2D<L, S, C>::launch(g, K, b, st);
    else
      return Fused3D<S, C>::launch(g, K, b, st);
  }
};

}  // namespace gplbm
