// Fused schedule in 2-D: one kernel per time step n -> n+1.  g runs on
// D2Q9 or D2Q5 (L), h on D2Q9 or D2Q5 (LH).
//
// A block owns an output tile T of TX x TY nodes (x-aligned, tiles.h) and
// computes T grown by one node on each side (T+1).  Every thread of T+1:
//   - pulls h~^n (sum -> c^n, mu^n) and g~^{n+1} (kept in registers),
//   - reads phi^n around itself from an LDS tile covering T+2 (gradient,
//     normal, source moment), forms phi^{n+1} and writes it to an LDS tile,
//   - runs the h collision of step n (anti-trapping current from
//     phi^{n+1} - phi^n).
// The post-collision h* of T+1 are then streamed inside the block: they go to
// an LDS exchange, and after one barrier every node of T gathers the
// population k arriving from x - e_k (its own h*_{opp k} where x - e_k lies
// beyond a wall) in index order, so that c^{n+1} is summed in the same order
// as a pull would sum it.  Finally the threads of T run the g
// collision of step n+1 (gradient of phi^{n+1} from the LDS tile) and write
// g~*^{n+1}, h~*^n and phi^{n+1}.
//
// HBM traffic per node and step is the minimum: Q + Qh reads, Q + Qh writes,
// one phi read and one phi write, plus the recomputed halo ring where the L2
// misses it.  The grid is persistent with XCD-ordered passes (tiles.h).
#pragma once

#include "kernels_split.h"
#include "tiles.h"

namespace gplbm {

// FP32: at most 80 VGPRs, so that two blocks of 11 waves share a CU.
template <int TX, int TY, class L, class LH, class S, class C, bool kGen>
__global__ void __launch_bounds__((TileShape<TX, TY>::NT), (sizeof(S) == 4 ? 6 : 1))
    k_fused2d(Geo g, Coef<C> Kin, StepBufs<S> b, int tiles_x, int ntiles) {
  const Coef<C> K = variant<kGen>(Kin);
  using Shape = TileShape<TX, TY>;
  constexpr int BX = Shape::BX, BY = Shape::BY, NT = Shape::NT;
  constexpr int AX = BX + 2, AY = BY + 2;  // phi^n tile with a 2-node halo
  __shared__ C phiA[AY][AX];
  __shared__ C phiB[BY][BX];
  __shared__ C hx[LH::Q][BY][BX];  // h*^n of T+1 (moving populations)

  int tx, ty;
  bool valid;
  Shape::node(threadIdx.x, tx, ty, valid);

  for (int tile = first_tile(); tile < ntiles; tile += gridDim.x) {
  const int X0 = (tile % tiles_x) * TX, Y0 = (tile / tiles_x) * TY;

  // phi^n on T+2 (periodic wrap, or clamp = mirror ghost at a wall)
  for (int l = threadIdx.x; l < AX * AY; l += NT) {
    const int lx = l % AX, ly = l / AX;
    int ux = X0 - 2 + lx, uy = Y0 - 2 + ly;
    ux = g.bcx ? min(max(ux, 0), g.nx - 1) : wrap_coord(ux, g.nx);
    uy = g.bcy ? min(max(uy, 0), g.ny - 1) : wrap_coord(uy, g.ny);
    phiA[ly][lx] = C(b.PHI[node_index(g, ux, uy, 0)]);
  }

  const int ux = X0 - 1 + tx, uy = Y0 - 1 + ty;  // unwrapped node of this thread
  const bool in_x = ux >= 0 && ux < g.nx, in_y = uy >= 0 && uy < g.ny;
  const bool active = valid && (in_x || !g.bcx) && (in_y || !g.bcy);
  const bool out = valid && in_x && in_y && tx >= 1 && tx <= TX && ty >= 1 && ty <= TY;
  const int x = g.bcx ? ux : wrap_coord(ux, g.nx);
  const int y = g.bcy ? uy : wrap_coord(uy, g.ny);
  const int64_t i = active ? node_index(g, x, y, 0) : 0;
  // neighbour offsets clamped at walls (mirror ghost of the gradient stencil)
  const int xm = (g.bcx && ux == 0) ? 0 : -1, xp = (g.bcx && ux == g.nx - 1) ? 0 : 1;
  const int ym = (g.bcy && uy == 0) ? 0 : -1, yp = (g.bcy && uy == g.ny - 1) ? 0 : 1;
  __syncthreads();

  C gn[L::Q];   // g~^{n+1}
  C hs[LH::Q];  // h~*^n
  C phin_c = C(0);
  if (active) {
    C h[LH::Q];
    double c = 0.0;
#pragma unroll
    for (int k = 0; k < LH::Q; ++k) {
      S v = pull<LH>(g, b.H, k, x, y, 0);
      h[k] = C(v);
      c = k == 0 ? double(v) : c + double(v);
    }
    double sg = 0.0;
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      S v = pull<L>(g, b.G, k, x, y, 0);
      gn[k] = C(v);
      sg = k == 0 ? double(v) : sg + double(v);
    }
    const C phi = phiA[ty + 1][tx + 1];
    const C mu = C(closure(K.q, c, double(phi)));
    auto at = [&](int dx, int dy, int) -> C {
      const int ox = dx < 0 ? xm : (dx > 0 ? xp : 0);
      const int oy = dy < 0 ? ym : (dy > 0 ? yp : 0);
      return phiA[ty + 1 + oy][tx + 1 + ox];
    };
    C gr[3], n[3];
    gradient_normal<L, C>(at, K.eps2, gr, n);
    const C sbar = source_moment<C>(K, phi, mu);
    const double phin = sg + 0.5 * double(sbar);
    phin_c = C(phin);
    const C dtphi = phin_c - phi;
    C F[3];
    h_flux<L, C>(K, mu, gr, n, dtphi, K.anti_trapping != 0, F);
    const C lam = h_lambda<C>(K, phi, mu);
    const C cc = C(c);
#pragma unroll
    for (int k = 0; k < LH::Q; ++k) hs[k] = C(S(h_update<LH, C>(K, k, h[k], cc, lam, F)));
    balance_rest<LH, S, C>(hs, c);
  }
  if (valid) {
    phiB[ty][tx] = phin_c;
    if (active) {
#pragma unroll
      for (int k = 0; k < LH::Q; ++k)
        if (k != LH::REST) hx[k][ty][tx] = hs[k];
    }
  }
  __syncthreads();

  if (out) {
  // streaming of h* inside the tile: population k arrives from x - e_k, or
  // is this node's own h*_{opp k} bounced back where x - e_k is beyond a wall
  double c1 = 0.0;
#pragma unroll
  for (int k = 0; k < LH::Q; ++k) {
    C v;
    if (k == LH::REST) {
      v = hs[k];
    } else {
      const bool wall = (g.bcx && (ux - LH::ex[k] < 0 || ux - LH::ex[k] >= g.nx)) ||
                        (g.bcy && (uy - LH::ey[k] < 0 || uy - LH::ey[k] >= g.ny));
      v = wall ? hs[LH::opp[k]] : hx[k][ty - LH::ey[k]][tx - LH::ex[k]];
    }
    c1 = k == 0 ? double(v) : c1 + double(v);
  }
  const C phi1 = phiB[ty][tx];
  const C mu1 = C(closure(K.q, c1, double(phi1)));
  auto at1 = [&](int dx, int dy, int) -> C {
    const int ox = dx < 0 ? xm : (dx > 0 ? xp : 0);
    const int oy = dy < 0 ? ym : (dy > 0 ? yp : 0);
    return phiB[ty + oy][tx + ox];
  };
  C gr[3], n[3];
  gradient_normal<L, C>(at1, K.eps2, gr, n);
  C G[L::Q];
  phi_sources<L, C>(K, phi1, mu1, n, G);
  C gs[L::Q];
  double sg1 = 0.0;
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    sg1 = k == 0 ? double(gn[k]) : sg1 + double(gn[k]);
    gs[k] = C(S(g_collide<L, C>(K, k, gn[k], phi1, G[k])));
  }
  balance_g_rest<L, S, C>(K, gs, sg1, phi1, source_moment<C>(K, phi1, mu1));
#pragma unroll
  for (int k = 0; k < L::Q; ++k) b.Gn[pop_index<L>(g, k, x, y, 0)] = S(gs[k]);
#pragma unroll
  for (int k = 0; k < LH::Q; ++k) b.Hn[pop_index<LH>(g, k, x, y, 0)] = S(hs[k]);
  b.PHIn[i] = S(phi1);
  }
  __syncthreads();  // the LDS tiles are refilled by the next tile
  }
}

#ifndef GPLBM_F2_TY
#define GPLBM_F2_TY 8
#endif
#ifndef GPLBM_F2_PERSIST
#define GPLBM_F2_PERSIST 1
#endif

inline bool fused2d_supported(int, int) { return true; }

template <class L, class LH, class S, class C, bool kGen>
struct Fused2D {
  static int launch(const Geo& g, const Coef<C>& K, const StepBufs<S>& b, hipStream_t st) {
    constexpr int TX = 64, TY = GPLBM_F2_TY;
    constexpr int NT = TileShape<TX, TY>::NT;
    auto kernel = k_fused2d<TX, TY, L, LH, S, C, kGen>;
    const int tiles_x = (g.nx + TX - 1) / TX;
    const int tiles_y = (g.ny + TY - 1) / TY;
    const int ntiles = tiles_x * tiles_y;
    static int resident[64] = {0};
#if GPLBM_F2_PERSIST
    const int grid = resident_grid(kernel, NT, ntiles, resident);
#else
    const int grid = (ntiles + kNumXcd - 1) / kNumXcd * kNumXcd;
#endif
    if (grid <= 0) return -1;
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(NT), 0, st, g, K, b, tiles_x, ntiles);
    return 0;
  }
};

}  // namespace gplbm
