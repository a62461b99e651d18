// Fused schedule in 3-D: one kernel per time step n -> n+1, marching in z.
// g runs on D3Q19 or D3Q7 (L), h on D3Q19 or D3Q7 (LH).
//
// A block owns an x-y output tile T of TX x TY nodes and a chunk of ZC planes,
// and computes the tile grown by one node in x and y (the region, BX x BY).
// It walks the planes p = z0-1 .. z1 (one halo plane below and above the
// chunk).  At plane p every thread
//   - pulls h~^n (-> c^n, mu^n) and g~^{n+1} (-> phi^{n+1}),
//   - takes phi^n of planes p-1, p, p+1 from a 3-plane LDS ring (T+2 in x-y)
//     for the gradient, writes phi^{n+1}(p) into a second ring,
//   - runs the h collision of step n.
// The post-collision h* are then streamed inside the block, to three planes:
// the e_z = +1 populations to plane p+1, the in-plane ones to plane p, the
// e_z = -1 ones to plane p-1.  Where the g carry is in registers the h* go to
// an LDS exchange and every node gathers its own contributions from x - e_k
// into three rolling partial sums (one barrier); with the LDS g carry they
// are pushed into a ring of three LDS accumulator planes in ordered passes.
// Because D3Q19 and D3Q7 are numbered by layers of e_z (+1, 0, -1), every
// node's c^{n+1} receives its populations in index order across the three
// planes either way, the order of a pull.
// After plane p, c^{n+1}(p-1) is complete and the threads of T run the g
// collision of step n+1 at plane p-1, on the g~^{n+1} pulled one plane
// earlier (kept in registers, or in LDS where registers are short).
//
// Tiles are x-aligned with the halo columns in extra lanes, and the grid is
// persistent with XCD-ordered passes (tiles.h): every output row is whole
// 128-byte lines (partial-line writes cost about a third of the write
// bandwidth), and neighbouring tiles march in step so that the lines of their
// shared halo are still in the L2 when the second tile reads them.
//
// Addressing: with the plane-major layout f[z][k][y][x] every population a
// thread pulls lies in one of three plane groups (z-1, z, z+1) of Q planes
// each (Qh for h).  Each group is a buffer resource in scalar registers; the
// population plane k*nx*ny is the uniform offset and the (x, y) source the
// per-lane offset, so a load costs no vector address arithmetic.
//
// Zero-flux walls (kWalls): a pull from beyond a wall reads the node's own
// opposite population; the phi^n tiles are loaded with clamped coordinates
// (the mirror ghost) and the phi^{n+1} stencil takes mirrored offsets.  A
// population that bounces at an x or y wall reaches its node from the node's
// own plane, not from the plane below or above, so the gather form keeps the
// index order of the pull sum by taking the e_z = +1 layer of a node's c^{n+1}
// at the node's own plane from a second, parity-buffered exchange of the
// plane below (or the node's own bounced values), and the bounced e_z = -1
// values from the node's own entries there; past a top wall a closing plane
// finishes the last one.
#pragma once

#include "kernels_fused2d.h"
#include "tiles.h"

namespace gplbm {

__device__ __forceinline__ int ring3(int q) { return (q + 6) % 3; }

// Raw buffer access: a resource (base, byte range) held in scalar registers,
// a 32-bit per-lane offset and a 32-bit uniform offset.  Offsets outside the
// range read 0 and drop writes.
constexpr int kBufferFlags = 0x00020000;  // gfx9 buffer descriptor, dword 3

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           kBufferFlags);
}

template <class S>
__device__ __forceinline__ S bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(S) == 8)
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  else
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

// non-temporal store (the written state is not read again in this step)
template <class S>
__device__ __forceinline__ void bstore_nt(S v, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                          uint32_t soff) {
  constexpr int kNT = 2;
  if constexpr (sizeof(S) == 8) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, voff, soff, kNT);
  } else {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b32(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(V, v), r, voff, soff, kNT);
  }
}

// Pulls of the populations of lattice P at z plane zp: population k comes
// from plane group zp - e_z and (x, y) - (e_x, e_y), whose byte offset inside
// a population plane is xyb[1 - e_y][1 - e_x].
template <class P, class S>
__device__ __forceinline__ void fetch_pops(const S* base, int zp, int nz, int plane,
                                           const uint32_t (&xyb)[3][3], S (&v)[P::Q]) {
  const int64_t groupB = int64_t(plane) * P::Q * sizeof(S);
  const uint32_t planeB = uint32_t(plane) * sizeof(S);
  const int zs[3] = {(zp == 0 ? nz - 1 : zp - 1), zp, (zp == nz - 1 ? 0 : zp + 1)};
  __amdgpu_buffer_rsrc_t R[3];
#pragma unroll
  for (int j = 0; j < 3; ++j)
    R[j] = make_rsrc(reinterpret_cast<const char*>(base) + zs[j] * groupB, uint32_t(groupB));
#pragma unroll
  for (int k = 0; k < P::Q; ++k)
    v[k] = bload<S>(R[1 - P::ez[k]], xyb[1 - P::ey[k]][1 - P::ex[k]], k * planeB);
}

// Carry of the pulled g~^{n+1} from its plane to the collision one plane
// later: in registers, or in two LDS buffers (by plane parity) written right
// after the pull, which frees 2Q registers in FP64.
enum class Carry { kRegisters, kLds };

// Zero-flux walls in the z-marching kernels.  A population whose source
// x - e_k lies beyond a wall is the node's own opposite population (halfway
// bounce-back); the gradient stencils use the mirror ghost, which the T+2
// tiles get by loading clamped coordinates along wall axes.
//
// Coordinate of a tile node along one axis: wrapped on a periodic axis,
// clamped (mirror ghost) on a wall axis.
__device__ __forceinline__ int tile_coord(int u, int n, int bc) {
  return bc ? min(max(u, 0), n - 1) : wrap_coord(u, n);
}

// Bit k set when population k of lattice P reaches the node at unwrapped
// coordinates (ux, uy) from beyond an x or a y wall.
template <class P>
__device__ __forceinline__ uint32_t xy_bounce_mask(const Geo& g, int ux, int uy) {
  uint32_t m = 0;
#pragma unroll
  for (int k = 0; k < P::Q; ++k) {
    const int sx = ux - P::ex[k], sy = uy - P::ey[k];
    const bool b = (g.bcx && (sx < 0 || sx >= g.nx)) || (g.bcy && (sy < 0 || sy >= g.ny));
    m |= b ? (1u << k) : 0u;
  }
  return m;
}


template <class L, class S>
struct Fused3DConfig;
// 32-plane z chunks: 11008 tiles at 512^3, 43 passes of the 256 resident
// blocks; 64-plane chunks (two halo planes per 66 instead of per 34) ran
// level in the plain FP64 step (20.06-20.26 against 20.20-20.24 ms) and 3%
// slower in its general instantiation (h^eq,alt 22.1 against 21.3-21.5)
template <>
struct Fused3DConfig<D3Q19, double> {
  static constexpr int TX = 64, TY = 6, ZC = 32;
  static constexpr Carry carry = Carry::kLds;
  static constexpr bool prefetch = false;
};
// FP32: the phi^n tile of the plane after next is fetched into registers
// while a plane is computed (512^3: 9.65-10.0 against 10.6-10.8 ms per step,
// with h on D3Q7 7.28 against 7.52; in FP64 it ran 2% slower, on D3Q7 12%
// slower in FP32 and level in FP64); 64-plane z chunks (9.86-9.92 against
// 9.97-10.01 ms with 32; 2752 tiles at 512^3, 10.75 passes)
template <>
struct Fused3DConfig<D3Q19, float> {
  static constexpr int TX = 64, TY = 12, ZC = 64;
  static constexpr Carry carry = Carry::kRegisters;
  static constexpr bool prefetch = true;
};
// g on D3Q7: 7 populations carried in registers; tile heights measured on
// the 512^3 step (FP64: 12 rows 7.05 ms, 8 rows 7.79, 6 rows 8.36; FP32: 8
// rows 4.05 ms, 12 rows 4.40, 6 rows 4.18); FP32 in 64-plane z chunks (4096
// tiles at 512^3, 16 passes of the 256 resident blocks: 3.97-3.98 against
// 4.05 ms with 32, with walls 5.17 against 5.29; FP64 gained 0.5%)
template <>
struct Fused3DConfig<D3Q7, double> {
  static constexpr int TX = 64, TY = 12, ZC = 32;
  static constexpr Carry carry = Carry::kRegisters;
  static constexpr bool prefetch = false;
};
template <>
struct Fused3DConfig<D3Q7, float> {
  static constexpr int TX = 64, TY = 8, ZC = 64;
  static constexpr Carry carry = Carry::kRegisters;
  static constexpr bool prefetch = false;
};

template <int TX, int TY, int ZC, Carry kCarryMode, bool kPrefetch, class L, class LH, class S,
          class C, bool kGen, bool kWalls>
__global__ void __launch_bounds__((TileShape<TX, TY>::NT))
    k_fused3d(Geo g, Coef<C> Kin, StepBufs<S> b, int tiles_x, int tiles_xy, int ntiles) {
  const Coef<C> K = variant<kGen>(Kin);
  using Shape = TileShape<TX, TY>;
  constexpr int Q = L::Q, QH = LH::Q;
  // e_z layers of the h lattice: +1 at [0, NU), 0 at [NU, NU+NM), -1 after
  constexpr int NU = count_ez<LH>(1), NM = count_ez<LH>(0), ND = count_ez<LH>(-1);
  constexpr int NPASS = NM > NU ? (NM > ND ? NM : ND) : (NU > ND ? NU : ND);
  static_assert(NU + NM + ND == QH, "h lattice must be numbered by layers of e_z");
  constexpr int BX = Shape::BX, BY = Shape::BY;
  constexpr int AX = BX + 2, AY = BY + 2;
  constexpr int NT = Shape::NT;
  constexpr int PHI_PER_THREAD = (AX * AY + NT - 1) / NT;
  constexpr bool kRegs = kCarryMode == Carry::kRegisters;
  // In-block streaming of h*: with the register carry of g the LDS has room
  // for an exchange of the post-collision h* of the plane, which the readers
  // gather from after one barrier, keeping their partial sums of c^{n+1} in
  // registers (g and h on D3Q19 in FP32 spills 8-11 VGPRs doing so and is
  // still faster, 10.0 against 10.6 ms at 512^3); with the LDS carry (FP64
  // D3Q19) they are pushed into an accumulator ring in NPASS ordered passes.
  // Both sum every c^{n+1} in population order.
  constexpr bool kGather = kRegs;
  static_assert(!kWalls || kGather, "walls need the gather form");
  __shared__ C phiA[3][AY][AX];  // phi^n, planes p-1, p, p+1
  __shared__ C phiB[3][BY][BX];  // phi^{n+1}, planes p-2, p-1, p
  // c^{n+1} being accumulated (push passes)
  __shared__ double acc[kGather ? 1 : 3][kGather ? 1 : BY][kGather ? 1 : BX];
  // h* of plane p, moving populations (gather)
  __shared__ C hx[kGather ? QH : 1][kGather ? BY : 1][kGather ? BX : 1];
  // With walls the e_z = +1 layer of the exchange is kept for one more plane
  // (by plane parity): the plane above gathers it after its own barrier, and
  // a node's own values in it are the bounce of its e_z = -1 populations.
  // The plane's two barriers order the reuse of a parity buffer.
  __shared__ C hxu[kWalls ? 2 : 1][kWalls ? NU : 1][kWalls ? BY : 1][kWalls ? BX : 1];
  // pulled g~^{n+1} of the output nodes by plane parity (LDS carry)
  __shared__ C gkeep[kRegs ? 1 : 2][kRegs ? 1 : Q][kRegs ? 1 : TY][kRegs ? 1 : TX];

  int tx, ty;
  bool valid;
  Shape::node(threadIdx.x, tx, ty, valid);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int plane = nx * ny;
  const uint32_t planeB = uint32_t(plane) * sizeof(S);     // one population plane
  const int64_t groupB = int64_t(plane) * Q * sizeof(S);   // one z plane group of g
  const int64_t groupH = int64_t(plane) * QH * sizeof(S);  // one z plane group of h
  const bool wz = kWalls && g.bcz;

  for (int tile = first_tile(); tile < ntiles; tile += gridDim.x) {
    const int chunk = tile / tiles_xy, txy = tile % tiles_xy;
    const int X0 = tile_column(txy, tiles_x, chunk, kWalls) * TX, Y0 = (txy / tiles_x) * TY;
    const int z0 = chunk * ZC, z1 = min(z0 + ZC, nz);

    const int ux = X0 - 1 + tx, uy = Y0 - 1 + ty;
    const bool out = valid && ux < nx && uy < ny && tx >= 1 && tx <= TX && ty >= 1 && ty <= TY;
    // region nodes beyond a wall take no part (with walls only)
    bool active = valid;
    if constexpr (kWalls)
      active = valid && (!g.bcx || (ux >= 0 && ux < nx)) && (!g.bcy || (uy >= 0 && uy < ny));
    const int x = kWalls ? tile_coord(ux, nx, g.bcx) : wrap_coord(ux, nx);
    const int y = kWalls ? tile_coord(uy, ny, g.bcy) : wrap_coord(uy, ny);
    // source offsets wrap also on wall axes: a source beyond a wall is never
    // read (its population bounces), the wrapped address keeps it in range
    const int xo[3] = {x == 0 ? nx - 1 : x - 1, x, x == nx - 1 ? 0 : x + 1};
    const int yo[3] = {(y == 0 ? ny - 1 : y - 1) * nx, y * nx, (y == ny - 1 ? 0 : y + 1) * nx};
    // byte offset, inside a population plane, of the source x - e_k (by e_x, e_y)
    uint32_t xyb[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) xyb[a][c] = uint32_t(yo[a] + xo[c]) * sizeof(S);
    const uint32_t selfB = xyb[1][1];
    // populations arriving from beyond an x or y wall (bit k), and the mirror
    // offsets of the phi^{n+1} stencil
    uint32_t bmh = 0, bmg = 0;
    int xm = -1, xp = 1, ym = -1, yp = 1;
    if constexpr (kWalls) {
      bmh = xy_bounce_mask<LH>(g, ux, uy);
      bmg = xy_bounce_mask<L>(g, ux, uy);
      xm = (g.bcx && ux == 0) ? 0 : -1;
      xp = (g.bcx && ux == nx - 1) ? 0 : 1;
      ym = (g.bcy && uy == 0) ? 0 : -1;
      yp = (g.bcy && uy == ny - 1) ? 0 : 1;
    }
    // phi^n tile positions this thread loads (T+2 in x-y; clamped along wall
    // axes, the mirror ghost)
    uint32_t phi_off[PHI_PER_THREAD];
#pragma unroll
    for (int j = 0; j < PHI_PER_THREAD; ++j) {
      const int l = min((int)threadIdx.x + j * NT, AX * AY - 1);
      const int gx = kWalls ? tile_coord(X0 - 2 + l % AX, nx, g.bcx) : wrap_coord(X0 - 2 + l % AX, nx);
      const int gy = kWalls ? tile_coord(Y0 - 2 + l / AX, ny, g.bcy) : wrap_coord(Y0 - 2 + l / AX, ny);
      phi_off[j] = uint32_t(gy * nx + gx);
    }
    auto fetch_phi = [&](int p, S (&v)[PHI_PER_THREAD]) {
      const int pz = kWalls ? tile_coord(p, nz, g.bcz) : wrap_coord(p, nz);
      const S* src = b.PHI + (int64_t)pz * plane;
#pragma unroll
      for (int j = 0; j < PHI_PER_THREAD; ++j) v[j] = src[phi_off[j]];
    };
    auto put_phi = [&](int p, const S (&v)[PHI_PER_THREAD]) {
#pragma unroll
      for (int j = 0; j < PHI_PER_THREAD; ++j) {
        const int l = threadIdx.x + j * NT;
        if (l < AX * AY) phiA[ring3(p)][l / AX][l % AX] = C(v[j]);
      }
    };
    auto load_phi = [&](int p) {
      S v[PHI_PER_THREAD];
      fetch_phi(p, v);
      put_phi(p, v);
    };
    // first plane: the halo plane below the chunk, or the bottom plane at a
    // z wall
    const int pfirst = (wz && z0 == 0) ? 0 : z0 - 1;
    load_phi(pfirst - 1);
    load_phi(pfirst);
    C g_old[kRegs ? Q : 1];
#pragma unroll
    for (int k = 0; k < (kRegs ? Q : 1); ++k) g_old[k] = C(0);
    // gather: c^{n+1} of this thread's node on planes p-1 and p, partly
    // summed (the e_z = +1 populations arrive one plane early, the e_z = -1
    // ones one plane late, each layer in ascending k)
    const bool inner = valid && tx >= 1 && tx <= TX && ty >= 1 && ty <= TY;
    double acc_dn = 0.0, acc_mid = 0.0;
    double sg_old = 0.0;

    // prefetch: the phi^n tile of the plane after next, in flight in
    // registers while the current plane is computed
    S phi_next[kPrefetch ? PHI_PER_THREAD : 1];
    if constexpr (kPrefetch) fetch_phi(pfirst + 1, phi_next);

    for (int p = pfirst; p <= z1; ++p) {
      // past a top wall: no plane, only the completion of plane nz - 1
      const bool closing = wz && p == nz;
      const bool work = !kWalls || (active && !closing);
      if constexpr (kPrefetch) {
        put_phi(p + 1, phi_next);
        fetch_phi(p + 2, phi_next);
      } else {
        load_phi(p + 1);
      }
      __syncthreads();
      const int zp = wz ? min(p, nz - 1) : wrap_coord(p, nz);
      // all e_z = +1 (-1) sources of this plane lie beyond the bottom (top) wall
      const bool bz_up = wz && p == 0;
      const int sA = ring3(p);
      const bool own_p = p >= z0 && p < z1;

      C hs[QH];
      C g_new[kRegs ? Q : 1];
      double sg = 0.0;
      if (work) {
        S hv[QH], gv[Q];
        if constexpr (!kWalls) {
          fetch_pops<LH, S>(b.H, zp, nz, plane, xyb, hv);
          fetch_pops<L, S>(b.G, zp, nz, plane, xyb, gv);
        } else {
          // pulls; a source beyond a wall gives the node's own opposite
          // population (bounce-back); a plane beyond a z wall is never read
          const bool bz_dn = wz && p == nz - 1;
          const int zs[3] = {wz ? max(zp - 1, 0) : (zp == 0 ? nz - 1 : zp - 1), zp,
                             wz ? min(zp + 1, nz - 1) : (zp == nz - 1 ? 0 : zp + 1)};
          __amdgpu_buffer_rsrc_t RH[3], RG[3];
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            RH[j] = make_rsrc(reinterpret_cast<const char*>(b.H) + zs[j] * groupH, uint32_t(groupH));
            RG[j] = make_rsrc(reinterpret_cast<const char*>(b.G) + zs[j] * groupB, uint32_t(groupB));
          }
#pragma unroll
          for (int k = 0; k < QH; ++k) {
            const bool bz = (LH::ez[k] > 0 && bz_up) || (LH::ez[k] < 0 && bz_dn);
            if (bz || ((bmh >> k) & 1u))
              hv[k] = bload<S>(RH[1], selfB, LH::opp[k] * planeB);
            else
              hv[k] = bload<S>(RH[1 - LH::ez[k]], xyb[1 - LH::ey[k]][1 - LH::ex[k]], k * planeB);
          }
#pragma unroll
          for (int k = 0; k < Q; ++k) {
            const bool bz = (L::ez[k] > 0 && bz_up) || (L::ez[k] < 0 && bz_dn);
            if (bz || ((bmg >> k) & 1u))
              gv[k] = bload<S>(RG[1], selfB, L::opp[k] * planeB);
            else
              gv[k] = bload<S>(RG[1 - L::ez[k]], xyb[1 - L::ey[k]][1 - L::ex[k]], k * planeB);
          }
        }

        C h[QH];
        double c = 0.0;
#pragma unroll
        for (int k = 0; k < QH; ++k) {
          h[k] = C(hv[k]);
          c = k == 0 ? double(hv[k]) : c + double(hv[k]);
        }
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          if constexpr (kRegs) g_new[k] = C(gv[k]);
          sg = k == 0 ? double(gv[k]) : sg + double(gv[k]);
        }
        if constexpr (!kRegs) {
          if (out && own_p) {
#pragma unroll
            for (int k = 0; k < Q; ++k) gkeep[p & 1][k][ty - 1][tx - 1] = C(gv[k]);
          }
        }
        const C phi = phiA[sA][ty + 1][tx + 1];
        const C mu = C(closure(K.q, c, double(phi)));
        auto atA = [&](int dx, int dy, int dz) -> C {
          return phiA[ring3(p + dz)][ty + 1 + dy][tx + 1 + dx];
        };
        C gr[3], n[3];
        gradient_normal<L, C>(atA, K.eps2, gr, n);
        const C sbar = source_moment<C>(K, phi, mu);
        const double phin = sg + 0.5 * double(sbar);
        const C phin_c = C(phin);
        if (active) phiB[sA][ty][tx] = phin_c;
        const C dtphi = phin_c - phi;
        C F[3];
        h_flux<L, C>(K, mu, gr, n, dtphi, K.anti_trapping != 0, F);
        const C lam = h_lambda<C>(K, phi, mu);
        const C cc = C(c);
#pragma unroll
        for (int k = 0; k < QH; ++k) hs[k] = C(S(h_update<LH, C>(K, k, h[k], cc, lam, F)));
        balance_rest<LH, S, C>(hs, c);

        if (out && own_p) {
          const auto Hw = make_rsrc(reinterpret_cast<char*>(b.Hn) + zp * groupH, uint32_t(groupH));
#pragma unroll
          for (int k = 0; k < QH; ++k) bstore_nt<S>(S(hs[k]), Hw, selfB, k * planeB);
          __builtin_nontemporal_store(S(phin_c), &b.PHIn[(int64_t)zp * plane + y * nx + x]);
        }
      }

      const bool up_ok = p + 1 >= z0 && p + 1 < z1, dn_ok = p - 1 >= z0 && p - 1 < z1;
      double acc_up = 0.0;
      if constexpr (kGather && !kWalls) {
        // every region node publishes its moving h*, then each inner node
        // gathers from x - e_k in population order
        if (valid) {
#pragma unroll
          for (int k = 0; k < QH; ++k)
            if (k != LH::REST) hx[k][ty][tx] = hs[k];
        }
        __syncthreads();
        if (inner) {
#pragma unroll
          for (int k = 0; k < QH; ++k) {
            const double v = k == LH::REST ? double(hs[k])
                                           : double(hx[k][ty - LH::ey[k]][tx - LH::ex[k]]);
            if (LH::ez[k] > 0)
              acc_up = k == 0 ? v : acc_up + v;
            else if (LH::ez[k] == 0)
              acc_mid = acc_mid + v;
            else
              acc_dn = acc_dn + v;
          }
        }
      }
      if constexpr (kWalls) {
        // the e_z = +1 layer goes to the parity buffer of plane p, the others
        // to the exchange; then the node's c^{n+1}(p) through its in-plane
        // layer (the e_z = +1 layer from plane p - 1, or bounced) and the
        // e_z = -1 layer of c^{n+1}(p - 1) (from plane p, or bounced: the
        // node's own e_z = +1 values of plane p - 1), each in population order
        const int ub = p & 1, pb = ub ^ 1;
        if (active && !closing) {
#pragma unroll
          for (int k = 0; k < QH; ++k) {
            if (k < NU)
              hxu[ub][k][ty][tx] = hs[k];
            else if (k != LH::REST)
              hx[k][ty][tx] = hs[k];
          }
        }
        __syncthreads();
        if (inner && active) {
          if (!closing) {
            double a = 0.0;
#pragma unroll
            for (int k = 0; k < NU; ++k) {
              const double v = (bz_up || ((bmh >> k) & 1u))
                                   ? double(hs[LH::opp[k]])
                                   : double(hxu[pb][k][ty - LH::ey[k]][tx - LH::ex[k]]);
              a = k == 0 ? v : a + v;
            }
#pragma unroll
            for (int k = NU; k < NU + NM; ++k) {
              double v;
              if (k == LH::REST)
                v = double(hs[k]);
              else if ((bmh >> k) & 1u)
                v = double(hs[LH::opp[k]]);
              else
                v = double(hx[k][ty - LH::ey[k]][tx - LH::ex[k]]);
              a = a + v;
            }
#pragma unroll
            for (int k = NU + NM; k < QH; ++k) {
              const double v = ((bmh >> k) & 1u) ? double(hxu[pb][LH::opp[k]][ty][tx])
                                                 : double(hx[k][ty - LH::ey[k]][tx - LH::ex[k]]);
              acc_dn = acc_dn + v;
            }
            acc_up = a;
          } else {
            // past the top wall every e_z = -1 population of plane nz - 1
            // bounces
#pragma unroll
            for (int k = NU + NM; k < QH; ++k) acc_dn = acc_dn + double(hxu[pb][LH::opp[k]][ty][tx]);
          }
        }
      }
      // push form: in-block streaming of h* into the accumulator ring, NPASS
      // passes: pass j carries population j (e_z=+1, to plane p+1),
      // population NU+j (e_z=0, to plane p) and population NU+NM+j (e_z=-1,
      // to plane p-1)
#pragma unroll
      for (int j = 0; j < (kGather ? 0 : NPASS); ++j) {
        if (j < NU && up_ok) {
          const int k = j;
          const int tx2 = tx + LH::ex[k], ty2 = ty + LH::ey[k];
          if (valid && tx2 >= 1 && tx2 <= TX && ty2 >= 1 && ty2 <= TY) {
            double& a = acc[ring3(p + 1)][ty2][tx2];
            a = k == 0 ? double(hs[k]) : a + double(hs[k]);
          }
        }
        if (j < NM && own_p) {
          const int k = NU + j;
          const int tx2 = tx + LH::ex[k], ty2 = ty + LH::ey[k];
          if (valid && tx2 >= 1 && tx2 <= TX && ty2 >= 1 && ty2 <= TY) {
            double& a = acc[sA][ty2][tx2];
            a = a + double(hs[k]);
          }
        }
        if (j < ND && dn_ok) {
          const int k = NU + NM + j;
          const int tx2 = tx + LH::ex[k], ty2 = ty + LH::ey[k];
          if (valid && tx2 >= 1 && tx2 <= TX && ty2 >= 1 && ty2 <= TY) {
            double& a = acc[ring3(p - 1)][ty2][tx2];
            a = a + double(hs[k]);
          }
        }
        __syncthreads();
      }

      // g collision of step n+1 at plane p-1
      if (out && dn_ok) {
        const int zq = wrap_coord(p - 1, nz);
        const int sB = ring3(p - 1);
        const double c1 = kGather ? acc_dn : acc[kGather ? 0 : sB][ty][tx];
        const C phi1 = phiB[sB][ty][tx];
        const C mu1 = C(closure(K.q, c1, double(phi1)));
        const int zm = (wz && p - 1 == 0) ? 0 : -1, zpl = (wz && p - 1 == nz - 1) ? 0 : 1;
        auto atB = [&](int dx, int dy, int dz) -> C {
          if constexpr (kWalls) {
            const int ox = dx < 0 ? xm : (dx > 0 ? xp : 0);
            const int oy = dy < 0 ? ym : (dy > 0 ? yp : 0);
            const int oz = dz < 0 ? zm : (dz > 0 ? zpl : 0);
            return phiB[ring3(p - 1 + oz)][ty + oy][tx + ox];
          } else {
            return phiB[ring3(p - 1 + dz)][ty + dy][tx + dx];
          }
        };
        C gr1[3], n1[3];
        gradient_normal<L, C>(atB, K.eps2, gr1, n1);
        C G[Q];
        phi_sources<L, C>(K, phi1, mu1, n1, G);
        const auto Gw = make_rsrc(reinterpret_cast<char*>(b.Gn) + zq * groupB, uint32_t(groupB));
        if constexpr (sizeof(S) < sizeof(double)) {
          // storage narrower than double: the zeroth moment of the stored g
          // is balanced through the rest population (balance_g_rest), each
          // moving population stored as soon as it is computed
          // sg_old: the double sum of these g, taken when they were pulled
          double s = 0.0;
#pragma unroll
          for (int k = 0; k < Q; ++k) {
            C gk;
            if constexpr (kRegs)
              gk = g_old[k];
            else
              gk = gkeep[(p - 1) & 1][k][ty - 1][tx - 1];
            if (k == L::REST) continue;
            const S v = S(g_collide<L, C>(K, k, gk, phi1, G[k]));
            bstore_nt<S>(v, Gw, selfB, k * planeB);
            s = s + double(v);
          }
          const double wg = K.omega_g_d;
          const double m0 = ((1.0 - wg) * sg_old + wg * double(phi1)) +
                            (1.0 - 0.5 * wg) * double(source_moment<C>(K, phi1, mu1));
          bstore_nt<S>(S(m0 - s), Gw, selfB, L::REST * planeB);
        } else {
#pragma unroll
          for (int k = 0; k < Q; ++k) {
            C gk;
            if constexpr (kRegs)
              gk = g_old[k];
            else
              gk = gkeep[(p - 1) & 1][k][ty - 1][tx - 1];
            bstore_nt<S>(S(g_collide<L, C>(K, k, gk, phi1, G[k])), Gw, selfB, k * planeB);
          }
        }
      }
      if constexpr (kRegs) {
#pragma unroll
        for (int k = 0; k < Q; ++k) g_old[k] = g_new[k];
      }
      sg_old = sg;
      if constexpr (kWalls) {
        acc_dn = acc_up;
      } else if constexpr (kGather) {
        acc_dn = acc_mid;
        acc_mid = acc_up;
      }
    }
    __syncthreads();  // the LDS rings are refilled by the next tile
  }
}

// 32-bit offsets inside a z plane group: Q * nx * ny * 8 bytes must fit
// (checked for the larger lattice, 19 populations); any boundary.
inline bool fused3d_supported(int nx, int ny, int nz, const int*) {
  return (int64_t)nx * ny * 19 * 8 < ((int64_t)1 << 32) && (int64_t)nx * ny * nz < ((int64_t)1 << 31);
}

// Domains with a zero-flux wall take the gather form of the in-block
// streaming, so FP64 on D3Q19 carries g in registers there, on 64 x 5 tiles
// (one 8-wave block per CU; 512^3: 20.25 ms against 20.08 ms periodic).
template <class L, class S>
struct Fused3DWallConfig : Fused3DConfig<L, S> {};
template <>
struct Fused3DWallConfig<D3Q19, double> {
  static constexpr int TX = 64, TY = 5, ZC = 32;
  static constexpr Carry carry = Carry::kRegisters;
  static constexpr bool prefetch = false;
};
// FP32 on D3Q19 with walls: 64 x 9 tiles (12 waves, 142 VGPRs, no spill),
// 11.01 ms per 512^3 step against 11.33 on the 64 x 12 tiles of the
// periodic grid (which spill about 25 VGPRs with walls; the order was the
// reverse before the tile columns turned per chunk, 12.43 against 11.95),
// 32-plane chunks, and without the prefetch of the periodic grid (which
// spills 45 VGPRs there: 19.0 against 16.3 ms)
template <>
struct Fused3DWallConfig<D3Q19, float> : Fused3DConfig<D3Q19, float> {
  static constexpr int TY = 9, ZC = 32;
  static constexpr bool prefetch = false;
};

template <class L, class LH, class S, class C, bool kGen>
struct Fused3D {
  template <class Cfg, bool kWalls>
  static int run(const Geo& g, const Coef<C>& K, const StepBufs<S>& b, hipStream_t st) {
    constexpr int TX = Cfg::TX, TY = Cfg::TY, ZC = Cfg::ZC;
    constexpr int NT = TileShape<TX, TY>::NT;
    auto kernel = k_fused3d<TX, TY, ZC, Cfg::carry, Cfg::prefetch, L, LH, S, C, kGen, kWalls>;
    const int tiles_x = (g.nx + TX - 1) / TX;
    const int tiles_y = (g.ny + TY - 1) / TY;
    const int chunks = (g.nz + ZC - 1) / ZC;
    const int tiles_xy = tiles_x * tiles_y;
    const int ntiles = tiles_xy * chunks;
    static int resident[64] = {0};
    const int grid = resident_grid(kernel, NT, ntiles, resident);
    if (grid <= 0) return -1;
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(NT), 0, st, g, K, b, tiles_x, tiles_xy, ntiles);
    return 0;
  }
  static int launch(const Geo& g, const Coef<C>& K, const StepBufs<S>& b, hipStream_t st) {
    if (g.bcx || g.bcy || g.bcz) return run<Fused3DWallConfig<L, S>, true>(g, K, b, st);
    return run<Fused3DConfig<L, S>, false>(g, K, b, st);
  }
};

template <class L, class LH, class S, class C, bool kGen>
struct FusedLaunch {
  static int launch(const Geo& g, const Coef<C>& K, const StepBufs<S>& b, hipStream_t st) {
    if constexpr (L::D == 2)
      return Fused2D<L, LH, S, C, kGen>::launch(g, K, b, st);
    else
      return Fused3D<L, LH, S, C, kGen>::launch(g, K, b, st);
  }
};

}  // namespace gplbm
