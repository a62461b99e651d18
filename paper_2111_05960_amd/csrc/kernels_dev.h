// Reduced-precision storage of the state on any lattice: the Q - 1 moving
// populations of each distribution are stored as FP16 or BF16 deviations from the local
// equilibrium of the node that wrote them, the rest populations, phi and
// Lambda = gamma D(phi) mu as FP32.  Collision arithmetic is FP32; the moments
// (c, phi) and the closure mu(c, phi) are FP64.
//
//   g: stored delta_k = S (g*_k - w_k phi(y))     (phi of the writing node y)
//   h: stored delta_k = S (h*_k - w_k Lambda(y))  (Lambda of the writing node)
// with S = 2^12 for FP16 (keeps the small deviations in the normal range) and
// S = 1 for BF16; rounding is round-to-nearest-even.  A reader decodes
// f = ref + delta / S with the reference of the source node, which is
// available to it (phi and Lambda are fields of the state).
//
// Solute mass: the writer sets the rest population of h so that the decoded
// populations it leaves behind sum exactly (in FP64, then one FP32 rounding)
// to the c it received - the collision conserves c exactly in arithmetic, so
// this only removes the rounding of the 16-bit encodings from the balance.
//
// Layout of one distribution: moving populations u16[z][m][y][x] (m = k
// before the rest vector, k - 1 after it), then the rest populations
// f32[z][y][x].  Every kernel takes the lattices of g and h as template
// arguments.
#pragma once

#include "kernels_fused3d.h"

namespace gplbm {

struct F16Codec {
  static constexpr float kScale = 4096.0f, kInv = 1.0f / 4096.0f;
  __device__ static uint16_t enc(float v) { return __builtin_bit_cast(uint16_t, (_Float16)v); }
  __device__ static float dec(uint16_t u) { return (float)__builtin_bit_cast(_Float16, u); }
};
struct BF16Codec {
  static constexpr float kScale = 1.0f, kInv = 1.0f;
  __device__ static uint16_t enc(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
  __device__ static float dec(uint16_t u) { return (float)__builtin_bit_cast(__bf16, u); }
};

// one distribution in the deviation format
struct DevDist {
  uint16_t* mov;
  float* rest;
};
struct DevState {
  DevDist G, H;
  float* PHI;
  float* LAM;
};
struct DevStep {
  DevState cur;  // G = g~*^n, H = h~*^{n-1}, PHI = phi^n, LAM = Lambda^{n-1}
  DevState nxt;  // written: G = g~*^{n+1}, H = h~*^n, PHI = phi^{n+1}, LAM = Lambda^n
};

using LD = D3Q19;    // default lattice of the per-node helpers
constexpr int kMov = 18;  // the most moving populations per node (D3Q19)

// slot of moving population k among the Q - 1 of lattice L
template <class L = LD>
__device__ __forceinline__ constexpr int mslot(int k) { return k < L::REST ? k : k - 1; }

// opposite populations share a weight (a bounced code decodes with w_k)
template <class L>
constexpr bool symmetric_weights() {
  for (int k = 0; k < L::Q; ++k)
    if (L::w[k] != L::w[L::opp[k]]) return false;
  return true;
}
static_assert(symmetric_weights<D3Q19>() && symmetric_weights<D3Q7>() &&
              symmetric_weights<D2Q9>() && symmetric_weights<D2Q5>(), "w_opp(k) = w_k");

// slot of plane q in a ring of four planes (q >= -8)
__device__ __forceinline__ int ring4(int q) { return (q + 8) & 3; }

template <class L = LD>
__device__ __forceinline__ int64_t mov_index(const Geo& g, int k, int x, int y, int z) {
  const int64_t plane = (int64_t)g.nx * g.ny;
  return ((int64_t)z * (L::Q - 1) + mslot<L>(k)) * plane + (int64_t)y * g.nx + x;
}

template <class Codec>
__device__ __forceinline__ float dev_decode(uint16_t raw, float ref) {
  return ref + Codec::dec(raw) * Codec::kInv;
}
template <class Codec>
__device__ __forceinline__ uint16_t dev_encode(float v, float ref) {
  return Codec::enc((v - ref) * Codec::kScale);
}

// Pull of population k at (x, y, z) from a distribution in the deviation
// format; ref is the field (phi for g, Lambda for h) of the source node.
template <class Codec, class L = LD>
__device__ __forceinline__ float pull_dev(const Geo& g, const DevDist& d, const float* reff, int k,
                                          int x, int y, int z) {
  if (k == L::REST) return d.rest[node_index(g, x, y, z)];
  int sx = x, sy = y, sz = z;
  const bool in = pull_axis(sx, L::ex[k], g.nx, g.bcx) && pull_axis(sy, L::ey[k], g.ny, g.bcy) &&
                  pull_axis(sz, L::ez[k], g.nz, g.bcz);
  const int kk = in ? k : L::opp[k];
  if (!in) sx = x, sy = y, sz = z;
  const float ref = float(L::w[kk]) * reff[node_index(g, sx, sy, sz)];
  return dev_decode<Codec>(d.mov[mov_index<L>(g, kk, sx, sy, sz)], ref);
}

// Encode the post-collision h of one node with the mass balance of the rest
// population; hdec receives the decoded values (what readers will see).
template <class Codec, class L = LD>
__device__ __forceinline__ void encode_h(const float hs[L::Q], float lam, double c_in,
                                         uint16_t enc[L::Q], float hdec[L::Q]) {
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    if (k == L::REST) continue;
    const float ref = float(L::w[k]) * lam;
    enc[k] = dev_encode<Codec>(hs[k], ref);
    hdec[k] = dev_decode<Codec>(enc[k], ref);
    s = s + double(hdec[k]);
  }
  hdec[L::REST] = float(c_in - s);
}

template <class Codec, class L = LD>
__device__ __forceinline__ void encode_g(const float gs[L::Q], float phi, uint16_t enc[L::Q],
                                         float gdec[L::Q]) {
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    if (k == L::REST) {
      gdec[k] = gs[k];
      continue;
    }
    const float ref = float(L::w[k]) * phi;
    enc[k] = dev_encode<Codec>(gs[k], ref);
    gdec[k] = dev_decode<Codec>(enc[k], ref);
  }
}

struct DevGlobalPhi {
  const Geo& g;
  const float* __restrict__ f;
  int x, y, z;
  __device__ float operator()(int dx, int dy, int dz) const {
    return f[node_index(g, stencil_axis(x + dx, g.nx, g.bcx), stencil_axis(y + dy, g.ny, g.bcy),
                        stencil_axis(z + dz, g.nz, g.bcz))];
  }
};

// ---------------------------------------------------------------------------
// Initialisation: first Lambda^0 and phi^0 as FP32 fields, then the
// populations (h~^0 scattered to the slots the first pull reads, encoded with
// the reference of the slot's node).

__global__ void __launch_bounds__(256) k_dev_init_fields(Geo g, Coef<float> K,
                                                         const double* __restrict__ phi0,
                                                         const double* __restrict__ c0,
                                                         DevState s) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t i = node_index(g, x, y, z);
  const float phi = float(phi0[i]);
  const float mu0 = float(closure(K.q, c0[i], double(phi)));
  s.PHI[i] = phi;
  s.LAM[i] = h_lambda<float>(K, phi, mu0);
}

template <class Codec, class L, class LH>
__global__ void __launch_bounds__(256) k_dev_init(Geo g, Coef<float> K,
                                                  const double* __restrict__ c0, DevState s) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t i = node_index(g, x, y, z);
  const float phi = s.PHI[i];
  const double cin = c0[i];
  float gr[3], n[3];
  gradient_normal<L, float>(DevGlobalPhi{g, s.PHI, x, y, z}, K.eps2, gr, n);
  const float mu0 = float(closure(K.q, cin, double(phi)));
  float G0[L::Q];
  phi_sources<L, float>(K, phi, mu0, n, G0);
  float F[3];
  h_flux<L, float>(K, mu0, gr, n, 0.0f, false, F);
  const float lam = s.LAM[i];
  // h~^0, encoded for the slot (x - e_k, k) or (x, opp k) at a wall
  double c = 0.0;
#pragma unroll
  for (int k = 0; k < LH::Q; ++k) {
    const float hv = h_initial<LH, float>(K, k, float(cin), lam, F);
    float dec;
    if (k == LH::REST) {
      s.H.rest[i] = hv;
      dec = hv;
    } else {
      int dx = x, dy = y, dz = z;
      const bool in = pull_axis(dx, LH::ex[k], g.nx, g.bcx) &&
                      pull_axis(dy, LH::ey[k], g.ny, g.bcy) &&
                      pull_axis(dz, LH::ez[k], g.nz, g.bcz);
      const int kk = in ? k : LH::opp[k];
      if (!in) dx = x, dy = y, dz = z;
      const float ref = float(LH::w[kk]) * s.LAM[node_index(g, dx, dy, dz)];
      const uint16_t e = dev_encode<Codec>(hv, ref);
      s.H.mov[mov_index<LH>(g, kk, dx, dy, dz)] = e;
      dec = dev_decode<Codec>(e, ref);
    }
    c = k == 0 ? double(dec) : c + double(dec);
  }
  // collision of g at time 0 with c^0 = sum of the decoded h~^0
  const float mu = float(closure(K.q, c, double(phi)));
  float Gk[L::Q], gs[L::Q];
  phi_sources<L, float>(K, phi, mu, n, Gk);
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    const float g0 = float(L::w[k]) * phi - 0.5f * G0[k];
    gs[k] = g_collide<L, float>(K, k, g0, phi, Gk[k]);
  }
  uint16_t enc[L::Q];
  float gdec[L::Q];
  encode_g<Codec, L>(gs, phi, enc, gdec);
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    if (k == L::REST)
      s.G.rest[i] = gdec[k];
    else
      s.G.mov[mov_index<L>(g, k, x, y, z)] = enc[k];
  }
}

// ---------------------------------------------------------------------------
// Split schedule in the deviation format (any boundaries).

template <class Codec, class L, class LH>
__global__ void __launch_bounds__(256) k_dev_split_h(Geo g, Coef<float> K, DevStep b) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t i = node_index(g, x, y, z);
  float h[LH::Q];
  double c = 0.0;
#pragma unroll
  for (int k = 0; k < LH::Q; ++k) {
    h[k] = pull_dev<Codec, LH>(g, b.cur.H, b.cur.LAM, k, x, y, z);
    c = k == 0 ? double(h[k]) : c + double(h[k]);
  }
  const float phi = b.cur.PHI[i];
  const float mu = float(closure(K.q, c, double(phi)));
  float gr[3], n[3];
  gradient_normal<L, float>(DevGlobalPhi{g, b.cur.PHI, x, y, z}, K.eps2, gr, n);
  const float sbar = source_moment<float>(K, phi, mu);
  double sg = 0.0;
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    const double v = double(pull_dev<Codec, L>(g, b.cur.G, b.cur.PHI, k, x, y, z));
    sg = k == 0 ? v : sg + v;
  }
  const float phin = float(sg + 0.5 * double(sbar));
  float F[3];
  h_flux<L, float>(K, mu, gr, n, phin - phi, K.anti_trapping != 0, F);
  const float lam = h_lambda<float>(K, phi, mu);
  const float cc = float(c);
  float hs[LH::Q];
#pragma unroll
  for (int k = 0; k < LH::Q; ++k)
    hs[k] = h_update<LH, float>(K, k, h[k], cc, lam, F);
  uint16_t enc[LH::Q];
  float hdec[LH::Q];
  encode_h<Codec, LH>(hs, lam, c, enc, hdec);
#pragma unroll
  for (int k = 0; k < LH::Q; ++k) {
    if (k == LH::REST)
      b.nxt.H.rest[i] = hdec[k];
    else
      b.nxt.H.mov[mov_index<LH>(g, k, x, y, z)] = enc[k];
  }
  b.nxt.LAM[i] = lam;
  b.nxt.PHI[i] = phin;
}

template <class Codec, class L, class LH>
__global__ void __launch_bounds__(256) k_dev_split_g(Geo g, Coef<float> K, DevStep b) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t i = node_index(g, x, y, z);
  double c = 0.0;
#pragma unroll
  for (int k = 0; k < LH::Q; ++k) {
    const double v = double(pull_dev<Codec, LH>(g, b.nxt.H, b.nxt.LAM, k, x, y, z));
    c = k == 0 ? v : c + v;
  }
  const float phi = b.nxt.PHI[i];
  const float mu = float(closure(K.q, c, double(phi)));
  float gr[3], n[3];
  gradient_normal<L, float>(DevGlobalPhi{g, b.nxt.PHI, x, y, z}, K.eps2, gr, n);
  float G[L::Q], gs[L::Q];
  phi_sources<L, float>(K, phi, mu, n, G);
  double sg = 0.0;
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    const float gk = pull_dev<Codec, L>(g, b.cur.G, b.cur.PHI, k, x, y, z);
    sg = k == 0 ? double(gk) : sg + double(gk);
    gs[k] = g_collide<L, float>(K, k, gk, phi, G[k]);
  }
  uint16_t enc[L::Q];
  float gdec[L::Q];
  encode_g<Codec, L>(gs, phi, enc, gdec);
  balance_g_rest<L, float, float>(K, gdec, sg, phi, source_moment<float>(K, phi, mu));
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    if (k == L::REST)
      b.nxt.G.rest[i] = gdec[k];
    else
      b.nxt.G.mov[mov_index<L>(g, k, x, y, z)] = enc[k];
  }
}

// read-out and diagnostics in the deviation format
template <class Codec, class L>
__global__ void __launch_bounds__(256) k_dev_fields(Geo g, ClosureK q, DevState s,
                                                    double* phi_out, double* c_out,
                                                    double* mu_out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t i = node_index(g, x, y, z);
  double c = 0.0;
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    const double v = double(pull_dev<Codec, L>(g, s.H, s.LAM, k, x, y, z));
    c = k == 0 ? v : c + v;
  }
  const double phi = double(s.PHI[i]);
  if (phi_out) phi_out[i] = phi;
  if (c_out) c_out[i] = c;
  if (mu_out) mu_out[i] = closure(q, c, phi);
}

template <class Codec, class L>
__global__ void __launch_bounds__(kDiagThreads) k_dev_diag_partial(Geo g, DevState s,
                                                                   double* __restrict__ part) {
  double v[kDiagVals] = {0.0, 0.0, 0.0, 0.0, INFINITY, -INFINITY, 0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.N; i += stride) {
    const int x = int(i % g.nx);
    const int y = int((i / g.nx) % g.ny);
    const int z = int(i / ((int64_t)g.nx * g.ny));
    double c = 0.0;
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      const double hv = double(pull_dev<Codec, L>(g, s.H, s.LAM, k, x, y, z));
      c = k == 0 ? hv : c + hv;
    }
    const double phi = double(s.PHI[i]);
    v[0] = v[0] + c;
    v[1] = v[1] + (1.0 - phi);
    v[2] = v[2] + (phi < 0.5 ? 1.0 : 0.0);
    v[3] = v[3] + phi;
    v[4] = fmin(v[4], phi);
    v[5] = fmax(v[5], phi);
    if (!isfinite(c) || !isfinite(phi)) v[6] = 1.0;
  }
  diag_block_reduce(v);
  if (threadIdx.x == 0)
    for (int j = 0; j < kDiagVals; ++j) part[blockIdx.x * kDiagVals + j] = v[j];
}

// ---------------------------------------------------------------------------
// output rows per tile of the fused deviation kernel (64 x 13 outputs, 1024
// threads at 4 waves per SIMD)
#ifndef GPLBM_DEV_TY
#define GPLBM_DEV_TY 13
#endif

// Fused z-marching schedule in the deviation format, periodic or with
// zero-flux walls.  Same structure as k_fused3d (x-aligned tiles, persistent
// grid, g carry in registers); in addition an LDS ring holds Lambda^{n-1} on
// T+2 for the h references, and the phi^n ring serves the g references.
//
// Walls (kWalls, any axis): a pull whose source lies beyond a wall reads the
// node's own opposite population, decoded with the node's own reference; the
// T+2 tiles are loaded with clamped coordinates (the mirror ghost of the
// gradient); the phi^{n+1} stencil of the g collision takes mirrored offsets;
// and the in-block h streaming keeps the index order of the pull sum: a node
// gathers the e_z = +1 layer of its c^{n+1} at its own plane, from the
// exchange of the plane below (kept one plane longer) or its own bounced
// values, takes the bounced e_z = -1 values from its own entries in that
// exchange, and a closing plane past a top wall finishes the last plane.

__device__ __forceinline__ uint16_t bload16(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(uint16_t, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore16_nt(uint16_t v, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                            uint32_t soff) {
  using V = decltype(__builtin_amdgcn_raw_buffer_load_b16(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(V, v), r, voff, soff, 2);
}

template <int TX, int TY, int ZC, class Codec, class LG, class LH, bool kGen, bool kWalls>
__global__ void __launch_bounds__((TileShape<TX, TY>::NT))
    k_dev_fused3d(Geo g, Coef<float> Kin, DevStep b, int tiles_x, int tiles_xy, int ntiles) {
  const Coef<float> K = variant<kGen>(Kin);
  using Shape = TileShape<TX, TY>;
  constexpr int Q = LG::Q;  // g lattice (D3Q19 or D3Q7)
  constexpr int BX = Shape::BX, BY = Shape::BY;
  constexpr int AX = BX + 2, AY = BY + 2;
  constexpr int NT = Shape::NT;
  // Rings of four planes and a double-buffered exchange, so that one barrier
  // per plane orders every LDS access: the tile of plane p + 2 is loaded, and
  // the next plane's exchange written, while other waves still read the
  // planes of p (see the hazards noted at the barrier).
  __shared__ float phiA[4][AY][AX];          // phi^n, planes p-1 .. p+2
  __shared__ float lamA[4][AY][AX];          // Lambda^{n-1}, planes p-1 .. p+2
  __shared__ float phiB[4][BY][BX];          // phi^{n+1}, planes p-3 .. p
  constexpr int QH = LH::Q;  // h lattice (D3Q19 or D3Q7)
  // e_z layers of the h lattice: +1 at [0, NU), 0 at [NU, NU + NM), -1 after
  constexpr int NU = count_ez<LH>(1), NM = count_ez<LH>(0);
  // Exchange of plane p: the 16-bit codes of the moving h*^n and Lambda^n,
  // their reference.  Periodic: every moving population in hxe and Lambda in
  // hxl, by plane parity.  Walls: the e_z = +1 layer in hxu and Lambda in hxl
  // by plane modulo 3 (the plane above gathers that layer after its own
  // barrier, and a node's own entries there are the bounce of its e_z = -1
  // populations: with one barrier per plane a buffer is rewritten two planes
  // after it was read), the other moving populations in hxe by parity.
  static_assert(!kWalls || LH::REST == NU, "the rest vector opens the in-plane layer");
  constexpr int NXE = kWalls ? QH - 1 - NU : QH - 1;
  __shared__ uint16_t hxe[2][NXE][BY][BX];
  __shared__ uint16_t hxu[kWalls ? 3 : 1][kWalls ? NU : 1][kWalls ? BY : 1][kWalls ? BX : 1];
  __shared__ float hxl[kWalls ? 3 : 2][BY][BX];

  int tx, ty;
  bool valid;
  Shape::node(threadIdx.x, tx, ty, valid);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int plane = nx * ny;
  const uint32_t planeB = uint32_t(plane) * 2u;            // one 16-bit population plane
  const int64_t groupB = int64_t(plane) * (Q - 1) * 2;        // one z group of moving g populations
  const int64_t groupBH = int64_t(plane) * (QH - 1) * 2;   // one z group of moving h populations
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
  // read (its population bounces), the wrapped address only keeps it in range
  const int xo[3] = {x == 0 ? nx - 1 : x - 1, x, x == nx - 1 ? 0 : x + 1};
  const int yo[3] = {(y == 0 ? ny - 1 : y - 1) * nx, y * nx, (y == ny - 1 ? 0 : y + 1) * nx};
  uint32_t xyb[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) xyb[a][c] = uint32_t(yo[a] + xo[c]) * 2u;
  const uint32_t selfB = xyb[1][1];
  const int self_xy = y * nx + x;
  // populations arriving from beyond an x or y wall (bit k), and the mirror
  // offsets of the phi^{n+1} stencil
  uint32_t bmh = 0, bmg = 0;
  int xm = -1, xp = 1, ym = -1, yp = 1;
  if constexpr (kWalls) {
    bmh = xy_bounce_mask<LH>(g, ux, uy);
    bmg = xy_bounce_mask<LG>(g, ux, uy);
    xm = (g.bcx && ux == 0) ? 0 : -1;
    xp = (g.bcx && ux == nx - 1) ? 0 : 1;
    ym = (g.bcy && uy == 0) ? 0 : -1;
    yp = (g.bcy && uy == ny - 1) ? 0 : 1;
  }

  auto load_tiles = [&](int p) {
    const int64_t zoff = (int64_t)(kWalls ? tile_coord(p, nz, g.bcz) : wrap_coord(p, nz)) * plane;
    for (int l = threadIdx.x; l < AX * AY; l += NT) {
      const int lx = l % AX, ly = l / AX;
      const int gx = kWalls ? tile_coord(X0 - 2 + lx, nx, g.bcx) : wrap_coord(X0 - 2 + lx, nx);
      const int gy = kWalls ? tile_coord(Y0 - 2 + ly, ny, g.bcy) : wrap_coord(Y0 - 2 + ly, ny);
      phiA[ring4(p)][ly][lx] = b.cur.PHI[zoff + gy * nx + gx];
      lamA[ring4(p)][ly][lx] = b.cur.LAM[zoff + gy * nx + gx];
    }
  };
  // first plane: the halo plane below the chunk, or the bottom plane at a z wall
  const int pfirst = (wz && z0 == 0) ? 0 : z0 - 1;
  load_tiles(pfirst - 1);
  load_tiles(pfirst);
  load_tiles(pfirst + 1);
  __syncthreads();

  float g_old[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) g_old[k] = 0.0f;
  // c^{n+1} of this thread's node on planes p - 1 and p, partly summed: the
  // e_z = +1 populations arrive one plane early, the e_z = -1 ones one plane
  // late, each group gathered in ascending k
  const bool inner = valid && tx >= 1 && tx <= TX && ty >= 1 && ty <= TY;
  double acc_dn = 0.0, acc_mid = 0.0;

  for (int p = pfirst; p <= z1; ++p) {
    // past a top wall: no plane, only the completion of plane nz - 1
    const bool closing = wz && p == nz;
    const int zp = wz ? min(p, nz - 1) : wrap_coord(p, nz);
    int zo[3];
    if (wz) {
      // a plane beyond the wall is never read (its populations bounce)
      zo[0] = max(zp - 1, 0);
      zo[1] = zp;
      zo[2] = min(zp + 1, nz - 1);
    } else {
      zo[0] = zp == 0 ? nz - 1 : zp - 1;
      zo[1] = zp;
      zo[2] = zp == nz - 1 ? 0 : zp + 1;
    }
    // all e_z = +1 (-1) sources of this plane lie beyond the bottom (top) wall
    const bool bz_up = wz && p == 0, bz_dn = wz && p == nz - 1;
    __amdgpu_buffer_rsrc_t Hz[3], Gz[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Hz[j] = make_rsrc(reinterpret_cast<const char*>(b.cur.H.mov) + zo[j] * groupBH, uint32_t(groupBH));
      Gz[j] = make_rsrc(reinterpret_cast<const char*>(b.cur.G.mov) + zo[j] * groupB, uint32_t(groupB));
    }
    const int64_t selfnode = (int64_t)zp * plane + self_xy;
    const int sA = ring4(p);

    float g_new[Q];
    float hdec[QH];
    float phin = 0.0f, lam = 0.0f;
    uint16_t enc[QH];
    if (!kWalls || (active && !closing)) {
      // pulls, decoded with the reference of the source node (LDS tiles), or
      // of the node itself for a population bounced back at a wall
      float h[QH];
      double c = 0.0, sg = 0.0;
      // populations bounced at a wall (bits k); a wavefront with none (all but
      // those of the tiles at a wall) takes the plain pulls
      uint32_t bh = 0u, bg = 0u;
      bool plain = true;
      if constexpr (kWalls) {
        bh = bmh | (bz_up ? ez_mask<LH>(1) : 0u) | (bz_dn ? ez_mask<LH>(-1) : 0u);
        bg = bmg | (bz_up ? ez_mask<LG>(1) : 0u) | (bz_dn ? ez_mask<LG>(-1) : 0u);
        plain = __builtin_amdgcn_ballot_w64((bh | bg) != 0u) == 0u;
      }
      if (!plain) {
        // Every pull first reads its neighbour (a wrapped address where x -
        // e_k lies beyond a wall: read, never used), then a lane with bounced
        // populations replaces those codes by its own opposite ones, and each
        // code decodes against the reference of the node that wrote it
        // (w_opp(k) = w_k): one batch of loads and no branch per population
        uint16_t ch[QH], cg[Q];
#pragma unroll
        for (int k = 0; k < QH; ++k)
          ch[k] = k == LH::REST ? uint16_t(0)
                                : bload16(Hz[1 - LH::ez[k]], xyb[1 - LH::ey[k]][1 - LH::ex[k]],
                                          mslot<LH>(k) * planeB);
#pragma unroll
        for (int k = 0; k < Q; ++k)
          cg[k] = k == LG::REST ? uint16_t(0)
                                : bload16(Gz[1 - LG::ez[k]], xyb[1 - LG::ey[k]][1 - LG::ex[k]],
                                          mslot<LG>(k) * planeB);
        if ((bh | bg) != 0u) {
#pragma unroll
          for (int k = 0; k < QH; ++k)
            if (k != LH::REST && ((bh >> k) & 1u))
              ch[k] = bload16(Hz[1], selfB, mslot<LH>(LH::opp[k]) * planeB);
#pragma unroll
          for (int k = 0; k < Q; ++k)
            if (k != LG::REST && ((bg >> k) & 1u))
              cg[k] = bload16(Gz[1], selfB, mslot<LG>(LG::opp[k]) * planeB);
        }
        const float lam_own = lamA[sA][ty + 1][tx + 1], phi_own = phiA[sA][ty + 1][tx + 1];
#pragma unroll
        for (int k = 0; k < QH; ++k) {
          float v;
          if (k == LH::REST) {
            v = b.cur.H.rest[selfnode];
          } else {
            const float src = lamA[ring4(p - LH::ez[k])][ty + 1 - LH::ey[k]][tx + 1 - LH::ex[k]];
            v = dev_decode<Codec>(ch[k], float(LH::w[k]) * (((bh >> k) & 1u) ? lam_own : src));
          }
          h[k] = v;
          c = k == 0 ? double(v) : c + double(v);
        }
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          float v;
          if (k == LG::REST) {
            v = b.cur.G.rest[selfnode];
          } else {
            const float src = phiA[ring4(p - LG::ez[k])][ty + 1 - LG::ey[k]][tx + 1 - LG::ex[k]];
            v = dev_decode<Codec>(cg[k], float(LG::w[k]) * (((bg >> k) & 1u) ? phi_own : src));
          }
          g_new[k] = v;
          sg = k == 0 ? double(v) : sg + double(v);
        }
      } else {
#pragma unroll
        for (int k = 0; k < QH; ++k) {
          float v;
          if (k == LH::REST) {
            v = b.cur.H.rest[selfnode];
          } else {
            const float ref = float(LH::w[k]) *
                              lamA[ring4(p - LH::ez[k])][ty + 1 - LH::ey[k]][tx + 1 - LH::ex[k]];
            v = dev_decode<Codec>(bload16(Hz[1 - LH::ez[k]], xyb[1 - LH::ey[k]][1 - LH::ex[k]],
                                          mslot<LH>(k) * planeB), ref);
          }
          h[k] = v;
          c = k == 0 ? double(v) : c + double(v);
        }
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          float v;
          if (k == LG::REST) {
            v = b.cur.G.rest[selfnode];
          } else {
            const float ref = float(LG::w[k]) *
                              phiA[ring4(p - LG::ez[k])][ty + 1 - LG::ey[k]][tx + 1 - LG::ex[k]];
            v = dev_decode<Codec>(bload16(Gz[1 - LG::ez[k]], xyb[1 - LG::ey[k]][1 - LG::ex[k]],
                                          mslot<LG>(k) * planeB), ref);
          }
          g_new[k] = v;
          sg = k == 0 ? double(v) : sg + double(v);
        }
      }
      const float phi = phiA[sA][ty + 1][tx + 1];
      const float mu = float(closure(K.q, c, double(phi)));
      auto atA = [&](int dx, int dy, int dz) -> float {
        return phiA[ring4(p + dz)][ty + 1 + dy][tx + 1 + dx];
      };
      float gr[3], n[3];
      gradient_normal<LG, float>(atA, K.eps2, gr, n);
      const float sbar = source_moment<float>(K, phi, mu);
      phin = float(sg + 0.5 * double(sbar));
      float F[3];
      h_flux<LG, float>(K, mu, gr, n, phin - phi, K.anti_trapping != 0, F);
      lam = h_lambda<float>(K, phi, mu);
      const float cc = float(c);
      float hs[QH];
#pragma unroll
      for (int k = 0; k < QH; ++k)
        hs[k] = h_update<LH, float>(K, k, h[k], cc, lam, F);
      encode_h<Codec, LH>(hs, lam, c, enc, hdec);
    }
    if (active && !closing) phiB[sA][ty][tx] = phin;

    const bool own_p = p >= z0 && p < z1;
    if (out && own_p) {
      const auto Hw = make_rsrc(reinterpret_cast<char*>(b.nxt.H.mov) + zp * groupBH, uint32_t(groupBH));
#pragma unroll
      for (int k = 0; k < QH; ++k)
        if (k != LH::REST) bstore16_nt(enc[k], Hw, selfB, mslot<LH>(k) * planeB);
      __builtin_nontemporal_store(hdec[LH::REST], &b.nxt.H.rest[selfnode]);
      __builtin_nontemporal_store(lam, &b.nxt.LAM[selfnode]);
      __builtin_nontemporal_store(phin, &b.nxt.PHI[selfnode]);
    }

    // streaming of h* inside the block: every region node publishes its
    // codes and Lambda, then each inner node gathers from x - e_k and decodes
    // (the same arithmetic as the writer's, so the same values), keeping the
    // population order of a pull without ordered passes
    const int xb = p & 1;
    // walls: buffers of planes p and p - 1 modulo 3 (p >= -1)
    const int ub = (p + 3) % 3, pb = (p + 2) % 3;
    const int lb = kWalls ? ub : xb;
    if (active && !closing) {
#pragma unroll
      for (int k = 0; k < QH; ++k) {
        if (k == LH::REST) continue;
        if (kWalls && k < NU)
          hxu[kWalls ? ub : 0][kWalls ? k : 0][ty][tx] = enc[k];
        else
          hxe[xb][kWalls ? k - NU - 1 : mslot<LH>(k)][ty][tx] = enc[k];
      }
      hxl[lb][ty][tx] = lam;
    }
    load_tiles(p + 2);
    // The one barrier of the plane.  Before it: reads of the phi / Lambda
    // planes p-1 .. p+1, writes of phi^{n+1}(p), of the exchange (p & 1) and
    // of the tile p+2.  After it: reads of the exchange (p & 1) and of
    // phi^{n+1}(p-2 .. p).  The slot of tile p+2 was last read before the
    // previous barrier, that of phi^{n+1}(p) after the barrier three planes
    // back, and the exchange buffer (p & 1) after the barrier two planes back
    // (with walls the buffers kept modulo 3, read also after the next
    // barrier, after the barrier three planes back).
    __syncthreads();
    const bool dn_ok = p - 1 >= z0 && p - 1 < z1;
    // decoded h* that population k of this node receives from x - e_k in the
    // exchange of plane p (not the e_z = +1 layer with walls)
    auto xchg = [&](int k) -> double {
      const int sy = ty - LH::ey[k], sx = tx - LH::ex[k];
      const float ref = float(LH::w[k]) * hxl[lb][sy][sx];
      return double(dev_decode<Codec>(hxe[xb][kWalls ? k - NU - 1 : mslot<LH>(k)][sy][sx], ref));
    };
    // walls: decoded e_z = +1 population k of plane p - 1 at region node
    // (sy, sx)
    auto xup = [&](int k, int sy, int sx) -> double {
      const float ref = float(LH::w[k]) * hxl[kWalls ? pb : 0][sy][sx];
      return double(dev_decode<Codec>(hxu[kWalls ? pb : 0][kWalls ? k : 0][sy][sx], ref));
    };
    double acc_up = 0.0;
    if constexpr (!kWalls) {
      if (inner) {
#pragma unroll
        for (int k = 0; k < QH; ++k) {
          const double v = k == LH::REST ? double(hdec[k]) : xchg(k);
          if (LH::ez[k] > 0)
            acc_up = k == 0 ? v : acc_up + v;
          else if (LH::ez[k] == 0)
            acc_mid = acc_mid + v;
          else
            acc_dn = acc_dn + v;
        }
      }
    } else if (inner && active) {
      if (!closing) {
        // c^{n+1}(p) through its in-plane layer: the e_z = +1 layer gathered
        // at the plane below, or bounced (the node's own opposite values)
        double a = 0.0;
#pragma unroll
        for (int k = 0; k < NU; ++k) {
          const bool bnc = bz_up || ((bmh >> k) & 1u);
          const double v = bnc ? double(hdec[LH::opp[k]]) : xup(k, ty - LH::ey[k], tx - LH::ex[k]);
          a = k == 0 ? v : a + v;
        }
#pragma unroll
        for (int k = NU; k < NU + NM; ++k) {
          double v;
          if (k == LH::REST)
            v = double(hdec[k]);
          else if ((bmh >> k) & 1u)
            v = double(hdec[LH::opp[k]]);
          else
            v = xchg(k);
          a = a + v;
        }
        // c^{n+1}(p - 1): its e_z = -1 layer, from this plane or bounced
        // (this node's own e_z = +1 values of plane p - 1)
#pragma unroll
        for (int k = NU + NM; k < QH; ++k) {
          const double v = ((bmh >> k) & 1u) ? xup(LH::opp[k], ty, tx) : xchg(k);
          acc_dn = acc_dn + v;
        }
        acc_up = a;
      } else {
        // past the top wall every e_z = -1 population of plane nz - 1 bounces
#pragma unroll
        for (int k = NU + NM; k < QH; ++k) acc_dn = acc_dn + xup(LH::opp[k], ty, tx);
      }
    }

    if (out && dn_ok) {
      const int zq = wrap_coord(p - 1, nz);
      const double c1 = acc_dn;
      const float phi1 = phiB[ring4(p - 1)][ty][tx];
      const float mu1 = float(closure(K.q, c1, double(phi1)));
      const int zm = (wz && p - 1 == 0) ? 0 : -1, zpl = (wz && p - 1 == nz - 1) ? 0 : 1;
      auto atB = [&](int dx, int dy, int dz) -> float {
        const int ox = dx < 0 ? xm : (dx > 0 ? xp : 0);
        const int oy = dy < 0 ? ym : (dy > 0 ? yp : 0);
        const int oz = dz < 0 ? zm : (dz > 0 ? zpl : 0);
        return phiB[ring4(p - 1 + oz)][ty + oy][tx + ox];
      };
      float gr1[3], n1[3];
      gradient_normal<LG, float>(atB, K.eps2, gr1, n1);
      float G[Q], gs[Q];
      phi_sources<LG, float>(K, phi1, mu1, n1, G);
      double sg1 = 0.0;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        sg1 = k == 0 ? double(g_old[k]) : sg1 + double(g_old[k]);
        gs[k] = g_collide<LG, float>(K, k, g_old[k], phi1, G[k]);
      }
      uint16_t genc[Q];
      float gdec[Q];
      encode_g<Codec, LG>(gs, phi1, genc, gdec);
      balance_g_rest<LG, float, float>(K, gdec, sg1, phi1, source_moment<float>(K, phi1, mu1));
      const auto Gw = make_rsrc(reinterpret_cast<char*>(b.nxt.G.mov) + zq * groupB, uint32_t(groupB));
#pragma unroll
      for (int k = 0; k < Q; ++k)
        if (k != LG::REST) bstore16_nt(genc[k], Gw, selfB, mslot<LG>(k) * planeB);
      __builtin_nontemporal_store(gdec[LG::REST], &b.nxt.G.rest[(int64_t)zq * plane + self_xy]);
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) g_old[k] = g_new[k];
    if constexpr (kWalls) {
      acc_dn = acc_up;
    } else {
      acc_dn = acc_mid;
      acc_mid = acc_up;
    }
  }
  __syncthreads();  // the LDS rings are refilled by the next tile
  }
}

// output rows per tile with walls: the wall bookkeeping (bounce masks,
// mirror offsets, the third exchange buffer) does not fit the 128 VGPRs of
// 16 waves per CU, so the walled z-march runs 64 x 9 tiles (12 waves, up to
// 168 VGPRs) instead of spilling
#ifndef GPLBM_DEV_WALL_TY
#define GPLBM_DEV_WALL_TY 9
#endif

template <class Codec, class LG, class LH, bool kGen>
struct DevFused3D {
  template <bool kWalls>
  static int run(const Geo& g, const Coef<float>& K, const DevStep& b, hipStream_t st) {
    // z chunks of 128 planes on periodic grids (2 halo planes per 130; 1280
    // tiles at 512^3, 5 passes of the 256 resident blocks): FP16 6.98-7.01
    // against 7.10 ms with 64, which ran 7.37 against 7.52 with 32; 32 with
    // walls (64 x 9 tiles: 7296 at 512^3, 28.5 passes, against 14.25 with 64)
    constexpr int TX = 64, TY = kWalls ? GPLBM_DEV_WALL_TY : GPLBM_DEV_TY, ZC = kWalls ? 32 : 128;
    constexpr int NT = TileShape<TX, TY>::NT;
    auto kernel = k_dev_fused3d<TX, TY, ZC, Codec, LG, LH, kGen, kWalls>;
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
  static int launch(const Geo& g, const Coef<float>& K, const DevStep& b, hipStream_t st) {
    return (g.bcx || g.bcy || g.bcz) ? run<true>(g, K, b, st) : run<false>(g, K, b, st);
  }
};

// ---------------------------------------------------------------------------
// Fused schedule in the deviation format on D2Q9 (any boundaries): one kernel
// per step, the 2-D tiling of the FP32 / FP64 fused kernel.  A block owns an
// output tile T (x-aligned, tiles.h) and computes T grown by one node (T+1):
//   - phi^n and Lambda^{n-1} of T+2 are staged in LDS; every pull decodes
//     with the reference (w_k phi or w_k Lambda) of its source node, or of the
//     node itself for a population bounced back at a wall;
//   - the threads of T+1 run the h collision of step n, write the 16-bit
//     codes (nodes of T) and publish the decoded h* to an LDS exchange;
//   - after one barrier each node of T gathers c^{n+1} from x - e_k in
//     population order (its own h*_{opp k} where x - e_k lies beyond a
//     wall), then runs the g collision of step n+1.
// The values and the order of every sum are those of the split kernels, so
// the two schedules give identical bits.
template <class P>
struct LatticeTag {
  using type = P;
};

template <int TX, int TY, class Codec, class L, class LH, bool kGen>
__global__ void __launch_bounds__((TileShape<TX, TY>::NT))
    k_dev_fused2d(Geo g, Coef<float> Kin, DevStep b, int tiles_x, int ntiles) {
  const Coef<float> K = variant<kGen>(Kin);
  // g on L (D2Q9 or D2Q5), h on LH (L, or D2Q5 under D2Q9)
  constexpr int Q = L::Q, QH = LH::Q;
  using Shape = TileShape<TX, TY>;
  constexpr int BX = Shape::BX, BY = Shape::BY, NT = Shape::NT;
  constexpr int AX = BX + 2, AY = BY + 2;
  __shared__ float phiA[AY][AX];  // phi^n on T+2
  __shared__ float lamA[AY][AX];  // Lambda^{n-1} on T+2
  __shared__ float phiB[BY][BX];  // phi^{n+1} on T+1
  __shared__ float hx[QH][BY][BX];  // decoded h*^n of T+1 (moving populations)

  int tx, ty;
  bool valid;
  Shape::node(threadIdx.x, tx, ty, valid);

  for (int tile = first_tile(); tile < ntiles; tile += gridDim.x) {
  const int X0 = (tile % tiles_x) * TX, Y0 = (tile / tiles_x) * TY;
  for (int l = threadIdx.x; l < AX * AY; l += NT) {
    const int lx = l % AX, ly = l / AX;
    int vx = X0 - 2 + lx, vy = Y0 - 2 + ly;
    vx = g.bcx ? min(max(vx, 0), g.nx - 1) : wrap_coord(vx, g.nx);
    vy = g.bcy ? min(max(vy, 0), g.ny - 1) : wrap_coord(vy, g.ny);
    const int64_t j = node_index(g, vx, vy, 0);
    phiA[ly][lx] = b.cur.PHI[j];
    lamA[ly][lx] = b.cur.LAM[j];
  }

  const int ux = X0 - 1 + tx, uy = Y0 - 1 + ty;  // unwrapped node of this thread
  const bool in_x = ux >= 0 && ux < g.nx, in_y = uy >= 0 && uy < g.ny;
  const bool active = valid && (in_x || !g.bcx) && (in_y || !g.bcy);
  const bool out = valid && in_x && in_y && tx >= 1 && tx <= TX && ty >= 1 && ty <= TY;
  const int x = g.bcx ? ux : wrap_coord(ux, g.nx);
  const int y = g.bcy ? uy : wrap_coord(uy, g.ny);
  const int64_t i = active ? node_index(g, x, y, 0) : 0;
  const int xm = (g.bcx && ux == 0) ? 0 : -1, xp = (g.bcx && ux == g.nx - 1) ? 0 : 1;
  const int ym = (g.bcy && uy == 0) ? 0 : -1, yp = (g.bcy && uy == g.ny - 1) ? 0 : 1;
  // population k (of lattice P) of this node comes from x - e_k, or bounces
  // back at a wall
  auto inside = [&](auto tag, int k) {
    using P = typename decltype(tag)::type;
    const int sx = ux - P::ex[k], sy = uy - P::ey[k];
    return !((g.bcx && (sx < 0 || sx >= g.nx)) || (g.bcy && (sy < 0 || sy >= g.ny)));
  };
  // pull of population k from a distribution in the deviation format, the
  // reference field of the source node read from its T+2 tile
  auto pull_tile = [&](auto tag, const DevDist& d, const float (*ref)[AX], int k) -> float {
    using P = typename decltype(tag)::type;
    if (k == P::REST) return d.rest[i];
    int sx = x, sy = y, kk = k, rx = tx + 1, ry = ty + 1;
    if (inside(tag, k)) {
      pull_axis(sx, P::ex[k], g.nx, g.bcx);
      pull_axis(sy, P::ey[k], g.ny, g.bcy);
      rx -= P::ex[k];
      ry -= P::ey[k];
    } else {
      kk = P::opp[k];
    }
    const float r = float(P::w[kk]) * ref[ry][rx];
    return dev_decode<Codec>(d.mov[mov_index<P>(g, kk, sx, sy, 0)], r);
  };
  const LatticeTag<L> tg{};
  const LatticeTag<LH> th{};
  __syncthreads();

  float gn[Q];          // g~^{n+1}
  float hdec[QH];       // h~*^n as readers decode it
  float phin = 0.0f;
  if (active) {
    float h[QH];
    double c = 0.0;
#pragma unroll
    for (int k = 0; k < QH; ++k) {
      h[k] = pull_tile(th, b.cur.H, lamA, k);
      c = k == 0 ? double(h[k]) : c + double(h[k]);
    }
    double sg = 0.0;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      gn[k] = pull_tile(tg, b.cur.G, phiA, k);
      sg = k == 0 ? double(gn[k]) : sg + double(gn[k]);
    }
    const float phi = phiA[ty + 1][tx + 1];
    const float mu = float(closure(K.q, c, double(phi)));
    auto at = [&](int dx, int dy, int) -> float {
      const int ox = dx < 0 ? xm : (dx > 0 ? xp : 0);
      const int oy = dy < 0 ? ym : (dy > 0 ? yp : 0);
      return phiA[ty + 1 + oy][tx + 1 + ox];
    };
    float gr[3], n[3];
    gradient_normal<L, float>(at, K.eps2, gr, n);
    const float sbar = source_moment<float>(K, phi, mu);
    phin = float(sg + 0.5 * double(sbar));
    float F[3];
    h_flux<L, float>(K, mu, gr, n, phin - phi, K.anti_trapping != 0, F);
    const float lam = h_lambda<float>(K, phi, mu);
    const float cc = float(c);
    float hs[QH];
#pragma unroll
    for (int k = 0; k < QH; ++k)
      hs[k] = h_update<LH, float>(K, k, h[k], cc, lam, F);
    uint16_t enc[QH];
    encode_h<Codec, LH>(hs, lam, c, enc, hdec);
    if (out) {
#pragma unroll
      for (int k = 0; k < QH; ++k)
        if (k != LH::REST) b.nxt.H.mov[mov_index<LH>(g, k, x, y, 0)] = enc[k];
      b.nxt.H.rest[i] = hdec[LH::REST];
      b.nxt.LAM[i] = lam;
      b.nxt.PHI[i] = phin;
    }
  }
  if (valid) {
    phiB[ty][tx] = phin;
    if (active) {
#pragma unroll
      for (int k = 0; k < QH; ++k)
        if (k != LH::REST) hx[k][ty][tx] = hdec[k];
    }
  }
  __syncthreads();

  if (out) {
    double c1 = 0.0;
#pragma unroll
    for (int k = 0; k < QH; ++k) {
      float v;
      if (k == LH::REST)
        v = hdec[k];
      else if (inside(th, k))
        v = hx[k][ty - LH::ey[k]][tx - LH::ex[k]];
      else
        v = hdec[LH::opp[k]];
      c1 = k == 0 ? double(v) : c1 + double(v);
    }
    const float phi1 = phiB[ty][tx];
    const float mu1 = float(closure(K.q, c1, double(phi1)));
    auto at1 = [&](int dx, int dy, int) -> float {
      const int ox = dx < 0 ? xm : (dx > 0 ? xp : 0);
      const int oy = dy < 0 ? ym : (dy > 0 ? yp : 0);
      return phiB[ty + oy][tx + ox];
    };
    float gr[3], n[3];
    gradient_normal<L, float>(at1, K.eps2, gr, n);
    float G[Q], gs[Q];
    phi_sources<L, float>(K, phi1, mu1, n, G);
    double sg1 = 0.0;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      sg1 = k == 0 ? double(gn[k]) : sg1 + double(gn[k]);
      gs[k] = g_collide<L, float>(K, k, gn[k], phi1, G[k]);
    }
    uint16_t genc[Q];
    float gdec[Q];
    encode_g<Codec, L>(gs, phi1, genc, gdec);
    balance_g_rest<L, float, float>(K, gdec, sg1, phi1, source_moment<float>(K, phi1, mu1));
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (k == L::REST)
        b.nxt.G.rest[i] = gdec[k];
      else
        b.nxt.G.mov[mov_index<L>(g, k, x, y, 0)] = genc[k];
    }
  }
  __syncthreads();  // the LDS tiles are refilled by the next tile
  }
}

// output rows per tile of the fused 2-D deviation kernel: 64 x 13 outputs,
// 1024 threads, one block per CU (1024^2 step: 55 us, against 62 / 70 / 74 /
// 78 us at 12 / 8 / 5 / 4 rows, the last two with two blocks per CU)
#ifndef GPLBM_DEV2_TY
#define GPLBM_DEV2_TY 13
#endif

template <class Codec, class L, class LH, bool kGen>
struct DevFused2D {
  static int launch(const Geo& g, const Coef<float>& K, const DevStep& b, hipStream_t st) {
    constexpr int TX = 64, TY = GPLBM_DEV2_TY;
    constexpr int NT = TileShape<TX, TY>::NT;
    auto kernel = k_dev_fused2d<TX, TY, Codec, L, LH, kGen>;
    const int tiles_x = (g.nx + TX - 1) / TX;
    const int tiles_y = (g.ny + TY - 1) / TY;
    const int ntiles = tiles_x * tiles_y;
    static int resident[64] = {0};
    const int grid = resident_grid(kernel, NT, ntiles, resident);
    if (grid <= 0) return -1;
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(NT), 0, st, g, K, b, tiles_x, ntiles);
    return 0;
  }
};

// 32-bit offsets inside a z plane group of moving populations; any boundary
inline bool dev_fused_supported(int nx, int ny, int nz, const int*) {
  return (int64_t)nx * ny * kMov * 2 < ((int64_t)1 << 31) &&
         (int64_t)nx * ny * nz < ((int64_t)1 << 31);
}

}  // namespace gplbm
