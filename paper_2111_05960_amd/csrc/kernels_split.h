// Split schedule: one time step n -> n+1 in two kernels.
//
//   h_step: c^n = sum_k h~^n_k (pull of H), mu^n, grad phi^n and the normal
//           from the phi^n stencil, phi^{n+1} = sum_k g~^{n+1}_k + S^n/2 (pull
//           of G), dphi/dt = phi^{n+1} - phi^n, anti-trapping current, h
//           collision  ->  H' = h~*^n, PHI' = phi^{n+1}
//   g_step: c^{n+1} (pull of H'), mu^{n+1}, grad phi^{n+1}, sources, g
//           collision of the pulled g~^{n+1}  ->  G' = g~*^{n+1}
//
// Each kernel reads both distributions once and writes one, so the step
// moves 6Q+3 values per node against the 4Q+2 of the fused schedule.  It has
// no tile halo and works for every boundary combination; it is the baseline
// the fused kernels are checked against.
//
// Also here: initialisation, field read-out and the diagnostics reduction,
// which all schedules share.
#pragma once

#include "geometry.h"
#include "node_math.h"

namespace gplbm {

template <class S>
struct StepBufs {
  const S* __restrict__ G;    // g~*^n
  const S* __restrict__ H;    // h~*^{n-1}
  const S* __restrict__ PHI;  // phi^n
  S* __restrict__ Hn;         // h~*^n
  S* __restrict__ PHIn;       // phi^{n+1}
  S* __restrict__ Gn;         // g~*^{n+1}
};

// phi at (x, y, z) + d from global memory with the stencil ghost rule.
template <class S, class C>
struct GlobalPhi {
  const Geo& g;
  const S* __restrict__ f;
  int x, y, z;
  __device__ C operator()(int dx, int dy, int dz) const {
    int xx = stencil_axis(x + dx, g.nx, g.bcx);
    int yy = stencil_axis(y + dy, g.ny, g.bcy);
    int zz = stencil_axis(z + dz, g.nz, g.bcz);
    return C(f[node_index(g, xx, yy, zz)]);
  }
};

template <class L, class LH, class S, class C, bool kGen>
__global__ void __launch_bounds__(256) k_split_h(Geo g, Coef<C> Kin, StepBufs<S> b) {
  const Coef<C> K = variant<kGen>(Kin);
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t i = node_index(g, x, y, z);

  C h[LH::Q];
  double c = 0.0;
#pragma unroll
  for (int k = 0; k < LH::Q; ++k) {
    S v = pull<LH>(g, b.H, k, x, y, z);
    h[k] = C(v);
    c = k == 0 ? double(v) : c + double(v);
  }
  const C phi = C(b.PHI[i]);
  const double mu_d = closure(K.q, c, double(phi));
  const C mu = C(mu_d);
  C gr[3], n[3];
  gradient_normal<L, C>(GlobalPhi<S, C>{g, b.PHI, x, y, z}, K.eps2, gr, n);
  const C sbar = source_moment<C>(K, phi, mu);

  double sg = 0.0;
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    double v = double(pull<L>(g, b.G, k, x, y, z));
    sg = k == 0 ? v : sg + v;
  }
  const double phin = sg + 0.5 * double(sbar);
  const C dtphi = C(phin) - phi;

  C F[3];
  h_flux<L, C>(K, mu, gr, n, dtphi, K.anti_trapping != 0, F);
  const C lam = h_lambda<C>(K, phi, mu);
  const C cc = C(c);
  C hs[LH::Q];
#pragma unroll
  for (int k = 0; k < LH::Q; ++k) hs[k] = C(S(h_update<LH, C>(K, k, h[k], cc, lam, F)));
  balance_rest<LH, S, C>(hs, c);
#pragma unroll
  for (int k = 0; k < LH::Q; ++k) b.Hn[pop_index<LH>(g, k, x, y, z)] = S(hs[k]);
  b.PHIn[i] = S(phin);
}

template <class L, class LH, class S, class C, bool kGen>
__global__ void __launch_bounds__(256) k_split_g(Geo g, Coef<C> Kin, StepBufs<S> b) {
  const Coef<C> K = variant<kGen>(Kin);
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t i = node_index(g, x, y, z);

  double c = 0.0;
#pragma unroll
  for (int k = 0; k < LH::Q; ++k) {
    double v = double(pull<LH>(g, (const S*)b.Hn, k, x, y, z));
    c = k == 0 ? v : c + v;
  }
  const C phi = C(b.PHIn[i]);
  const C mu = C(closure(K.q, c, double(phi)));
  C gr[3], n[3];
  gradient_normal<L, C>(GlobalPhi<S, C>{g, b.PHIn, x, y, z}, K.eps2, gr, n);
  C G[L::Q];
  phi_sources<L, C>(K, phi, mu, n, G);
  C gs[L::Q];
  double sg = 0.0;
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    const S v = pull<L>(g, b.G, k, x, y, z);
    sg = k == 0 ? double(v) : sg + double(v);
    gs[k] = C(S(g_collide<L, C>(K, k, C(v), phi, G[k])));
  }
  balance_g_rest<L, S, C>(K, gs, sg, phi, source_moment<C>(K, phi, mu));
#pragma unroll
  for (int k = 0; k < L::Q; ++k) b.Gn[pop_index<L>(g, k, x, y, z)] = S(gs[k]);
}

// ---------------------------------------------------------------------------
// Initialisation: g~^0 = w_k phi0 - G^0_k / 2, h~^0 = h^eq_k - H^0_k / 2
// (no anti-trapping current), then the collision of g at time 0 so that the
// state satisfies the invariant of geometry.h at n = 0.  h~^0 is stored
// "unstreamed": each value goes to the slot the pull of the first step reads
// it from (the inverse of the pull permutation).

template <class L, class LH, class S, class C>
__global__ void __launch_bounds__(256) k_init(Geo g, Coef<C> K, const double* __restrict__ phi0,
                                              const double* __restrict__ c0, S* __restrict__ G,
                                              S* __restrict__ H, S* __restrict__ PHI) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t i = node_index(g, x, y, z);

  const C phi = C(phi0[i]);
  const double cin = c0[i];
  C gr[3], n[3];
  // the stencil reads phi0 converted to the arithmetic type
  struct InitPhi {
    const Geo& g;
    const double* __restrict__ f;
    int x, y, z;
    __device__ C operator()(int dx, int dy, int dz) const {
      int xx = stencil_axis(x + dx, g.nx, g.bcx);
      int yy = stencil_axis(y + dy, g.ny, g.bcy);
      int zz = stencil_axis(z + dz, g.nz, g.bcz);
      return C(f[node_index(g, xx, yy, zz)]);
    }
  };
  gradient_normal<L, C>(InitPhi{g, phi0, x, y, z}, K.eps2, gr, n);

  // initial populations from (phi0, c0)
  const C mu0 = C(closure(K.q, cin, double(phi)));
  C G0[L::Q];
  phi_sources<L, C>(K, phi, mu0, n, G0);
  C F[3];
  h_flux<L, C>(K, mu0, gr, n, C(0), false, F);
  const C lam = h_lambda<C>(K, phi, mu0);
  S hs[LH::Q];
  double c = 0.0;
#pragma unroll
  for (int k = 0; k < LH::Q; ++k) {
    hs[k] = S(h_initial<LH, C>(K, k, C(cin), lam, F));
    c = k == 0 ? double(hs[k]) : c + double(hs[k]);
  }
  // collision of g at time 0 with c^0 = sum_k h~^0_k
  const C mu = C(closure(K.q, c, double(phi)));
  C Gk[L::Q];
  phi_sources<L, C>(K, phi, mu, n, Gk);
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    C g0 = S(C(L::w[k]) * phi - C(0.5) * G0[k]);
    G[pop_index<L>(g, k, x, y, z)] = S(g_collide<L, C>(K, k, g0, phi, Gk[k]));
  }
  // h~^0 into the slots the first pull reads
#pragma unroll
  for (int k = 0; k < LH::Q; ++k) {
    int dx = x, dy = y, dz = z;
    // destination x - e_k of the value arriving at x along k
    bool in = pull_axis(dx, LH::ex[k], g.nx, g.bcx) && pull_axis(dy, LH::ey[k], g.ny, g.bcy);
    if (LH::D == 3) in = in && pull_axis(dz, LH::ez[k], g.nz, g.bcz);
    if (in)
      H[pop_index<LH>(g, k, dx, dy, dz)] = hs[k];
    else
      H[pop_index<LH>(g, LH::opp[k], x, y, z)] = hs[k];
  }
  PHI[i] = S(phi);
}

// ---------------------------------------------------------------------------
// Read-out of phi^n, c^n, mu^n as doubles.

template <class L, class S>
__global__ void __launch_bounds__(256) k_fields(Geo g, ClosureK q, const S* __restrict__ H,
                                                const S* __restrict__ PHI, double* phi_out,
                                                double* c_out, double* mu_out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t i = node_index(g, x, y, z);
  double c = 0.0;
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    double v = double(pull<L>(g, H, k, x, y, z));
    c = k == 0 ? v : c + v;
  }
  const double phi = double(PHI[i]);
  if (phi_out) phi_out[i] = phi;
  if (c_out) c_out[i] = c;
  if (mu_out) mu_out[i] = closure(q, c, phi);
}

// ---------------------------------------------------------------------------
// Diagnostics: fixed-shape two-pass reduction in double, wavefront shuffles
// inside each block (deterministic: the association of every sum depends
// only on the launch shape).

constexpr int kDiagThreads = 256;
constexpr int kDiagBlocks = 1024;
constexpr int kDiagVals = 8;  // mass, solid, count, sum phi, min, max, nonfinite, spare
constexpr int kDiagWaves = kDiagThreads / 64;

// Combination of two partial diagnostics (sums, min, max, flag).
__device__ __forceinline__ void diag_combine(double* v, const double* u) {
  v[0] = v[0] + u[0];
  v[1] = v[1] + u[1];
  v[2] = v[2] + u[2];
  v[3] = v[3] + u[3];
  v[4] = fmin(v[4], u[4]);
  v[5] = fmax(v[5], u[5]);
  v[6] = fmax(v[6], u[6]);
}

// Block reduction of the per-thread partials: within each wavefront by
// shuffles with halving offsets (lane l takes lane l + off), then the
// wavefront results in wave order.  The association depends only on the
// launch shape, so the result is deterministic.  Thread 0 returns the total.
__device__ __forceinline__ void diag_block_reduce(double* v) {
  __shared__ double wred[kDiagWaves][kDiagVals];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    double u[kDiagVals];
#pragma unroll
    for (int j = 0; j < kDiagVals; ++j) u[j] = __shfl_down(v[j], off, 64);
    diag_combine(v, u);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < kDiagVals; ++j) wred[wave][j] = v[j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kDiagWaves; ++w) diag_combine(v, wred[w]);
  }
}

template <class L, class S>
__global__ void __launch_bounds__(kDiagThreads) k_diag_partial(Geo g, const S* __restrict__ H,
                                                               const S* __restrict__ PHI,
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
      double hv = double(pull<L>(g, H, k, x, y, z));
      c = k == 0 ? hv : c + hv;
    }
    const double phi = double(PHI[i]);
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

__global__ void __launch_bounds__(kDiagThreads) k_diag_final(const double* __restrict__ part,
                                                             int nblocks, double* __restrict__ out) {
  double v[kDiagVals] = {0.0, 0.0, 0.0, 0.0, INFINITY, -INFINITY, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += kDiagThreads) {
    const double* p = part + b * kDiagVals;
    v[0] = v[0] + p[0];
    v[1] = v[1] + p[1];
    v[2] = v[2] + p[2];
    v[3] = v[3] + p[3];
    v[4] = fmin(v[4], p[4]);
    v[5] = fmax(v[5], p[5]);
    v[6] = fmax(v[6], p[6]);
  }
  diag_block_reduce(v);
  if (threadIdx.x == 0)
    for (int j = 0; j < kDiagVals; ++j) out[j] = v[j];
}

}  // namespace gplbm
