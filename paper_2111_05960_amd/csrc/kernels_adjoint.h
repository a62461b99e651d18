// Hand-written adjoint (reverse mode) of the coupled step, FP64.
//
// The forward step maps the state S_n = (G = g~*^n, H = h~*^{n-1}, PHI = phi^n)
// to S_{n+1} (geometry.h).  Given the adjoint of S_{n+1} (Gb', Hb', Pb') and
// the forward states S_n and S_{n+1}, one reverse step produces the adjoint of
// S_n and accumulates the parameter adjoints (lambda, D_l) per node.  Every
// operation of the step is linear in the populations, so the reverse of a
// collision is a weighted copy; the nonlinear parts (closure products, p'(phi),
// the normal, mu D' grad phi, the anti-trapping product, D(phi) mu) are
// differentiated by hand at the forward values, which the reverse kernels
// recompute from S_n and S_{n+1}.
//
// Two kernels per reverse step (each node reads its neighbours only through
// the previous kernel's output):
//   ra: gathers the adjoint of G' from the previous reverse step, then the
//       reverse of the g collision of step n+1: adjoint of the pulled
//       g~^{n+1} (A1), of grad phi^{n+1} (A2, plus the previous step's B3),
//       of c^{n+1} (A3) and the local adjoint of phi^{n+1} (A4, plus the
//       previous step's B4);
//   rb: adjoint of h~*^n (gathered from the previous step, plus c^{n+1} from
//       the node it streams to), total adjoint of phi^{n+1} (A4 and the
//       stencil transpose of A2), reverse of the h collision of step n and of
//       phi^{n+1} = sum g~^{n+1} + S^n / 2: B1, B2, B3, B4.
// The transposes of the pulls and of the gradient stencil are done as gathers
// by the consumer, so the adjoint of a state is never written out.
// Parameters are held fixed except lambda and D_l (gamma, M_phi, W and a do
// not follow D_l).
#pragma once

#include <type_traits>

#include "kernels_dev.h"
#include "kernels_split.h"

namespace gplbm {

// Intermediates of one reverse step that the next one (or the reverse of the
// initialisation) gathers from; double-buffered by step parity.  The adjoint
// of the state S_n is never materialised: its G, H and PHI parts are the
// gathers  Gb(slot) = A1(dest) + B2(dest),  Hb(slot) = B1(dest),
// Pb = B4 + stencil transpose of B3  (dest = the node and population that
// pull the slot).
struct AdjSet {
  double* A1;  // Q*N: adjoint of the pulled g~^{n+1}
  double* B1;  // Q*N: adjoint of the pulled h~^n
  double* B2;  // N:   adjoint of phi^{n+1} (every pulled g adds to it)
  double* B3;  // 3*N: adjoint of grad phi^n
  double* B4;  // N:   local adjoint of phi^n
};

struct AdjWork {
  AdjSet set[2];
  double *A2, *A3, *A4;  // 3*N, N, N: adjoint of grad phi^{n+1}, c^{n+1}, local phi^{n+1}
  double *lamb, *dlb;    // per-node accumulators of dJ/dlambda, dJ/dD_l
  double* red;           // reduction scratch
};

// A forward state in the storage type S of the context (FP64 or FP32); the
// reverse kernels recompute the forward quantities from it in FP64.
template <class S>
struct FwdState {
  const S* G;
  const S* H;
  const S* PHI;
};

// A forward state in a deviation format (any lattices): the h populations decode
// with the Lambda field of the state, phi is FP32.  The reverse kernels take
// the decoded values as the state and differentiate the FP64 step there.
template <class Codec>
struct DevFwdState {
  DevDist H;
  const float* PHI;
  const float* LAM;
};

// Destination of the value stored in slot (k, x, y, z) under the pull
// streaming: the node x + e_k reads it as population k, or, when x + e_k
// lies beyond a zero-flux wall, x itself reads it as population opp(k).
// Returns the destination population; (dx, dy, dz) the destination node.
template <class L>
__device__ __forceinline__ int push_dest(const Geo& g, int k, int x, int y, int z, int& dx, int& dy,
                                         int& dz) {
  dx = x;
  dy = y;
  dz = z;
  // moving "backwards" by -e_k with pull_axis gives x + e_k
  bool in = pull_axis(dx, -L::ex[k], g.nx, g.bcx) && pull_axis(dy, -L::ey[k], g.ny, g.bcy);
  if (L::D == 3) in = in && pull_axis(dz, -L::ez[k], g.nz, g.bcz);
  if (!in) {
    dx = x;
    dy = y;
    dz = z;
    return L::opp[k];
  }
  return k;
}

// Addressing of the reverse steps.  AdjAddrGeneral takes any boundary, by
// the rules of geometry.h; AdjAddrPeriodic serves grids periodic on every
// axis, where each neighbour is the node plus a wrapped offset (precomputed
// per node, the plane ones uniform over a block), without the per-population
// wall tests.  Both give the same indices on a periodic grid.
struct AdjAddrGeneral {
  const Geo& g;
  int x, y, z;
  __device__ AdjAddrGeneral(const Geo& g_, int x_, int y_, int z_) : g(g_), x(x_), y(y_), z(z_) {}
  __device__ int64_t self() const { return node_index(g, x, y, z); }
  // slot that population k of lattice P pulls at this node: (k, x - e_k), or
  // (opp k, x) when x - e_k lies beyond a wall
  template <class P>
  __device__ int64_t pull_slot(int k) const {
    int sx = x, sy = y, sz = z;
    bool in = pull_axis(sx, P::ex[k], g.nx, g.bcx) && pull_axis(sy, P::ey[k], g.ny, g.bcy);
    if (P::D == 3) in = in && pull_axis(sz, P::ez[k], g.nz, g.bcz);
    if (!in) return pop_index<P>(g, P::opp[k], x, y, z);
    return pop_index<P>(g, k, sx, sy, sz);
  }
  // node and population that pull slot k of this node
  template <class P>
  __device__ void push(int k, int64_t& dpop, int64_t& dnode) const {
    int dx, dy, dz;
    const int kk = push_dest<P>(g, k, x, y, z, dx, dy, dz);
    dpop = pop_index<P>(g, kk, dx, dy, dz);
    dnode = node_index(g, dx, dy, dz);
  }
  // source node of the value population k of lattice P pulls (the node
  // itself for a bounced population), and its slot in the deviation layout
  template <class P>
  __device__ void pull_dev_slot(int k, int64_t& node, int64_t& slot, int& kk) const {
    int sx = x, sy = y, sz = z;
    bool in = pull_axis(sx, P::ex[k], g.nx, g.bcx) && pull_axis(sy, P::ey[k], g.ny, g.bcy);
    if (P::D == 3) in = in && pull_axis(sz, P::ez[k], g.nz, g.bcz);
    kk = in ? k : P::opp[k];
    if (!in) sx = x, sy = y, sz = z;
    node = node_index(g, sx, sy, sz);
    slot = mov_index<P>(g, kk, sx, sy, sz);
  }
  // node x + (dx, dy, dz) of the gradient stencil (mirror ghost at walls)
  __device__ int64_t stencil(int dx, int dy, int dz) const {
    return node_index(g, stencil_axis(x + dx, g.nx, g.bcx), stencil_axis(y + dy, g.ny, g.bcy),
                      stencil_axis(z + dz, g.nz, g.bcz));
  }
};

struct AdjAddrPeriodic {
  int64_t plane;
  int z, zm, zp;             // planes z, z - 1, z + 1 (wrapped)
  int xy;                    // y nx + x
  int oxm, oxp, oym, oyp;    // in-plane offsets of x - 1, x + 1, y - 1, y + 1 (wrapped)
  __device__ AdjAddrPeriodic(const Geo& g, int x, int y, int z_) {
    plane = (int64_t)g.nx * g.ny;
    z = z_;
    zm = z == 0 ? g.nz - 1 : z - 1;
    zp = z == g.nz - 1 ? 0 : z + 1;
    xy = y * g.nx + x;
    oxm = x == 0 ? g.nx - 1 : -1;
    oxp = x == g.nx - 1 ? 1 - g.nx : 1;
    oym = y == 0 ? (g.ny - 1) * g.nx : -g.nx;
    oyp = y == g.ny - 1 ? (1 - g.ny) * g.nx : g.nx;
  }
  __device__ int xyn(int dx, int dy) const {
    return xy + (dx < 0 ? oxm : (dx > 0 ? oxp : 0)) + (dy < 0 ? oym : (dy > 0 ? oyp : 0));
  }
  __device__ int zn(int dz) const { return dz < 0 ? zm : (dz > 0 ? zp : z); }
  __device__ int64_t node(int dx, int dy, int dz) const { return (int64_t)zn(dz) * plane + xyn(dx, dy); }
  __device__ int64_t self() const { return (int64_t)z * plane + xy; }
  template <class P>
  __device__ int64_t pull_slot(int k) const {
    return ((int64_t)zn(-P::ez[k]) * P::Q + k) * plane + xyn(-P::ex[k], -P::ey[k]);
  }
  template <class P>
  __device__ void push(int k, int64_t& dpop, int64_t& dnode) const {
    dpop = ((int64_t)zn(P::ez[k]) * P::Q + k) * plane + xyn(P::ex[k], P::ey[k]);
    dnode = node(P::ex[k], P::ey[k], P::ez[k]);
  }
  template <class P>
  __device__ void pull_dev_slot(int k, int64_t& src, int64_t& slot, int& kk) const {
    kk = k;
    src = node(-P::ex[k], -P::ey[k], -P::ez[k]);
    slot = ((int64_t)zn(-P::ez[k]) * (P::Q - 1) + mslot<P>(k)) * plane + xyn(-P::ex[k], -P::ey[k]);
  }
  __device__ int64_t stencil(int dx, int dy, int dz) const { return node(dx, dy, dz); }
};

template <class S, class A>
struct AddrPhi {
  const S* __restrict__ f;
  const A& a;
  __device__ double operator()(int dx, int dy, int dz) const { return double(f[a.stencil(dx, dy, dz)]); }
};

// Forward quantities at one node from a state: c, mu, phi, grad phi, normal.
template <class L>
struct NodeFwd {
  double c, mu, phi, g[3], n[3], s;  // s = sqrt(|grad|^2 + eps^2)
};

template <class L, class LH, class S, class A>
__device__ __forceinline__ NodeFwd<L> node_fwd_at(const Coef<double>& K, const FwdState<S>& F,
                                                  const A& a) {
  NodeFwd<L> f;
  double c = 0.0;
#pragma unroll
  for (int k = 0; k < LH::Q; ++k) {
    const double v = double(F.H[a.template pull_slot<LH>(k)]);
    c = k == 0 ? v : c + v;
  }
  f.c = c;
  f.phi = double(F.PHI[a.self()]);
  f.mu = closure(K.q, c, f.phi);
  gradient_normal<L, double>(AddrPhi<S, A>{F.PHI, a}, K.eps2, f.g, f.n);
  double nn = f.g[0] * f.g[0] + f.g[1] * f.g[1];
  if (L::D == 3) nn = nn + f.g[2] * f.g[2];
  f.s = sqrt(nn + K.eps2);
  return f;
}

template <class L, class LH, class Codec, class A>
__device__ __forceinline__ NodeFwd<L> node_fwd_at(const Coef<double>& K, const DevFwdState<Codec>& F,
                                                  const A& a) {
  NodeFwd<L> f;
  double c = 0.0;
#pragma unroll
  for (int k = 0; k < LH::Q; ++k) {
    float v;
    if (k == LH::REST) {
      v = F.H.rest[a.self()];
    } else {
      int64_t src, slot;
      int kk;
      a.template pull_dev_slot<LH>(k, src, slot, kk);
      v = dev_decode<Codec>(F.H.mov[slot], float(LH::w[kk]) * F.LAM[src]);
    }
    c = k == 0 ? double(v) : c + double(v);
  }
  f.c = c;
  f.phi = double(F.PHI[a.self()]);
  f.mu = closure(K.q, c, f.phi);
  gradient_normal<L, double>(AddrPhi<float, A>{F.PHI, a}, K.eps2, f.g, f.n);
  double nn = f.g[0] * f.g[0] + f.g[1] * f.g[1];
  if (L::D == 3) nn = nn + f.g[2] * f.g[2];
  f.s = sqrt(nn + K.eps2);
  return f;
}

template <class L, class LH, class S>
__device__ __forceinline__ NodeFwd<L> node_fwd(const Geo& g, const Coef<double>& K, const FwdState<S>& F,
                                               int x, int y, int z) {
  NodeFwd<L> f;
  double c = 0.0;
#pragma unroll
  for (int k = 0; k < LH::Q; ++k) {
    const double v = double(pull<LH>(g, F.H, k, x, y, z));
    c = k == 0 ? v : c + v;
  }
  f.c = c;
  f.phi = double(F.PHI[node_index(g, x, y, z)]);
  f.mu = closure(K.q, c, f.phi);
  gradient_normal<L, double>(GlobalPhi<S, double>{g, F.PHI, x, y, z}, K.eps2, f.g, f.n);
  double nn = f.g[0] * f.g[0] + f.g[1] * f.g[1];
  if (L::D == 3) nn = nn + f.g[2] * f.g[2];
  f.s = sqrt(nn + K.eps2);
  return f;
}

template <class L, class LH, class Codec>
__device__ __forceinline__ NodeFwd<L> node_fwd(const Geo& g, const Coef<double>& K,
                                               const DevFwdState<Codec>& F, int x, int y, int z) {
  NodeFwd<L> f;
  double c = 0.0;
#pragma unroll
  for (int k = 0; k < LH::Q; ++k) {
    const double v = double(pull_dev<Codec, LH>(g, F.H, F.LAM, k, x, y, z));
    c = k == 0 ? v : c + v;
  }
  f.c = c;
  f.phi = double(F.PHI[node_index(g, x, y, z)]);
  f.mu = closure(K.q, c, f.phi);
  gradient_normal<L, double>(GlobalPhi<float, double>{g, F.PHI, x, y, z}, K.eps2, f.g, f.n);
  double nn = f.g[0] * f.g[0] + f.g[1] * f.g[1];
  if (L::D == 3) nn = nn + f.g[2] * f.g[2];
  f.s = sqrt(nn + K.eps2);
  return f;
}

// Derivatives of the closure mu(c, phi): 1 and c_s - c_l for equal
// curvatures; for general quadratic free energies, with
// mu = fac (c - phi m_l - (1 - phi) m_s), fac = E / (eps_s phi + eps_l (1 - phi)):
// d mu / dc = fac, d mu / dphi = -fac (eps_s - eps_l) / den r + fac (m_s - m_l).
__device__ __forceinline__ void closure_grad(const Coef<double>& K, double c, double phi,
                                             double& dmu_dc, double& dmu_dphi) {
  if (K.q.quad) {
    const double den = (K.q.eps_s * phi) + (K.q.eps_l * (1.0 - phi));
    const double fac = K.q.efac / den;
    const double r = (c - phi * K.q.m_l) - (1.0 - phi) * K.q.m_s;
    dmu_dc = fac;
    dmu_dphi = -fac * (K.q.eps_s - K.q.eps_l) / den * r + fac * (K.q.m_s - K.q.m_l);
  } else {
    dmu_dc = 1.0;
    dmu_dphi = K.q.cs - K.q.cl;
  }
}

// Bracket B(mu) of S_phi = p'(phi) B and its slope B'(mu): dc (mu - mu_eq) and
// dc, or k2 mu^2 / 2 - (m_l - m_s) mu - df_min and k2 mu - (m_l - m_s).
__device__ __forceinline__ void bracket_and_slope(const Coef<double>& K, double mu, double& B,
                                                  double& Bp) {
  if (K.fe_quad) {
    B = ((K.k2 * (mu * mu)) * 0.5 - (K.dml * mu)) - K.dfm;
    Bp = K.k2 * mu - K.dml;
  } else {
    B = K.dc * (mu - K.mueq_c);
    Bp = K.dc;
  }
}

// Adjoint of the phi sources G_k (given their adjoints Gb_k) and of the
// extra adjoint sbar_b of their zeroth moment, at (phi, mu, n).  Adds to
// phi_b, mu_b, n_b and returns the lambda adjoint.
template <class L>
__device__ __forceinline__ double sources_adj(const Coef<double>& K, double lam_M_W2, double phi,
                                              double mu, const double n[3], const double* Gb,
                                              double sbar_b, double& phi_b, double& mu_b,
                                              double nb[3]) {
  const double pp = phi * (1.0 - phi);
  // p' of the coupling takes phi limited to [0, 1] (zero derivative outside)
  const double pl = limit01(phi);
  const double ppl = pl * (1.0 - pl);
  const bool in01 = phi >= 0.0 && phi <= 1.0;
  double Gst_b = sbar_b, kphi_b = 0.0, Gdw_b = 0.0;
  if (K.counter_term) {
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      if (Gb == nullptr) break;
      const double wg = L::w[k] * Gb[k];
      Gst_b += wg;
      if (k != L::REST) {
        const double en = edot<L, double>(k, n[0], n[1], n[2]);
        kphi_b += en * wg;
        const double kphi = K.k4w * pp;
        if (L::ex[k]) nb[0] += (L::ex[k] > 0 ? 1.0 : -1.0) * kphi * wg;
        if (L::ey[k]) nb[1] += (L::ey[k] > 0 ? 1.0 : -1.0) * kphi * wg;
        if (L::D == 3 && L::ez[k]) nb[2] += (L::ez[k] > 0 ? 1.0 : -1.0) * kphi * wg;
      }
    }
  } else {
    double s = 0.0;
    if (Gb != nullptr) {
#pragma unroll
      for (int k = 0; k < L::Q; ++k) s += L::w[k] * Gb[k];
    }
    Gst_b += s;
    Gdw_b = s + sbar_b;
  }
  double B, Bp;
  bracket_and_slope(K, mu, B, Bp);
  const double Sphi = (6.0 * ppl) * B;
  const double ppl_b = (K.kst * 6.0 * B) * Gst_b;
  double pp_b = K.k4w * kphi_b;
  mu_b += (K.kst * 6.0 * ppl * Bp) * Gst_b;
  if (!K.counter_term) {
    pp_b += K.kdw * 2.0 * (1.0 - 2.0 * phi) * Gdw_b;
    phi_b += K.kdw * 2.0 * pp * (-2.0) * Gdw_b;
  }
  phi_b += (1.0 - 2.0 * phi) * pp_b;
  if (in01) phi_b += (1.0 - 2.0 * pl) * ppl_b;
  return -lam_M_W2 * Sphi * Gst_b;
}

// Adjoint of the normal n = g / s: adds the gradient adjoint to gb.
template <class L>
__device__ __forceinline__ void normal_adj(const NodeFwd<L>& f, const double nb[3], double gb[3]) {
  const double nd = f.n[0] * nb[0] + f.n[1] * nb[1] + (L::D == 3 ? f.n[2] * nb[2] : 0.0);
  for (int a = 0; a < L::D; ++a) gb[a] += (nb[a] - f.n[a] * nd) / f.s;
}

// Gather of the transposed gradient stencil at node (x, y, z):
// sum over k != rest and over the nodes q with stencil(q + e_k) = (x, y, z)
// of (1 / xi_s^2) w_k e_k . gb(q).
__device__ __forceinline__ int preimage(int z, int e, int n, int bc, int out[2]) {
  if (!bc) {
    int v = z - e;
    v = v < 0 ? v + n : (v >= n ? v - n : v);
    out[0] = v;
    return 1;
  }
  int m = 0;
  if (e == 0) {
    out[m++] = z;
  } else if (e > 0) {
    if (z - 1 >= 0) out[m++] = z - 1;
    if (z == n - 1) out[m++] = z;
  } else {
    if (z + 1 <= n - 1) out[m++] = z + 1;
    if (z == 0) out[m++] = z;
  }
  return m;
}

template <class L>
__device__ __forceinline__ double stencil_adj_gather(const Geo& g, const double* gb3, int x, int y,
                                                     int z) {
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    if (k == L::REST) continue;
    int px[2], py[2], pz[2];
    const int mx = preimage(x, L::ex[k], g.nx, g.bcx, px);
    const int my = preimage(y, L::ey[k], g.ny, g.bcy, py);
    const int mz = L::D == 3 ? preimage(z, L::ez[k], g.nz, g.bcz, pz) : (pz[0] = z, 1);
    for (int a = 0; a < mx; ++a)
      for (int b = 0; b < my; ++b)
        for (int c = 0; c < mz; ++c) {
          const int64_t q = node_index(g, px[a], py[b], pz[c]);
          const double e_g = edot<L, double>(k, gb3[q], gb3[g.N + q], L::D == 3 ? gb3[2 * g.N + q] : 0.0);
          acc += L::inv_cs2 * L::w[k] * e_g;
        }
  }
  return acc;
}

// --------------------------------------------------------------------------

// The same gather on a periodic grid: one preimage per population, x - e_k.
template <class L>
__device__ __forceinline__ double stencil_adj_gather_at(const Geo& g, const double* gb3,
                                                        const AdjAddrPeriodic& a) {
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    if (k == L::REST) continue;
    const int64_t q = a.node(-L::ex[k], -L::ey[k], -L::ez[k]);
    const double e_g = edot<L, double>(k, gb3[q], gb3[g.N + q], L::D == 3 ? gb3[2 * g.N + q] : 0.0);
    acc += L::inv_cs2 * L::w[k] * e_g;
  }
  return acc;
}
template <class L>
__device__ __forceinline__ double stencil_adj_gather_at(const Geo& g, const double* gb3,
                                                        const AdjAddrGeneral& a) {
  return stencil_adj_gather<L>(g, gb3, a.x, a.y, a.z);
}

// Adjoint of G' in slot (k, x, y, z), gathered from the previous set.
template <class L>
__device__ __forceinline__ double gather_Gb(const Geo& g, const AdjSet& P, int k, int x, int y, int z) {
  int dx, dy, dz;
  const int kk = push_dest<L>(g, k, x, y, z, dx, dy, dz);
  return P.A1[pop_index<L>(g, kk, dx, dy, dz)] + P.B2[node_index(g, dx, dy, dz)];
}

// kGen: the general instantiation keeps the scheme flags (h^eq,alt, general
// free energies) of the run; the basic one fixes them off at compile time.
// The two halves of a reverse step at one node (the two kernels below).
//
// reverse_g: the reverse of the g collision of step n+1.  Writes the adjoint
// of the node's pulled g~^{n+1} (C.A1) when write_a1 is set, and returns the
// adjoint of grad phi^{n+1} with the previous step's B3 added (a2), of c^{n+1}
// (a3), the local adjoint of phi^{n+1} with the previous step's B4 added (a4),
// and the lambda adjoint (lb).  The h collision of step n+1 (previous reverse
// step) also used grad phi^{n+1} and phi^{n+1}: their adjoints are added here,
// so that the second half applies the transposed stencil once.
template <class L, class LH, class FS, class Addr>
__device__ __forceinline__ void reverse_g(const Geo& g, const Coef<double>& K, double lam_M_W2,
                                          const FS& S1, const AdjSet& P, const AdjSet& C,
                                          const Addr& ad, int z, bool write_a1, double (&a2)[3],
                                          double& a3, double& a4, double& lb) {
  const int64_t i = ad.self();
  const NodeFwd<L> f = node_fwd_at<L, LH>(K, S1, ad);  // c^{n+1}, mu^{n+1}, ...
  const double om = K.omega_g;
  double Gb[L::Q];
  double phi_b = 0.0, mu_b = 0.0, nb[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    int64_t dpop, dnode;
    ad.template push<L>(k, dpop, dnode);
    const double a = P.A1[dpop] + P.B2[dnode];
    if (write_a1)
      C.A1[((int64_t)z * L::Q + k) * ((int64_t)g.nx * g.ny) + (i - (int64_t)z * g.nx * g.ny)] =
          (1.0 - om) * a;
    Gb[k] = (1.0 - 0.5 * om) * a;
    phi_b += om * L::w[k] * a;
  }
  lb = sources_adj<L>(K, lam_M_W2, f.phi, f.mu, f.n, Gb, 0.0, phi_b, mu_b, nb);
  double gb[3] = {0.0, 0.0, 0.0};
  normal_adj<L>(f, nb, gb);
  for (int a = 0; a < 3; ++a) a2[a] = a < L::D ? gb[a] + P.B3[a * g.N + i] : 0.0;
  double dmu_dc, dmu_dphi;
  closure_grad(K, f.c, f.phi, dmu_dc, dmu_dphi);
  a3 = dmu_dc * mu_b;   // adjoint of c^{n+1}
  phi_b += dmu_dphi * mu_b;  // closure
  a4 = phi_b + P.B4[i];
}

// reverse_h: the reverse of the h collision of step n and of phi^{n+1} =
// sum g~^{n+1} + S^n / 2.  a3_at(k, dnode): the a3 of the node that pulls
// slot k of this node (dnode its global index); p1b: the adjoint of
// phi^{n+1} at this node gathered so far (a4 and the transposed stencil of
// a2).  Writes B1 .. B4 of the node into C and accumulates its parameter
// adjoints.
template <class L, class LH, class FS, class Addr, class FA3>
__device__ __forceinline__ void reverse_h(const Geo& g, const Coef<double>& K, double lam_M_W2,
                                          const FS& S0, const FS& S1, const AdjSet& P,
                                          const AdjSet& C, const AdjWork& w, const Addr& ad, int z,
                                          const FA3& a3_at, double p1b) {
  const int64_t i = ad.self();
  // total adjoint of h~*^n in this node's slots
  double Hb[LH::Q];
#pragma unroll
  for (int k = 0; k < LH::Q; ++k) {
    int64_t dpop, dnode;
    ad.template push<LH>(k, dpop, dnode);
    Hb[k] = P.B1[dpop] + a3_at(k, dnode);
  }
  // forward quantities of step n
  const NodeFwd<L> f = node_fwd_at<L, LH>(K, S0, ad);
  const double phi1 = double(S1.PHI[i]);
  const double dtphi = phi1 - f.phi;
  const double oh = K.omega_h;
  const double Dp = K.Dp;
  // D = D_l q + D_s (1 - q), q = phi limited to [0, 1]
  const double qd = limit01(f.phi);
  const double D = (K.Dl * qd) + (K.Ds * (1.0 - qd));
  const bool q_in = f.phi >= 0.0 && f.phi <= 1.0;
  // reverse of h* = (1 - oh) h + oh heq + (1 - oh/2) H
  double hb[LH::Q];
  double c_b = 0.0, lam_b = 0.0, Fb[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < LH::Q; ++k) {
    hb[k] = (1.0 - oh) * Hb[k];
    const double heq_b = oh * Hb[k];
    if (k == LH::REST) {
      c_b += heq_b;
      lam_b += -(1.0 - LH::w[k]) * heq_b;
    } else {
      lam_b += LH::w[k] * heq_b;
      // the flux enters through H_k = gamma w_k e_k.F (source scheme) or
      // through h^eq,alt_k = w_k (Lambda + e_k.F / xi_s^2)
      const double HHb = K.h_alt ? heq_b * (LH::w[k] * LH::inv_cs2)
                                 : (1.0 - 0.5 * oh) * Hb[k] * (K.gamma * LH::w[k]);
      if (LH::ex[k]) Fb[0] += (LH::ex[k] > 0 ? HHb : -HHb);
      if (LH::ey[k]) Fb[1] += (LH::ey[k] > 0 ? HHb : -HHb);
      if (LH::D == 3 && LH::ez[k]) Fb[2] += (LH::ez[k] > 0 ? HHb : -HHb);
    }
  }
  double mu_b = 0.0, phi_b = 0.0, dl_b = 0.0, gb[3] = {0.0, 0.0, 0.0}, nb[3] = {0.0, 0.0, 0.0};
  // Lambda = gamma D mu
  mu_b += K.gamma * D * lam_b;
  const double D_b = K.gamma * f.mu * lam_b;
  if (q_in) phi_b += (K.Dl - K.Ds) * D_b;
  dl_b += qd * D_b;
  // F = mu D' grad + jfac dtphi n
  const double gF = f.g[0] * Fb[0] + f.g[1] * Fb[1] + (L::D == 3 ? f.g[2] * Fb[2] : 0.0);
  mu_b += Dp * gF;
  dl_b += f.mu * gF;
  for (int a = 0; a < L::D; ++a) gb[a] += f.mu * Dp * Fb[a];
  if (K.anti_trapping) {
    const double nF = f.n[0] * Fb[0] + f.n[1] * Fb[1] + (L::D == 3 ? f.n[2] * Fb[2] : 0.0);
    // j_at = jf dphi/dt n, jf = a W dc, or a W (ks mu + m_s - m_l)
    const double jf = K.fe_quad ? K.aW * ((K.ks * f.mu + K.ms) - K.ml) : K.jfac;
    const double dt_b = jf * nF;
    for (int a = 0; a < L::D; ++a) nb[a] += jf * dtphi * Fb[a];
    if (K.fe_quad) mu_b += K.aW * K.ks * dtphi * nF;
    p1b += dt_b;
    phi_b -= dt_b;
  }
  // phi^{n+1} = sum g~^{n+1} + sbar^n / 2
  const double lb = sources_adj<L>(K, lam_M_W2, f.phi, f.mu, f.n, nullptr, 0.5 * p1b, phi_b, mu_b, nb);
  normal_adj<L>(f, nb, gb);
  // closure and c^n = sum h~^n
  {
    double dmu_dc, dmu_dphi;
    closure_grad(K, f.c, f.phi, dmu_dc, dmu_dphi);
    c_b += dmu_dc * mu_b;
    phi_b += dmu_dphi * mu_b;
  }
#pragma unroll
  for (int k = 0; k < LH::Q; ++k)
    C.B1[((int64_t)z * LH::Q + k) * ((int64_t)g.nx * g.ny) + (i - (int64_t)z * g.nx * g.ny)] = hb[k] + c_b;
  C.B2[i] = p1b;
  for (int a = 0; a < 3; ++a) C.B3[a * g.N + i] = gb[a];
  C.B4[i] = phi_b;
  w.lamb[i] += lb;
  w.dlb[i] += dl_b;
}

// kPer: every axis periodic (AdjAddrPeriodic), else any boundary.
template <class L, class LH, class FS, bool kGen, bool kPer>
__global__ void __launch_bounds__(256) k_adj_ra(Geo g, Coef<double> Kin, double lam_M_W2,
                                                FS S1, AdjSet P, AdjSet C, AdjWork w) {
  const Coef<double> K = variant<kGen>(Kin);
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  using Addr = std::conditional_t<kPer, AdjAddrPeriodic, AdjAddrGeneral>;
  const Addr ad(g, x, y, z);
  const int64_t i = ad.self();
  double a2[3], a3, a4, lb;
  reverse_g<L, LH>(g, K, lam_M_W2, S1, P, C, ad, z, true, a2, a3, a4, lb);
  for (int a = 0; a < L::D; ++a) w.A2[a * g.N + i] = a2[a];
  w.A3[i] = a3;
  w.A4[i] = a4;
  w.lamb[i] += lb;
}

template <class L, class LH, class FS, bool kGen, bool kPer>
__global__ void __launch_bounds__(256) k_adj_rb(Geo g, Coef<double> Kin, double lam_M_W2,
                                                FS S0, FS S1, AdjSet P, AdjSet C, AdjWork w) {
  const Coef<double> K = variant<kGen>(Kin);
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  using Addr = std::conditional_t<kPer, AdjAddrPeriodic, AdjAddrGeneral>;
  const Addr ad(g, x, y, z);
  const int64_t i = ad.self();
  // adjoint of phi^{n+1} at this node (A2, A4 hold both collisions' parts)
  const double p1b = w.A4[i] + stencil_adj_gather_at<L>(g, w.A2, ad);
  auto a3_at = [&](int, int64_t dnode) { return w.A3[dnode]; };
  reverse_h<L, LH>(g, K, lam_M_W2, S0, S1, P, C, w, ad, z, a3_at, p1b);
}

// Seed: the adjoint of S_K from dJ/dphi^K and dJ/dc^K (c^K = sum of the
// pulled H), written as a set the first reverse step gathers from:
// Gb = 0, Hb(slot) = dJ/dc^K(dest), Pb = dJ/dphi^K.
template <class L, class LH>
__global__ void __launch_bounds__(256) k_adj_seed(Geo g, const double* __restrict__ phib,
                                                  const double* __restrict__ cb, AdjSet P, AdjWork w) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t i = node_index(g, x, y, z);
  const double cv = cb ? cb[i] : 0.0;
#pragma unroll
  for (int k = 0; k < L::Q; ++k) P.A1[pop_index<L>(g, k, x, y, z)] = 0.0;
#pragma unroll
  for (int k = 0; k < LH::Q; ++k) P.B1[pop_index<LH>(g, k, x, y, z)] = cv;
  P.B2[i] = 0.0;
  for (int a = 0; a < 3; ++a) P.B3[a * g.N + i] = 0.0;
  P.B4[i] = phib ? phib[i] : 0.0;
  w.lamb[i] = 0.0;
  w.dlb[i] = 0.0;
}

// Adjoint of the initialisation (phi0, c0) -> S_0, local part: writes the
// adjoint of c0 and, in B4 / B3, the local part of the adjoint of phi0 and the
// adjoint of grad phi0.
template <class L, class LH>
__global__ void __launch_bounds__(256) k_adj_init_a(Geo g, Coef<double> K, double lam_M_W2,
                                                    const double* __restrict__ phi0,
                                                    const double* __restrict__ c0, AdjSet P,
                                                    AdjSet C, AdjWork w, double* __restrict__ c0b) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t i = node_index(g, x, y, z);
  const double phi = phi0[i], cin = c0[i];
  NodeFwd<L> f;
  f.phi = phi;
  gradient_normal<L, double>(GlobalPhi<double, double>{g, phi0, x, y, z}, K.eps2, f.g, f.n);
  {
    double nn = f.g[0] * f.g[0] + f.g[1] * f.g[1];
    if (L::D == 3) nn = nn + f.g[2] * f.g[2];
    f.s = sqrt(nn + K.eps2);
  }
  const double mu0 = closure(K.q, cin, phi);
  // forward h~^0 and c^0
  double F[3];
  h_flux<L, double>(K, mu0, f.g, f.n, 0.0, false, F);
  const double lam = h_lambda<double>(K, phi, mu0);
  double c = 0.0;
#pragma unroll
  for (int k = 0; k < LH::Q; ++k) {
    const double hv = h_initial<LH, double>(K, k, cin, lam, F);
    c = k == 0 ? hv : c + hv;
  }
  const double mu = closure(K.q, c, phi);
  // adjoints of the pulled h~^0 (from H of S_0) and of G of S_0
  double hb[LH::Q], Gb[L::Q], g0b[L::Q];
  double phi_b = P.B4[i] + stencil_adj_gather<L>(g, P.B3, x, y, z);
  double mu_b = 0.0, mu0_b = 0.0, nb[3] = {0.0, 0.0, 0.0};
  double lb = 0.0;
  const double om = K.omega_g;
#pragma unroll
  for (int k = 0; k < LH::Q; ++k) hb[k] = P.B1[pop_index<LH>(g, k, x, y, z)];  // gathered Hb
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    const double gsb = gather_Gb<L>(g, P, k, x, y, z);
    g0b[k] = (1.0 - om) * gsb;
    Gb[k] = (1.0 - 0.5 * om) * gsb;
    phi_b += om * L::w[k] * gsb;
  }
  // g collision at time 0 (sources at phi, mu(c^0), n)
  lb += sources_adj<L>(K, lam_M_W2, phi, mu, f.n, Gb, 0.0, phi_b, mu_b, nb);
  double dmu_dc, dmu_dphi;
  closure_grad(K, c, phi, dmu_dc, dmu_dphi);
  const double c_b = dmu_dc * mu_b;  // c^0 = sum h~^0
  phi_b += dmu_dphi * mu_b;
  // g~^0 = w phi - G^0 / 2
  double G0b[L::Q];
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    phi_b += L::w[k] * g0b[k];
    G0b[k] = -0.5 * g0b[k];
  }
  lb += sources_adj<L>(K, lam_M_W2, phi, mu0, f.n, G0b, 0.0, phi_b, mu0_b, nb);
  // h~^0 = heq(c0, Lambda0) - H^0 / 2
  double cin_b = 0.0, lam_b = 0.0, Fb[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < LH::Q; ++k) {
    const double hk = hb[k] + c_b;
    if (k == LH::REST) {
      cin_b += hk;
      lam_b += -(1.0 - LH::w[k]) * hk;
    } else {
      lam_b += LH::w[k] * hk;
      // h~^0 = h^eq - H/2, or h^eq,alt
      const double HHb = K.h_alt ? hk * (LH::w[k] * LH::inv_cs2) : -0.5 * hk * (K.gamma * LH::w[k]);
      if (LH::ex[k]) Fb[0] += (LH::ex[k] > 0 ? HHb : -HHb);
      if (LH::ey[k]) Fb[1] += (LH::ey[k] > 0 ? HHb : -HHb);
      if (LH::D == 3 && LH::ez[k]) Fb[2] += (LH::ez[k] > 0 ? HHb : -HHb);
    }
  }
  const double qd = limit01(phi);
  const double D = (K.Dl * qd) + (K.Ds * (1.0 - qd));
  double dl_b = 0.0, gb[3] = {0.0, 0.0, 0.0};
  mu0_b += K.gamma * D * lam_b;
  const double D_b = K.gamma * mu0 * lam_b;
  if (phi >= 0.0 && phi <= 1.0) phi_b += (K.Dl - K.Ds) * D_b;
  dl_b += qd * D_b;
  const double gF = f.g[0] * Fb[0] + f.g[1] * Fb[1] + (L::D == 3 ? f.g[2] * Fb[2] : 0.0);
  mu0_b += K.Dp * gF;
  dl_b += mu0 * gF;
  for (int d = 0; d < L::D; ++d) gb[d] += mu0 * K.Dp * Fb[d];
  normal_adj<L>(f, nb, gb);
  // mu0 = closure(c0, phi0)
  closure_grad(K, cin, phi, dmu_dc, dmu_dphi);
  cin_b += dmu_dc * mu0_b;
  phi_b += dmu_dphi * mu0_b;
  c0b[i] = cin_b;
  C.B4[i] = phi_b;
  for (int d = 0; d < 3; ++d) C.B3[d * g.N + i] = gb[d];
  w.lamb[i] += lb;
  w.dlb[i] += dl_b;
}

template <class L>
__global__ void __launch_bounds__(256) k_adj_init_b(Geo g, AdjSet C, double* __restrict__ phi0b) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t i = node_index(g, x, y, z);
  phi0b[i] = C.B4[i] + stencil_adj_gather<L>(g, C.B3, x, y, z);
}

// Deterministic sum of the two per-node accumulators (fixed launch shape).
__global__ void __launch_bounds__(kDiagThreads) k_adj_reduce(const double* __restrict__ a,
                                                             const double* __restrict__ b, int64_t n,
                                                             double* __restrict__ part) {
  __shared__ double ra[kDiagThreads], rb[kDiagThreads];
  double sa = 0.0, sb = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    sa = sa + a[i];
    sb = sb + b[i];
  }
  ra[threadIdx.x] = sa;
  rb[threadIdx.x] = sb;
  __syncthreads();
  for (int s = kDiagThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      ra[threadIdx.x] = ra[threadIdx.x] + ra[threadIdx.x + s];
      rb[threadIdx.x] = rb[threadIdx.x] + rb[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ra[0];
    part[2 * blockIdx.x + 1] = rb[0];
  }
}

__global__ void k_adj_reduce_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int b = 0; b < nb; ++b) {
      sa = sa + part[2 * b];
      sb = sb + part[2 * b + 1];
    }
    out[0] = sa;
    out[1] = sb;
  }
}

}  // namespace gplbm
