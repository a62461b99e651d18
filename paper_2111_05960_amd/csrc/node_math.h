// Per-node arithmetic of the coupled step, shared by every kernel schedule.
//
// Each expression is written in the exact order in which it is evaluated
// (the library is compiled with -ffp-contract=off), and moments are summed in
// ascending population index.  Multiplications by a lattice-vector component
// of 0 or +-1 are replaced by skipping or negating the operand, which is
// exact.  With these rules the FP64 path is reproducible to the last bit
// from the formulas alone.
//
//   closure           mu = mu_eq + (c - (c_l phi + c_s (1 - phi)))
//                     Eqs. (PotChim_Equilibirum), (Coexistence_Interpol);
//                     general quadratic free energies, Eq. (Closure):
//                     mu = (sqrt(eps_s eps_l) / (eps_s phi + eps_l (1 - phi)))
//                          ((c - phi m_l) - (1 - phi) m_s)
//   gradient          grad = (1/xi_s^2) sum_k w_k e_k d_k, d_k = (phi(x+e_k) - phi(x-e_k))/2
//                     Eqs. (DerivDirec_Grad), (Grad); central differences on D2Q5 / D3Q7
//   normal            n = grad / sqrt(|grad|^2 + eps_n^2)
//   phi sources       G^st = kst S_phi, S_phi = 6 p(1-p) dc (mu - mu_eq), p = phi on [0, 1],
//                     kst = -lambda M / W^2               Eqs. (SourceG_ST), (SourceTerm_Coexistence)
//                     general: S_phi = 6 p(1-p) ((k2 mu^2 / 2 - (m_l - m_s) mu) - df_min),
//                     k2 = (eps_l - eps_s) / sqrt(eps_l eps_s)   Eq. (SourceTerm)
//                     G^ct_k = (4/W) phi(1-phi) e_k.n     Eq. (SourceG_CT)
//                     G^dw = kdw 2 phi(1-phi)(1-2phi), kdw = -8 M / W^2   Eq. (SourceG_dw)
//                     G_k = w_k (G^st + G^curv)           Eq. (TermG)
//   g collision       g* = (g - omega_g ((g - w_k phi) + G_k/2)) + G_k
//                     Eq. (LBE_PhaseField_Eq), omega_g = 1/(M / xi_s^2 + 1/2)
//   h source          F = (mu (D_l - D_s)) grad + (a W dc) dphi/dt n,
//                     H_k = (gamma w_k) e_k.F             Eq. (SourceTerm_LBE_h)
//                     general: dc -> (ks mu + m_s) - m_l,
//                     ks = -(eps_s - eps_l) / sqrt(eps_s eps_l)   Eq. (Anti-Trapping_Quadratic)
//   h equilibrium     Lambda = (gamma D(phi)) mu, D = D_l q + D_s (1-q), q = phi on [0, 1]
//                     h^eq_rest = c - (1 - w_rest) Lambda, h^eq_k = w_k Lambda
//                     Eq. (Heq_Composition)
//   h collision       h* = (h - omega_h ((h - h^eq_k) + H_k/2)) + H_k
//                     Eq. (LBE_Composition), omega_h = 1/(1/(gamma xi_s^2) + 1/2)
//   h alternative     h^eq,alt_k = w_k (Lambda + e_k.F / xi_s^2) (k moving),
//                     h* = h - omega_h (h - h^eq,alt_k), no source
//                     Eqs. (LBE_Concent_Alt), (Seq_Concent_Alt)
#pragma once

#include <hip/hip_runtime.h>

#include "lattice.h"

namespace gplbm {

// Closure constants (always double).  quad = 0: equal curvatures (c_l, c_s,
// mu_eq); quad = 1: general quadratic free energies (efac = sqrt(eps_s eps_l)).
struct ClosureK {
  int quad;
  double cl, cs, mueq;
  double efac, eps_s, eps_l, m_s, m_l;
};

__device__ __forceinline__ double closure(const ClosureK& q, double c, double phi) {
  if (q.quad) {
    double fac = q.efac / ((q.eps_s * phi) + (q.eps_l * (1.0 - phi)));
    return fac * ((c - (phi * q.m_l)) - ((1.0 - phi) * q.m_s));
  }
  double cco = (q.cl * phi) + (q.cs * (1.0 - phi));
  return q.mueq + (c - cco);
}

// Per-run constants, computed once on the host in double and converted to
// the arithmetic type C of the kernel.
template <class C>
struct Coef {
  C omega_g, omega_h;  // BGK rates of the two LBEs
  double omega_g_d;    // omega_g in double (zeroth-moment balance of g)
  C dc;                // c_s^co - c_l^co
  C kst;               // -lambda M / W^2
  C k4w;               // 4 / W
  C kdw;               // -8 M / W^2
  C jfac;              // a W dc
  C Dp;                // D_l - D_s
  C Dl, Ds, gamma;
  C eps2;              // eps_n^2
  C mueq_c;            // mu_eq in C
  int counter_term, anti_trapping;
  int h_alt;           // 1: relaxation to h^eq,alt without source
  int fe_quad;         // 1: general quadratic free energies
  ClosureK q;          // closure
  C k2, dml, dfm;      // general source: (eps_l-eps_s)/sqrt(eps_l eps_s), m_l - m_s, df_min
  C ks, ms, ml, aW;    // general anti-trapping: -(eps_s-eps_l)/sqrt(eps_s eps_l), m_s, m_l, a W
};

// The coefficients a step kernel works with: the general instantiation
// (kGen) keeps the run's scheme flags, the basic one fixes them to the source
// scheme and equal curvatures at compile time, so that its code carries none
// of the general branches.
template <bool kGen, class C>
__device__ __forceinline__ Coef<C> variant(const Coef<C>& K) {
  Coef<C> R = K;
  if constexpr (!kGen) {
    R.h_alt = 0;
    R.fe_quad = 0;
    R.q.quad = 0;
  }
  return R;
}

// e_k . v with the zero components skipped and -1 as a negation.
template <class L, class C>
__device__ __forceinline__ C edot(int k, C v0, C v1, C v2) {
  C r = C(0);
  bool first = true;
  if (L::ex[k] != 0) {
    r = L::ex[k] > 0 ? v0 : -v0;
    first = false;
  }
  if (L::ey[k] != 0) {
    r = first ? (L::ey[k] > 0 ? v1 : -v1) : (L::ey[k] > 0 ? r + v1 : r - v1);
    first = false;
  }
  if (L::D == 3 && L::ez[k] != 0) {
    r = first ? (L::ez[k] > 0 ? v2 : -v2) : (L::ez[k] > 0 ? r + v2 : r - v2);
  }
  return r;
}

// Gradient and normal from an accessor phi_at(dx, dy, dz) returning the
// phase field at x + (dx, dy, dz) (ghost rule already applied).
template <class L, class C, class F>
__device__ __forceinline__ void gradient_normal(const F& phi_at, C eps2, C g[3], C n[3]) {
  C a0 = C(0), a1 = C(0), a2 = C(0);
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    if (k == L::REST) continue;
    C d = C(0.5) * (phi_at(L::ex[k], L::ey[k], L::ez[k]) -
                    phi_at(-L::ex[k], -L::ey[k], -L::ez[k]));
    C wd = C(L::w[k]) * d;
    if (L::ex[k] > 0) a0 = a0 + wd;
    if (L::ex[k] < 0) a0 = a0 - wd;
    if (L::ey[k] > 0) a1 = a1 + wd;
    if (L::ey[k] < 0) a1 = a1 - wd;
    if (L::D == 3) {
      if (L::ez[k] > 0) a2 = a2 + wd;
      if (L::ez[k] < 0) a2 = a2 - wd;
    }
  }
  g[0] = C(L::inv_cs2) * a0;
  g[1] = C(L::inv_cs2) * a1;
  g[2] = C(L::inv_cs2) * a2;
  C nn = g[0] * g[0] + g[1] * g[1];
  if (L::D == 3) nn = nn + g[2] * g[2];
  C den = sqrt(nn + eps2);
  n[0] = g[0] / den;
  n[1] = g[1] / den;
  n[2] = L::D == 3 ? g[2] / den : C(0);
}

// phi limited to [0, 1], the argument of the interpolation functions p' (of
// S_phi) and q (of D): the paper defines them on the range of the phase
// field, which the discrete phi overshoots by ~1e-3 at interfaces; outside
// it the unlimited q makes the diffusivity negative and the unlimited p'
// reverses the coupling source.  phi itself is never limited.
template <class C>
__device__ __forceinline__ C limit01(C phi) {
  return phi < C(0) ? C(0) : (phi > C(1) ? C(1) : phi);
}

// Coupling source S_phi = p'(phi) * bracket.
template <class C>
__device__ __forceinline__ C coupling(const Coef<C>& K, C pprime, C mu) {
  if (K.fe_quad) return pprime * (((K.k2 * (mu * mu)) * C(0.5) - (K.dml * mu)) - K.dfm);
  return (pprime * K.dc) * (mu - K.mueq_c);
}

// Zeroth moment of the phi source at a node (closed form): G^st, plus G^dw
// without the counter term.
template <class C>
__device__ __forceinline__ C source_moment(const Coef<C>& K, C phi, C mu) {
  C pp = phi * (C(1) - phi);
  C pl = limit01(phi);
  C pprime = C(6) * (pl * (C(1) - pl));
  C Sphi = coupling<C>(K, pprime, mu);
  C Gst = K.kst * Sphi;
  if (K.counter_term) return Gst;
  C wdw = C(2) * (pp * (C(1) - C(2) * phi));
  C Gdw = K.kdw * wdw;
  return Gst + Gdw;
}

// Population sources G_k of the phi-LBE.
template <class L, class C>
__device__ __forceinline__ void phi_sources(const Coef<C>& K, C phi, C mu, const C n[3],
                                            C G[L::Q]) {
  C pp = phi * (C(1) - phi);
  C pl = limit01(phi);
  C pprime = C(6) * (pl * (C(1) - pl));
  C Sphi = coupling<C>(K, pprime, mu);
  C Gst = K.kst * Sphi;
  if (K.counter_term) {
    C kphi = K.k4w * pp;
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      if (k == L::REST)
        G[k] = C(L::w[k]) * Gst;
      else
        G[k] = C(L::w[k]) * (Gst + kphi * edot<L, C>(k, n[0], n[1], n[2]));
    }
  } else {
    C wdw = C(2) * (pp * (C(1) - C(2) * phi));
    C Gdw = K.kdw * wdw;
    C s = Gst + Gdw;
#pragma unroll
    for (int k = 0; k < L::Q; ++k) G[k] = C(L::w[k]) * s;
  }
}

template <class L, class C>
__device__ __forceinline__ C g_collide(const Coef<C>& K, int k, C g, C phi, C Gk) {
  C t = (g - C(L::w[k]) * phi) + C(0.5) * Gk;
  return (g - K.omega_g * t) + Gk;
}

// Flux F = (mu D') grad + j_at of the h source (j_at only when enabled).
template <class L, class C>
__device__ __forceinline__ void h_flux(const Coef<C>& K, C mu, const C g[3], const C n[3],
                                       C dtphi, bool with_at, C F[3]) {
  C md = mu * K.Dp;
  C jf = K.jfac;
  if (K.fe_quad) jf = K.aW * (((K.ks * mu) + K.ms) - K.ml);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    F[a] = md * g[a];
    if (with_at) F[a] = F[a] + (jf * dtphi) * n[a];
  }
}

template <class C>
__device__ __forceinline__ C h_lambda(const Coef<C>& K, C phi, C mu) {
  C q = limit01(phi);
  C D = (K.Dl * q) + (K.Ds * (C(1) - q));
  return (K.gamma * D) * mu;
}

template <class L, class C>
__device__ __forceinline__ C h_eq(int k, C c, C lam) {
  if (k == L::REST) return c - C(1.0 - L::w[k]) * lam;
  return C(L::w[k]) * lam;
}

template <class L, class C>
__device__ __forceinline__ C h_source(const Coef<C>& K, int k, const C F[3]) {
  if (k == L::REST) return C(0);
  return (K.gamma * C(L::w[k])) * edot<L, C>(k, F[0], F[1], F[2]);
}

template <class L, class C>
__device__ __forceinline__ C h_collide(const Coef<C>& K, int k, C h, C heq, C Hk) {
  if (k == L::REST) {
    C t = h - heq;
    return h - K.omega_h * t;
  }
  C t = (h - heq) + C(0.5) * Hk;
  return (h - K.omega_h * t) + Hk;
}

// Alternative equilibrium with the flux F folded into the moving populations.
template <class L, class C>
__device__ __forceinline__ C h_eq_alt(int k, C c, C lam, const C F[3]) {
  if (k == L::REST) return c - C(1.0 - L::w[k]) * lam;
  return C(L::w[k]) * (lam + edot<L, C>(k, F[0], F[1], F[2]) / C(L::cs2));
}

// Post-collision h_k of either scheme.
template <class L, class C>
__device__ __forceinline__ C h_update(const Coef<C>& K, int k, C h, C c, C lam, const C F[3]) {
  if (K.h_alt) {
    C t = h - h_eq_alt<L, C>(k, c, lam, F);
    return h - K.omega_h * t;
  }
  return h_collide<L, C>(K, k, h, h_eq<L, C>(k, c, lam), h_source<L, C>(K, k, F));
}

// Post-collision h stored in a type S narrower than double (FP32 storage):
// the rest population takes the value that makes the stored populations sum,
// in double, to the c the node received (the collision conserves c exactly
// in arithmetic, so this takes the rounding of the other stored populations
// out of the solute balance), and the rounding residue of the rest
// population itself is added to the first moving population before that one
// is rounded, so one rounding of a moving population (a few 1e-3 of c) per
// node and step remains.  At a stationary node the same residue recurs every
// step, so an unbalanced rest population alone drifts the solute linearly
// (1.6e-6 relative over 5000 steps on a 64^3 porous crop).  hs holds the
// values as stored (rounded to S); no-op for double storage.
template <class LH, class S, class C>
__device__ __forceinline__ void balance_rest(C (&hs)[LH::Q], double c_in) {
  if constexpr (sizeof(S) < sizeof(double)) {
    constexpr int km = LH::REST == 0 ? 1 : 0;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < LH::Q; ++k)
      if (k != LH::REST) s = s + double(hs[k]);
    const double x = c_in - s;
    const S r = S(x);
    hs[LH::REST] = C(r);
    hs[km] = C(S(double(hs[km]) + (x - double(r))));
  }
}

// Post-collision g stored in a type S narrower than double: the rest
// population takes the value that makes the stored populations sum, in
// double, to the zeroth moment of the collision in exact arithmetic,
//   sum_k g*_k = (1 - omega_g) sum_k g_k + omega_g phi + (1 - omega_g / 2) sbar
// (sum_k w_k = 1 and sum_k G_k = sbar, the counter-term parts cancelling).
// In float the weights themselves do not sum to 1 (1 + 1.5e-8 on D3Q19) and
// every population is rounded the same way from step to step near a
// stationary interface, which biases phi along the neutral translation mode
// of the interface; with the balance one rounding of the rest population per
// node and step remains.  sg: the double sum of the g_k the collision took;
// gs holds the values as stored (rounded to S); no-op for double storage.
template <class L, class S, class C>
__device__ __forceinline__ void balance_g_rest(const Coef<C>& K, C (&gs)[L::Q], double sg, C phi,
                                               C sbar) {
  if constexpr (sizeof(S) < sizeof(double)) {
    const double wg = K.omega_g_d;
    const double m0 = ((1.0 - wg) * sg + wg * double(phi)) + (1.0 - 0.5 * wg) * double(sbar);
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < L::Q; ++k)
      if (k != L::REST) s = s + double(gs[k]);
    gs[L::REST] = C(S(m0 - s));
  }
}

// Initial h~^0_k of either scheme: the equilibrium shifted by -H_k/2, or
// h^eq,alt itself (no source, no shift).
template <class L, class C>
__device__ __forceinline__ C h_initial(const Coef<C>& K, int k, C c, C lam, const C F[3]) {
  if (K.h_alt) return h_eq_alt<L, C>(k, c, lam, F);
  return h_eq<L, C>(k, c, lam) - C(0.5) * h_source<L, C>(K, k, F);
}

}  // namespace gplbm
