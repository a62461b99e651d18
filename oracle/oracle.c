/*
 * Plain FP64 CPU oracle of the coupled phi / c lattice-Boltzmann step of the
 * grand-potential phase-field model of dissolution and precipitation
 * (Boutin, Verdier & Cartalade, arXiv:2111.05960).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU library is
 * checked against.  Only tests/, the smoke entry and the CPU-baseline leg of
 * the benchmark load it.  It shares no code, header or constant table with
 * the HIP library, and the product path never calls it.
 *
 * Everything is double precision, in lattice units (dx = dt = 1, s = 1;
 * xi_s^2 = 1/3, or 1/4 on D3Q7).  Arrays are structure-of-arrays f[k][z][y][x], x fastest.
 * The state at time n is the "natural" one: post-streaming populations
 * g~^n_k(x), h~^n_k(x) and the phase field phi^n(x).
 *
 * One step n -> n+1 follows the paper's order (Sec. 3.2 then Sec. 3.3):
 *   S1  c^n = sum_k h~^n_k ; mu^n by the closure, Eq. (PotChim_Equilibirum)
 *       with Eq. (Coexistence_Interpol), h(phi) = phi (equal curvatures
 *       eps_s = eps_l), or Eq. (Closure) for general quadratic free
 *       energies.
 *   S2  directional derivatives and the gradient, Eqs. (DerivDirec_Grad) and
 *       (Grad), grad = (1 / xi_s^2) sum_k w_k e_k d_k on the lattice of g
 *       (central differences on D2Q5 / D3Q7); normal
 *       n = grad / sqrt(|grad|^2 + eps_n^2).
 *   S3  sources of the phi-LBE, Eqs. (TermG), (SourceG_ST), (SourceG_dw) or
 *       (SourceG_CT), with S_phi from Eq. (SourceTerm_Equilibrium) (general:
 *       Eq. (SourceTerm)) and p'(phi) = 6 phi (1 - phi) (Tab. 2).
 *   S4  BGK collision with the trapezoidal source, Eq. (LBE_PhaseField_Eq),
 *       g~eq = w_k phi - G_k / 2, 1/(tau_g + 1/2) with M_phi = xi_s^2 tau_g
 *       (tau_g = 3 M_phi; 4 M_phi on D3Q7, so that the mobility is M_phi
 *       on every lattice, as for tau_h).
 *   S5  streaming (periodic wrap or halfway bounce-back).
 *   S6  phi^{n+1} = sum_k g~^{n+1}_k + (1/2) sum_k G_k, Eq. (Moment_Phi), with
 *       the source moment taken from this step's collision at the same node.
 *   S7  dphi/dt = phi^{n+1} - phi^n (explicit Euler, h solved after g) and the
 *       anti-trapping current, Eq. (Anti-trapping_Equilibrium) (general:
 *       Eq. (Anti-Trapping_Quadratic)).
 *   S8  BGK collision of h, Eqs. (LBE_Composition), (Heq_Composition) and
 *       (SourceTerm_LBE_h), with D(phi) = D_l q + D_s (1 - q), q = phi on [0, 1], and
 *       1/(tau_h + 1/2), tau_h = 1 / (gamma xi_s^2): 3 / gamma on D2Q9,
 *       D3Q19 and D2Q5 (xi_s^2 = 1/3), 4 / gamma on D3Q7 (xi_s^2 = 1/4), so
 *       that the diffusivity is D in every case.  Alternative scheme
 *       (h_scheme = ORC_H_EQ_ALT): Eqs. (LBE_Concent_Alt) and
 *       (Seq_Concent_Alt), relaxation to h^eq,alt with F folded into the
 *       moving populations, w_k (Lambda + e_k . F / xi_s^2), and no source.
 *   S9  streaming of h.
 *
 * Evaluation order.  Every floating-point expression below is written out in
 * the exact order in which it is evaluated (C evaluates left to right, and the
 * file is compiled with -ffp-contract=off), and every sum over k runs in
 * ascending population index.  The GPU library reproduces the same order, so
 * the two agree bit for bit in FP64 wherever the same operations are applied.
 *
 * Readings where the paper is silent (stated once here, applied below):
 *   - the source moment in S6 is the closed-form zeroth moment of G_k:
 *     G^st (+ G^dw), the counter-term contributions cancel pairwise;
 *   - the normal is regularised with eps_n;
 *   - at a zero-flux wall the neighbour value of phi used by S2 is the mirror
 *     copy (phi(-1) = phi(0), phi(n) = phi(n-1)), and streaming is halfway
 *     bounce-back (the wall wins over a periodic wrap on another axis);
 *   - the initial populations are the equilibria shifted by the variable
 *     change: g~^0 = w_k phi0 - G^0_k / 2, h~^0 = h^eq_k - H^0_k / 2 with no
 *     anti-trapping current (dphi/dt unknown at t = 0); with h^eq,alt there
 *     is no source, and h~^0 = h^eq,alt_k with the same F (no j_at);
 *   - the interpolation functions p (in S_phi) and q (in D) are defined by
 *     the paper on [0, 1], the range of the phase field; the discrete phi
 *     overshoots that range by ~1e-3 at interfaces, so p'(phi) and q(phi)
 *     are evaluated at phi limited to [0, 1] (phi itself is never
 *     limited): outside the range the unlimited q gives a negative
 *     diffusivity (D_s = 0, phi < 0), which makes the c-equation
 *     anti-diffusive, and the unlimited p' reverses the sign of the
 *     coupling source, which then drives phi further out;
 *   - the general free energies keep the paper's h(phi) = phi,
 *     q(phi) = phi + (1 - phi) D_s / D_l and a = a_at: the paper fixes these
 *     choices for eps_s = eps_l and defers eps_s != eps_l, so the same
 *     interpolations are taken there.
 * Parity unpinned: the source moment of S6, the initial populations and the
 * value of eps_n are such choices; no value the paper prints fixes them.
 * The pins check what follows from them (the recurrence of uniform fields,
 * the moments at t = 0, the Stefan front within its bar), and the GPU is held
 * to this file on them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "oracle.h"

/* ---------------------------------------------------------------------- */
/* Velocity sets.  D2Q9 follows the paper's numbering (Sec. 3.1).  D3Q19 is
 * not listed in the paper; its numbering is this oracle's convention and is
 * grouped by e_z: the five e_z=+1 vectors, the rest vector, the eight
 * in-plane moving vectors, the five e_z=-1 vectors.  The lighter sets for
 * h (the paper names D2Q5 and D3Q7 among the standard lattices, Sec. 3.1):
 * D2Q5 = the first five vectors of D2Q9, weights 1/3, 1/6 (xi_s^2 = 1/3);
 * D3Q7 grouped by e_z like D3Q19: (0,0,1), rest, +-x, +-y, (0,0,-1),
 * weights 1/4 (rest), 1/8 (xi_s^2 = 1/4).                                  */

static const int d2q9_e[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const double d2q9_w[9] = {
    4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

static const int d3q19_e[19][3] = {
    {0, 0, 1}, {1, 0, 1}, {-1, 0, 1}, {0, 1, 1}, {0, -1, 1},
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0},
    {0, 0, -1}, {-1, 0, -1}, {1, 0, -1}, {0, -1, -1}, {0, 1, -1}};
static const double d3q19_w[19] = {
    1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

static const int d2q5_e[5][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0}};
static const double d2q5_w[5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};
static const int d3q7_e[7][3] = {{0, 0, 1}, {0, 0, 0}, {1, 0, 0}, {-1, 0, 0},
                                 {0, 1, 0}, {0, -1, 0}, {0, 0, -1}};
static const double d3q7_w[7] = {1.0 / 8.0, 1.0 / 4.0, 1.0 / 8.0, 1.0 / 8.0,
                                 1.0 / 8.0, 1.0 / 8.0, 1.0 / 8.0};

struct orc_state {
  orc_params p;
  int Q, D, rest;           /* lattice of g (and of the gradient stencil) */
  double inv_cs2g;          /* 1 / xi_s^2 of the g lattice: 3, or 4 on D3Q7 */
  int e[19][3];
  int opp[19];
  double w[19];
  int Qh, resth;            /* lattice of h */
  int eh[19][3];
  int opph[19];
  double wh[19];
  double cs2h;              /* xi_s^2 of the h lattice */
  int64_t N;
  /* natural state */
  double *g, *h, *phi;
  /* per-step work arrays */
  double *gs, *hs, *phin, *c, *mu, *grad, *nrm, *sbar;
  int64_t step;
  int ready;
};

/* ---------------------------------------------------------------------- */

static int64_t node(const orc_state* s, int x, int y, int z) {
  return (int64_t)x + (int64_t)s->p.nx * ((int64_t)y + (int64_t)s->p.ny * z);
}

/* Neighbour coordinate along one axis for the gradient stencil: periodic wrap
 * or mirror copy at a zero-flux wall. */
static int stencil_coord(int v, int n, int bc) {
  if (v >= 0 && v < n) return v;
  if (bc == ORC_PERIODIC) return (v + n) % n;
  return v < 0 ? 0 : n - 1;
}

/* phi at x + d (d a lattice vector), with the S2 ghost rule. */
static double phi_at(const orc_state* s, const double* f, int x, int y, int z,
                     const int* d) {
  int xx = stencil_coord(x + d[0], s->p.nx, s->p.bc[0]);
  int yy = stencil_coord(y + d[1], s->p.ny, s->p.bc[1]);
  int zz = stencil_coord(z + d[2], s->p.nz, s->p.bc[2]);
  return f[node(s, xx, yy, zz)];
}

/* Source node of the pull x - e_k.  Returns 0 and sets *src when the source
 * lies in the domain (after periodic wrap), 1 when the population crosses a
 * zero-flux wall (halfway bounce-back). */
static int pull_source(const orc_state* s, const int (*e)[3], int x, int y,
                       int z, int k, int64_t* src) {
  int c3[3] = {x - e[k][0], y - e[k][1], z - e[k][2]};
  int n3[3] = {s->p.nx, s->p.ny, s->p.nz};
  for (int a = 0; a < 3; ++a) {
    if (c3[a] < 0 || c3[a] >= n3[a]) {
      if (s->p.bc[a] == ORC_ZERO_FLUX) return 1;
      c3[a] = (c3[a] + n3[a]) % n3[a];
    }
  }
  *src = node(s, c3[0], c3[1], c3[2]);
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Local pieces of the scheme (one node).                                  */

/* Closure, h(phi) = phi.  Equal curvatures, Eqs. (PotChim_Equilibirum) and
 * (Coexistence_Interpol): mu = mu_eq + (c - c_co(phi)),
 * c_co(phi) = c_l phi + c_s (1 - phi).  General quadratic free energies,
 * Eq. (Closure): mu = sqrt(eps_s eps_l) / (eps_s phi + eps_l (1 - phi))
 * (c - phi m_l - (1 - phi) m_s). */
static double closure(const orc_params* p, double c, double phi) {
  if (p->free_energy == ORC_FE_QUADRATIC) {
    double fac = sqrt(p->eps_s * p->eps_l) / ((p->eps_s * phi) + (p->eps_l * (1.0 - phi)));
    return fac * ((c - (phi * p->m_l)) - ((1.0 - phi) * p->m_s));
  }
  double cco = (p->c_l_co * phi) + (p->c_s_co * (1.0 - phi));
  return p->mu_eq + (c - cco);
}

/* Bracket of the coupling source for general quadratic free energies,
 * S_phi = p'(phi) * bracket, Eq. (SourceTerm):
 * ((eps_l - eps_s) / sqrt(eps_l eps_s)) mu^2 / 2 - (m_l - m_s) mu - df_min.
 * (Equal curvatures: dc (mu - mu_eq), Eq. (SourceTerm_Equilibrium).) */
static double coupling_bracket(const orc_params* p, double mu) {
  if (p->free_energy == ORC_FE_QUADRATIC) {
    double k2 = (p->eps_l - p->eps_s) / sqrt(p->eps_l * p->eps_s);
    return (((k2 * (mu * mu)) * 0.5) - ((p->m_l - p->m_s) * mu)) - p->df_min;
  }
  return (p->c_s_co - p->c_l_co) * (mu - p->mu_eq);
}

/* Composition jump of the anti-trapping current, j_at = a W jump dphi/dt n.
 * Equal curvatures, Eq. (Anti-trapping_Equilibrium): c_s_co - c_l_co.
 * General, Eq. (Anti-Trapping_Quadratic):
 * -((eps_s - eps_l) / sqrt(eps_s eps_l)) mu + m_s - m_l. */
static double at_jump(const orc_params* p, double mu) {
  if (p->free_energy == ORC_FE_QUADRATIC) {
    double ks = -((p->eps_s - p->eps_l) / sqrt(p->eps_s * p->eps_l));
    return ((ks * mu) + p->m_s) - p->m_l;
  }
  return p->c_s_co - p->c_l_co;
}

/* S2: gradient of phi at (x,y,z) by directional derivatives, and the
 * regularised normal. */
static void gradient_normal(const orc_state* s, const double* f, int x, int y,
                            int z, double* g3, double* n3) {
  double acc[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < s->Q; ++k) {
    if (k == s->rest) continue;
    int m[3] = {-s->e[k][0], -s->e[k][1], -s->e[k][2]};
    double dk = 0.5 * (phi_at(s, f, x, y, z, s->e[k]) - phi_at(s, f, x, y, z, m));
    for (int a = 0; a < s->D; ++a) {
      acc[a] = acc[a] + (s->w[k] * (double)s->e[k][a]) * dk;
    }
  }
  double nn = 0.0;
  for (int a = 0; a < 3; ++a) g3[a] = 0.0;
  for (int a = 0; a < s->D; ++a) {
    g3[a] = s->inv_cs2g * acc[a];
    nn = nn + g3[a] * g3[a];
  }
  double den = sqrt(nn + s->p.eps_n * s->p.eps_n);
  for (int a = 0; a < 3; ++a) n3[a] = 0.0;
  for (int a = 0; a < s->D; ++a) n3[a] = g3[a] / den;
}

/* e_k . v, in axis order. */
static double edot(const orc_state* s, int k, const double* v) {
  double r = 0.0;
  for (int a = 0; a < s->D; ++a) r = r + (double)s->e[k][a] * v[a];
  return r;
}

/* phi limited to [0, 1]: the argument of the interpolation functions p' and
 * q, which the paper defines on the range of the phase field. */
static double limit01(double phi) {
  if (phi < 0.0) return 0.0;
  if (phi > 1.0) return 1.0;
  return phi;
}

/* S3: population sources G_k of the phi-LBE and their zeroth moment Sbar. */
static void phi_sources(const orc_state* s, double phi, double mu,
                        const double* n3, double* G, double* sbar) {
  const orc_params* p = &s->p;
  /* G^st = -(lambda M / W^2) S_phi, p'(phi) of the interpolation p on
   * [0, 1] */
  double pl = limit01(phi);
  double pprime = 6.0 * (pl * (1.0 - pl));
  double Sphi;
  if (p->free_energy == ORC_FE_QUADRATIC)
    Sphi = pprime * coupling_bracket(p, mu);
  else /* S_phi = p'(phi) dc (mu - mu_eq) */
    Sphi = (pprime * (p->c_s_co - p->c_l_co)) * (mu - p->mu_eq);
  double Gst = -((p->lambda * p->M_phi) / (p->W * p->W)) * Sphi;
  if (p->counter_term) {
    /* G^ct_k = (4/W) phi (1 - phi) e_k . n */
    double kphi = (4.0 / p->W) * (phi * (1.0 - phi));
    for (int k = 0; k < s->Q; ++k) G[k] = s->w[k] * (Gst + kphi * edot(s, k, n3));
    *sbar = Gst;
  } else {
    /* G^dw = -(8 M / W^2) w'_dw, w'_dw = 2 phi (1 - phi) (1 - 2 phi) */
    double wdw = 2.0 * ((phi * (1.0 - phi)) * (1.0 - 2.0 * phi));
    double Gdw = -((8.0 * p->M_phi) / (p->W * p->W)) * wdw;
    for (int k = 0; k < s->Q; ++k) G[k] = s->w[k] * (Gst + Gdw);
    *sbar = Gst + Gdw;
  }
}

/* Equilibrium of h, Eq. (Heq_Composition), on the h lattice. */
static double h_equilibrium(const orc_state* s, int k, double c, double lam) {
  if (k == s->resth) return c - (1.0 - s->wh[k]) * lam;
  return s->wh[k] * lam;
}

/* Lambda = gamma D(phi) mu, D(phi) = D_l q + D_s (1 - q), q = phi on
 * [0, 1] (the interpolation D_l q(phi) of Eq. Mixed-Formulation). */
static double h_lambda(const orc_params* p, double phi, double mu) {
  double q = limit01(phi);
  double D = (p->D_l * q) + (p->D_s * (1.0 - q));
  return (p->gamma * D) * mu;
}

/* H_k = gamma w_k e_k . F, on the h lattice */
static double h_source(const orc_state* s, int k, const double* F) {
  double r = 0.0;
  for (int a = 0; a < s->D; ++a) r = r + (double)s->eh[k][a] * F[a];
  return (s->p.gamma * s->wh[k]) * r;
}

/* Alternative equilibrium, Eq. (Seq_Concent_Alt), on the h lattice: the rest
 * population as in Eq. (Heq_Composition), the moving ones
 * w_k (Lambda + e_k . F / xi_s^2). */
static double h_equilibrium_alt(const orc_state* s, int k, double c, double lam,
                                const double* F) {
  if (k == s->resth) return c - (1.0 - s->wh[k]) * lam;
  double r = 0.0;
  for (int a = 0; a < s->D; ++a) r = r + (double)s->eh[k][a] * F[a];
  return s->wh[k] * (lam + r / s->cs2h);
}

/* ---------------------------------------------------------------------- */

orc_state* orc_create(const orc_params* p) {
  if (!p) return NULL;
  if (p->lattice < ORC_D2Q9 || p->lattice > ORC_D3Q7) return NULL;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return NULL;
  if ((p->lattice == ORC_D2Q9 || p->lattice == ORC_D2Q5) && p->nz != 1) return NULL;
  if (p->h_lattice != 0 && p->h_lattice != 1) return NULL;
  if (p->h_scheme != ORC_H_SOURCE && p->h_scheme != ORC_H_EQ_ALT) return NULL;
  if (p->free_energy != ORC_FE_EQUAL && p->free_energy != ORC_FE_QUADRATIC) return NULL;
  if (p->free_energy == ORC_FE_QUADRATIC && !(p->eps_s > 0.0 && p->eps_l > 0.0)) return NULL;
  orc_state* s = (orc_state*)calloc(1, sizeof(orc_state));
  s->p = *p;
  s->inv_cs2g = 3.0;
  if (p->lattice == ORC_D2Q9) {
    s->Q = 9; s->D = 2; s->rest = 0;
    memcpy(s->e, d2q9_e, sizeof(d2q9_e));
    memcpy(s->w, d2q9_w, sizeof(d2q9_w));
    s->p.bc[2] = ORC_PERIODIC;
  } else if (p->lattice == ORC_D3Q19) {
    s->Q = 19; s->D = 3; s->rest = 5;
    memcpy(s->e, d3q19_e, sizeof(d3q19_e));
    memcpy(s->w, d3q19_w, sizeof(d3q19_w));
  } else if (p->lattice == ORC_D2Q5) {
    s->Q = 5; s->D = 2; s->rest = 0;
    memcpy(s->e, d2q5_e, sizeof(d2q5_e));
    memcpy(s->w, d2q5_w, sizeof(d2q5_w));
    s->p.bc[2] = ORC_PERIODIC;
  } else {
    s->Q = 7; s->D = 3; s->rest = 1;
    memcpy(s->e, d3q7_e, sizeof(d3q7_e));
    memcpy(s->w, d3q7_w, sizeof(d3q7_w));
    s->inv_cs2g = 4.0;
  }
  const int light_g = p->lattice == ORC_D2Q5 || p->lattice == ORC_D3Q7;
  for (int k = 0; k < s->Q; ++k)
    for (int j = 0; j < s->Q; ++j)
      if (s->e[j][0] == -s->e[k][0] && s->e[j][1] == -s->e[k][1] &&
          s->e[j][2] == -s->e[k][2])
        s->opp[k] = j;
  if (p->h_lattice == 0 || light_g) {
    s->Qh = s->Q; s->resth = s->rest;
    memcpy(s->eh, s->e, sizeof(s->e));
    memcpy(s->wh, s->w, sizeof(s->w));
    s->cs2h = p->lattice == ORC_D3Q7 ? 1.0 / 4.0 : 1.0 / 3.0;
  } else if (p->lattice == ORC_D2Q9) {
    s->Qh = 5; s->resth = 0;
    memcpy(s->eh, d2q5_e, sizeof(d2q5_e));
    memcpy(s->wh, d2q5_w, sizeof(d2q5_w));
    s->cs2h = 1.0 / 3.0;
  } else {
    s->Qh = 7; s->resth = 1;
    memcpy(s->eh, d3q7_e, sizeof(d3q7_e));
    memcpy(s->wh, d3q7_w, sizeof(d3q7_w));
    s->cs2h = 1.0 / 4.0;
  }
  for (int k = 0; k < s->Qh; ++k)
    for (int j = 0; j < s->Qh; ++j)
      if (s->eh[j][0] == -s->eh[k][0] && s->eh[j][1] == -s->eh[k][1] &&
          s->eh[j][2] == -s->eh[k][2])
        s->opph[k] = j;
  s->N = (int64_t)p->nx * p->ny * p->nz;
  int64_t N = s->N, Q = s->Q, Qh = s->Qh;
  s->g = (double*)calloc(Q * N, sizeof(double));
  s->h = (double*)calloc(Qh * N, sizeof(double));
  s->gs = (double*)calloc(Q * N, sizeof(double));
  s->hs = (double*)calloc(Qh * N, sizeof(double));
  s->phi = (double*)calloc(N, sizeof(double));
  s->phin = (double*)calloc(N, sizeof(double));
  s->c = (double*)calloc(N, sizeof(double));
  s->mu = (double*)calloc(N, sizeof(double));
  s->sbar = (double*)calloc(N, sizeof(double));
  s->grad = (double*)calloc(3 * N, sizeof(double));
  s->nrm = (double*)calloc(3 * N, sizeof(double));
  if (!s->g || !s->h || !s->gs || !s->hs || !s->phi || !s->phin || !s->c ||
      !s->mu || !s->sbar || !s->grad || !s->nrm) {
    orc_destroy(s);
    return NULL;
  }
  return s;
}

void orc_destroy(orc_state* s) {
  if (!s) return;
  free(s->g); free(s->h); free(s->gs); free(s->hs); free(s->phi);
  free(s->phin); free(s->c); free(s->mu); free(s->sbar); free(s->grad);
  free(s->nrm);
  free(s);
}

int orc_q(const orc_state* s) { return s->Q; }
int orc_qh(const orc_state* s) { return s->Qh; }
int64_t orc_nodes(const orc_state* s) { return s->N; }
int64_t orc_step_count(const orc_state* s) { return s->step; }

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Initialisation from phi0 and c0 (the reading of the paper's silence on the
 * initial populations is in the file header). */
int orc_init(orc_state* s, const double* phi0, const double* c0) {
  const orc_params* p = &s->p;
  const int nx = p->nx, ny = p->ny, nz = p->nz, Q = s->Q, Qh = s->Qh;
  const int64_t N = s->N;
  memcpy(s->phi, phi0, N * sizeof(double));
#pragma omp parallel for
  for (int64_t i = 0; i < N; ++i) {
    int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
    double g3[3], n3[3], G[19], sbar, F[3] = {0.0, 0.0, 0.0};
    double phi = phi0[i], c = c0[i];
    double mu = closure(p, c, phi);
    gradient_normal(s, phi0, x, y, z, g3, n3);
    phi_sources(s, phi, mu, n3, G, &sbar);
    for (int k = 0; k < Q; ++k) s->g[k * N + i] = s->w[k] * phi - 0.5 * G[k];
    for (int a = 0; a < s->D; ++a) F[a] = (mu * (p->D_l - p->D_s)) * g3[a];
    double lam = h_lambda(p, phi, mu);
    for (int k = 0; k < Qh; ++k) {
      if (p->h_scheme == ORC_H_EQ_ALT)
        s->h[k * N + i] = h_equilibrium_alt(s, k, c, lam, F);
      else
        s->h[k * N + i] = h_equilibrium(s, k, c, lam) - 0.5 * h_source(s, k, F);
    }
  }
  (void)ny; (void)nz;
  s->step = 0;
  s->ready = 1;
  return 0;
}

/* One time step n -> n+1 (S1..S9). */
static void step_once(orc_state* s) {
  const orc_params* p = &s->p;
  const int nx = p->nx, ny = p->ny, Q = s->Q, Qh = s->Qh, D = s->D;
  const int64_t N = s->N;
  const double omega_g = 1.0 / (s->inv_cs2g * p->M_phi + 0.5);
  const double omega_h = 1.0 / (1.0 / (p->gamma * s->cs2h) + 0.5);

  /* S1-S4: moments, closure, gradient, sources, collision of g. */
#pragma omp parallel for
  for (int64_t i = 0; i < N; ++i) {
    int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
    double c = 0.0;
    for (int k = 0; k < Qh; ++k) c = c + s->h[k * N + i];
    double phi = s->phi[i];
    double mu = closure(p, c, phi);
    double g3[3], n3[3], G[19], sbar;
    gradient_normal(s, s->phi, x, y, z, g3, n3);
    phi_sources(s, phi, mu, n3, G, &sbar);
    for (int k = 0; k < Q; ++k) {
      double gk = s->g[k * N + i];
      double t = (gk - s->w[k] * phi) + 0.5 * G[k];
      s->gs[k * N + i] = (gk - omega_g * t) + G[k];
    }
    s->c[i] = c;
    s->mu[i] = mu;
    s->sbar[i] = sbar;
    for (int a = 0; a < 3; ++a) {
      s->grad[3 * i + a] = g3[a];
      s->nrm[3 * i + a] = n3[a];
    }
  }
  /* S5: streaming of g into s->g (now g~^{n+1}). */
#pragma omp parallel for
  for (int64_t i = 0; i < N; ++i) {
    int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
    for (int k = 0; k < Q; ++k) {
      int64_t src;
      if (pull_source(s, s->e, x, y, z, k, &src))
        s->g[k * N + i] = s->gs[s->opp[k] * N + i];
      else
        s->g[k * N + i] = s->gs[k * N + src];
    }
  }
  /* S6: phi^{n+1}. */
#pragma omp parallel for
  for (int64_t i = 0; i < N; ++i) {
    double sum = 0.0;
    for (int k = 0; k < Q; ++k) sum = sum + s->g[k * N + i];
    s->phin[i] = sum + 0.5 * s->sbar[i];
  }
  /* S7-S8: anti-trapping current and collision of h. */
#pragma omp parallel for
  for (int64_t i = 0; i < N; ++i) {
    double phi = s->phi[i], mu = s->mu[i], c = s->c[i];
    double F[3] = {0.0, 0.0, 0.0};
    double dtphi = s->phin[i] - phi;
    double jump = at_jump(p, mu);
    for (int a = 0; a < D; ++a) {
      double j = 0.0;
      if (p->anti_trapping)
        j = (((p->a_at * p->W) * jump) * dtphi) * s->nrm[3 * i + a];
      F[a] = (mu * (p->D_l - p->D_s)) * s->grad[3 * i + a] + j;
    }
    double lam = h_lambda(p, phi, mu);
    for (int k = 0; k < Qh; ++k) {
      double hk = s->h[k * N + i];
      if (p->h_scheme == ORC_H_EQ_ALT) {
        /* Eq. (LBE_Concent_Alt): relaxation to h^eq,alt, no source */
        double t = hk - h_equilibrium_alt(s, k, c, lam, F);
        s->hs[k * N + i] = hk - omega_h * t;
      } else {
        double Hk = h_source(s, k, F);
        double t = (hk - h_equilibrium(s, k, c, lam)) + 0.5 * Hk;
        s->hs[k * N + i] = (hk - omega_h * t) + Hk;
      }
    }
  }
  /* S9: streaming of h. */
#pragma omp parallel for
  for (int64_t i = 0; i < N; ++i) {
    int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
    for (int k = 0; k < Qh; ++k) {
      int64_t src;
      if (pull_source(s, s->eh, x, y, z, k, &src))
        s->h[k * N + i] = s->hs[s->opph[k] * N + i];
      else
        s->h[k * N + i] = s->hs[k * N + src];
    }
  }
  double* t = s->phi; s->phi = s->phin; s->phin = t;
  s->step += 1;
}

int orc_step(orc_state* s, int64_t nsteps) {
  if (!s->ready) return -5;
  for (int64_t n = 0; n < nsteps; ++n) step_once(s);
  return 0;
}

/* phi^n, c^n and mu^n at the current time. */
void orc_fields(const orc_state* s, double* phi, double* c, double* mu) {
  const int64_t N = s->N;
  const int Q = s->Qh;
#pragma omp parallel for
  for (int64_t i = 0; i < N; ++i) {
    double cc = 0.0;
    for (int k = 0; k < Q; ++k) cc = cc + s->h[k * N + i];
    if (phi) phi[i] = s->phi[i];
    if (c) c[i] = cc;
    if (mu) mu[i] = closure(&s->p, cc, s->phi[i]);
  }
}

/* Gradient and normal of the current phi (stage S2), 3 values per node. */
void orc_gradient(const orc_state* s, double* grad3, double* nrm3) {
  const int nx = s->p.nx, ny = s->p.ny;
  const int64_t N = s->N;
#pragma omp parallel for
  for (int64_t i = 0; i < N; ++i) {
    int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
    double g3[3], n3[3];
    gradient_normal(s, s->phi, x, y, z, g3, n3);
    for (int a = 0; a < 3; ++a) {
      if (grad3) grad3[3 * i + a] = g3[a];
      if (nrm3) nrm3[3 * i + a] = n3[a];
    }
  }
}

void orc_get_state(const orc_state* s, double* g, double* h, double* phi) {
  const int64_t QN = (int64_t)s->Q * s->N, QhN = (int64_t)s->Qh * s->N;
  if (g) memcpy(g, s->g, QN * sizeof(double));
  if (h) memcpy(h, s->h, QhN * sizeof(double));
  if (phi) memcpy(phi, s->phi, s->N * sizeof(double));
}

void orc_set_state(orc_state* s, const double* g, const double* h,
                   const double* phi, int64_t step) {
  const int64_t QN = (int64_t)s->Q * s->N, QhN = (int64_t)s->Qh * s->N;
  memcpy(s->g, g, QN * sizeof(double));
  memcpy(s->h, h, QhN * sizeof(double));
  memcpy(s->phi, phi, s->N * sizeof(double));
  s->step = step;
  s->ready = 1;
}

/* Diagnostics at the current time, summed sequentially in node order:
 * out[0] total solute sum_x c, out[1] mean (1 - phi), out[2] fraction of
 * nodes with phi < 1/2, out[3] sum_x phi, out[4] min phi, out[5] max phi,
 * out[6] 1 if any phi or c is not finite, out[7] step. */
void orc_diagnostics(const orc_state* s, double* out) {
  const int64_t N = s->N;
  const int Q = s->Qh;
  double mass = 0.0, solid = 0.0, count = 0.0, sphi = 0.0;
  double mn = INFINITY, mx = -INFINITY;
  int bad = 0;
  for (int64_t i = 0; i < N; ++i) {
    double cc = 0.0;
    for (int k = 0; k < Q; ++k) cc = cc + s->h[k * N + i];
    double phi = s->phi[i];
    if (!isfinite(cc) || !isfinite(phi)) bad = 1;
    mass = mass + cc;
    solid = solid + (1.0 - phi);
    if (phi < 0.5) count = count + 1.0;
    sphi = sphi + phi;
    if (phi < mn) mn = phi;
    if (phi > mx) mx = phi;
  }
  out[0] = mass;
  out[1] = solid / (double)N;
  out[2] = count / (double)N;
  out[3] = sphi;
  out[4] = mn;
  out[5] = mx;
  out[6] = bad ? 1.0 : 0.0;
  out[7] = (double)s->step;
}

void orc_local(const orc_params* p, double phi, double c, double mu, double* out) {
  out[0] = closure(p, c, phi);
  out[1] = coupling_bracket(p, mu);
  out[2] = at_jump(p, mu);
}
