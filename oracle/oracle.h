/*
 * C interface of the FP64 CPU oracle (test infrastructure only; see
 * oracle.c for what it computes and the readings of the paper it applies).
 * Host pointers only.  Arrays are structure-of-arrays f[k][z][y][x],
 * x fastest; node index i = x + nx*(y + ny*z).
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_D2Q9 = 0, ORC_D3Q19 = 1, ORC_D2Q5 = 2, ORC_D3Q7 = 3 }; /* lattice of g */
enum { ORC_PERIODIC = 0, ORC_ZERO_FLUX = 1 };
enum { ORC_H_SOURCE = 0, ORC_H_EQ_ALT = 1 };        /* h_scheme */
enum { ORC_FE_EQUAL = 0, ORC_FE_QUADRATIC = 1 };    /* free_energy */

typedef struct {
  int32_t lattice;
  int32_t nx, ny, nz;
  int32_t bc[3];
  int32_t counter_term;  /* 1: counter term G^ct_k, 0: double-well term G^dw */
  int32_t anti_trapping; /* 1: anti-trapping current in the h source */
  int32_t h_lattice;     /* 0: h on the lattice of g; 1: h on D2Q5 / D3Q7 (g on
                            D2Q5 / D3Q7 always takes h on the same lattice) */
  int32_t h_scheme;      /* ORC_H_SOURCE: source H_k; ORC_H_EQ_ALT: h^eq,alt, H = 0 */
  int32_t free_energy;   /* ORC_FE_EQUAL: eps_s = eps_l (c_s_co, c_l_co, mu_eq);
                            ORC_FE_QUADRATIC: general (eps_s, eps_l, m_s, m_l, df_min) */
  double W, M_phi, lambda, D_l, D_s, gamma, a_at;
  double c_s_co, c_l_co, mu_eq, eps_n;
  double eps_s, eps_l, m_s, m_l, df_min;
} orc_params;

typedef struct orc_state orc_state;

orc_state* orc_create(const orc_params* p);
void orc_destroy(orc_state* s);
int orc_q(const orc_state* s);  /* populations of g */
int orc_qh(const orc_state* s); /* populations of h */
int64_t orc_nodes(const orc_state* s);
int64_t orc_step_count(const orc_state* s);
int orc_threads(void);
int orc_init(orc_state* s, const double* phi0, const double* c0);
int orc_step(orc_state* s, int64_t nsteps);
void orc_fields(const orc_state* s, double* phi, double* c, double* mu);
void orc_gradient(const orc_state* s, double* grad3, double* nrm3);
void orc_get_state(const orc_state* s, double* g, double* h, double* phi);
void orc_set_state(orc_state* s, const double* g, const double* h,
                   const double* phi, int64_t step);
void orc_diagnostics(const orc_state* s, double* out8);
/* The local forms at one point, for pins: out[0] = closure mu(c, phi),
 * out[1] = bracket of S_phi at mu, out[2] = composition jump of j_at at mu. */
void orc_local(const orc_params* p, double phi, double c, double mu, double* out3);

#ifdef __cplusplus
}
#endif
#endif
