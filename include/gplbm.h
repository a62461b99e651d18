/*
 * gplbm — coupled phase-field / composition lattice-Boltzmann step of the
 * grand-potential model of dissolution and precipitation (Boutin, Verdier &
 * Cartalade, arXiv:2111.05960), on AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Plain pointers and sizes only.  Every device pointer is a HIP
 * device address on the device that was current when gplbm_create ran; the
 * stream argument is a hipStream_t passed as void*.
 *
 * What one step computes (lattice units dx = dt = 1; xi_s^2 = 1/3 on D2Q9,
 * D3Q19 and D2Q5, 1/4 on D3Q7):
 *   - phi-LBE, Sec. 3.2: BGK collision with trapezoidal source,
 *     Eq. (LBE_PhaseField_Eq), g^eq = w_k phi (Eq. Geq_Allen-Cahn_Eq-1),
 *     sources Eqs. (TermG), (SourceG_ST), (SourceG_dw) / (SourceG_CT) with
 *     S_phi of Eq. (SourceTerm_Coexistence), phi moment Eq. (Moment_Phi),
 *     gradient by directional derivatives Eqs. (DerivDirec_Grad), (Grad);
 *   - c-LBE, Sec. 3.3: Eqs. (LBE_Composition), (Heq_Composition),
 *     (SourceTerm_LBE_h), c moment Eq. (Moment0_LBM_Concent), closure
 *     Eqs. (PotChim_Equilibirum)-(Coexistence_Interpol), anti-trapping
 *     current Eq. (Anti-trapping_Equilibrium) with dphi/dt by explicit Euler
 *     (the c-LBE is solved after the phi-LBE).
 * Readings where the paper is silent (shared with the CPU reference):
 *   the phi moment uses the closed-form zeroth moment of this step's
 *   source at the same node (G^st, plus G^dw without the counter term); the
 *   normal is grad phi / sqrt(|grad phi|^2 + eps_n^2); walls are halfway
 *   bounce-back with a mirror ghost for the gradient; the initial
 *   populations are the equilibria shifted by the trapezoidal variable
 *   change, without anti-trapping current.
 *
 * Ownership.  The caller owns every device buffer and the stream.  The
 * library never allocates device memory: gplbm_state_bytes says how large a
 * device buffer gplbm_create must borrow for the whole state (populations,
 * phase field, reduction scratch).  The context (host memory) is owned by the
 * library until gplbm_destroy.  Calls on one context are not thread safe.
 *
 * Errors.  Every int-returning call returns GPLBM_OK (0) or a negative code;
 * gplbm_last_error gives the text of the last failure on a context.
 */
#ifndef GPLBM_H
#define GPLBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define GPLBM_OK 0
#define GPLBM_E_INVALID (-1)   /* bad parameter, null pointer, unsupported combination */
#define GPLBM_E_SIZE (-2)      /* borrowed buffer too small */
#define GPLBM_E_DEVICE (-3)    /* HIP runtime error (text in gplbm_last_error) */
#define GPLBM_E_NONFINITE (-4) /* diagnostics found a non-finite phi or c */
#define GPLBM_E_STATE (-5)     /* step / read before gplbm_init_fields */

/* lattices of g (phi).  D2Q5 / D3Q7 (Sec. 3.1 lists them among the usual
 * sets): tau_g = M_phi / xi_s^2 (4 M_phi on D3Q7) and the gradient of
 * Eqs. (DerivDirec_Grad), (Grad) with the factor 1 / xi_s^2, i.e. central
 * differences; h then runs on the same lattice.  Every precision, the
 * adjoint included. */
#define GPLBM_D2Q9 0
#define GPLBM_D3Q19 1
#define GPLBM_D2Q5 2
#define GPLBM_D3Q7 3

/* lattice of h under D2Q9 / D3Q19 (under D2Q5 / D3Q7, h always runs on the
 * lattice of g).  LIGHT: D2Q5 under D2Q9, D3Q7 under D3Q19 (Sec. 3.3 leaves
 * the lattice of the c-LBE open; its equilibrium needs only the zeroth and
 * an isotropic second moment).  The relaxation time becomes
 * tau_h = 1 / (gamma xi_s^2) (3 / gamma, or 4 / gamma on D3Q7) so that the
 * diffusivity stays D(phi); H_k = gamma w_k e_k . F on the h lattice.  Every
 * precision, the adjoint included. */
#define GPLBM_H_FULL 0
#define GPLBM_H_LIGHT 1

/* scheme of the c-LBE.  SOURCE: Eqs. (LBE_Composition), (Heq_Composition),
 * (SourceTerm_LBE_h).  EQ_ALT: Eqs. (LBE_Concent_Alt), (Seq_Concent_Alt), the
 * flux F = mu D' grad phi + j_at folded into the moving populations of the
 * equilibrium, w_k (gamma D mu + e_k . F / xi_s^2), no source; the initial
 * populations are that equilibrium (no variable-change shift).  Every
 * precision, the adjoint included. */
#define GPLBM_H_SOURCE 0
#define GPLBM_H_EQ_ALT 1

/* free energies of the two phases (parabolas, Sec. 2.3).  EQUAL: equal
 * curvatures, parameterised by c_s_co, c_l_co, mu_eq (closure
 * Eq. (PotChim_Equilibirum), source Eq. (SourceTerm_Equilibrium),
 * anti-trapping Eq. (Anti-trapping_Equilibrium)).  QUADRATIC: general
 * eps_s != eps_l, parameterised by eps_s, eps_l, m_s, m_l, df_min (closure
 * Eq. (Closure), source Eq. (SourceTerm), anti-trapping
 * Eq. (Anti-Trapping_Quadratic)), with the interpolations h(phi) = phi,
 * q(phi) and a of the equal case.  Every precision, the adjoint
 * included. */
#define GPLBM_FE_EQUAL 0
#define GPLBM_FE_QUADRATIC 1

/* boundary conditions per axis */
#define GPLBM_PERIODIC 0
#define GPLBM_ZERO_FLUX 1 /* halfway bounce-back, walls at -1/2 and n-1/2 */

/* storage / arithmetic precision of the populations and of phi */
#define GPLBM_FP64 0 /* everything in double */
#define GPLBM_FP32 1 /* float storage and collision; moments and closure in double */
/* any lattice combination, either h scheme, either free-energy form: the
 * Q - 1 (Qh - 1) moving populations of g (h) stored as 16-bit deviations
 * from the writing node's equilibrium (w_k phi for g, w_k gamma D(phi) mu for
 * h), rest populations, phi and gamma D(phi) mu as float; float collision,
 * double moments and closure; solute mass balanced through the rest
 * population.  FP16 deviations are scaled by 2^12, BF16 ones are not. */
#define GPLBM_FP16_DEV 2
#define GPLBM_BF16_DEV 3

/* kernel schedule */
#define GPLBM_SCHED_AUTO 0  /* fused when the geometry allows it, else split */
#define GPLBM_SCHED_SPLIT 1 /* two kernels per step */
#define GPLBM_SCHED_FUSED 2 /* one kernel per step (tile halo recompute) */

typedef struct gplbm_params {
  int32_t lattice;       /* GPLBM_D2Q9, GPLBM_D3Q19, GPLBM_D2Q5 or GPLBM_D3Q7 (g) */
  int32_t nx, ny, nz;    /* nodes; nz = 1 in 2-D; node i = x + nx*(y + ny*z) */
  int32_t bc[3];         /* per axis x, y, z: GPLBM_PERIODIC or GPLBM_ZERO_FLUX */
  int32_t precision;     /* GPLBM_FP64, GPLBM_FP32, GPLBM_FP16_DEV or GPLBM_BF16_DEV */
  int32_t counter_term;  /* 1: counter term G^ct_k (Eq. ModelA_EqPhi_CounterTerm); 0: G^dw */
  int32_t anti_trapping; /* 1: anti-trapping current in the h source */
  int32_t schedule;      /* GPLBM_SCHED_* */
  int32_t h_lattice;     /* GPLBM_H_FULL or GPLBM_H_LIGHT */
  int32_t h_scheme;      /* GPLBM_H_SOURCE or GPLBM_H_EQ_ALT */
  int32_t free_energy;   /* GPLBM_FE_EQUAL or GPLBM_FE_QUADRATIC */
  double W;              /* interface width */
  double M_phi;          /* phase-field mobility; tau_g = M_phi / xi_s^2 */
  double lambda;         /* coupling constant */
  double D_l, D_s;       /* diffusivities of liquid and solid */
  double gamma;          /* relaxation control of the c-LBE; tau_h = 1 / (gamma xi_s^2) */
  double a_at;           /* anti-trapping coefficient a (1/4 for D_s = 0) */
  double c_s_co, c_l_co; /* coexistence compositions */
  double mu_eq;          /* equilibrium chemical potential */
  double eps_n;          /* regularisation of the normal */
  /* GPLBM_FE_QUADRATIC only: curvatures eps_s, eps_l > 0 (only their ratio
   * enters), compositions m_s, m_l at the minima, reduced df_min = f_s^min -
   * f_l^min; c_s_co, c_l_co, mu_eq are then unused */
  double eps_s, eps_l, m_s, m_l, df_min;
} gplbm_params;

typedef struct gplbm_diag {
  int64_t step;                /* time level n of the fields described */
  double total_mass;           /* sum over nodes of c^n */
  double solid_fraction;       /* mean of 1 - phi^n */
  double solid_fraction_count; /* fraction of nodes with phi^n < 1/2 */
  double sum_phi;              /* sum over nodes of phi^n */
  double phi_min, phi_max;
  int32_t nonfinite;           /* 1 if some phi^n or c^n is not finite */
  int32_t reserved;
} gplbm_diag;

typedef struct gplbm_ctx gplbm_ctx;

/* Bytes of device memory gplbm_create must borrow for these parameters.
 * Returns GPLBM_E_INVALID for parameters gplbm_create would reject. */
int gplbm_state_bytes(const gplbm_params* p, uint64_t* bytes);

/* Bytes of one saved state (gplbm_save_state / gplbm_load_state). */
int gplbm_checkpoint_bytes(const gplbm_params* p, uint64_t* bytes);

/* Create a context on the current device.  dev_buf (device, >= bytes from
 * gplbm_state_bytes, 256-byte aligned) is borrowed until gplbm_destroy.
 * stream: hipStream_t (as void*), may be NULL for the null stream.
 * Rejects M_phi <= 0, gamma <= 0, W <= 0, sizes < 1, nz != 1 for D2Q9. */
int gplbm_create(const gplbm_params* p, void* dev_buf, uint64_t bytes, void* stream,
                 gplbm_ctx** out);

/* Change the stream later calls are ordered on. */
int gplbm_set_stream(gplbm_ctx* ctx, void* stream);

/* Initial condition (time 0) from phi0 and c0: device pointers to N doubles
 * each (N = nx*ny*nz, x fastest).  Asynchronous on the context's stream. */
int gplbm_init_fields(gplbm_ctx* ctx, const double* phi0, const double* c0);

/* Advance nsteps >= 0 time steps.  Asynchronous on the context's stream. */
int gplbm_step(gplbm_ctx* ctx, int64_t nsteps);

/* One step from a saved state to another (both in the gplbm_save_state
 * format, device, distinct); the context's own state and step count are left
 * unchanged.  Lets a checkpointing driver rebuild a segment of states without
 * copies.  Asynchronous on the context's stream. */
int gplbm_step_to(gplbm_ctx* ctx, const void* src_state, void* dst_state);

/* A segment of steps between saved states: states j = 0 .. n lie at
 * states + j * stride bytes (device; states 256-byte aligned, stride a
 * multiple of 256 and at least gplbm_checkpoint_bytes); state 0 is given, and the call computes state j+1
 * from state j for j < n, as n calls of gplbm_step_to would (a checkpointing
 * driver rebuilds a segment from its checkpoint with one call).  The
 * context's own state is left unchanged.  Asynchronous on the context's
 * stream; GPLBM_E_INVALID for a null pointer, n < 0 or a stride that is too
 * small or misaligned. */
int gplbm_step_chain(gplbm_ctx* ctx, void* states, uint64_t stride, int64_t n);

/* Current time level n. */
int64_t gplbm_step_count(const gplbm_ctx* ctx);

/* phi^n, c^n and mu^n as doubles into device arrays of N entries each; a
 * NULL pointer skips that field.  Asynchronous on the context's stream. */
int gplbm_read_fields(gplbm_ctx* ctx, double* phi, double* c, double* mu);

/* FP64 diagnostics of the current time level into host memory.  Reduced on
 * the device in a fixed order (deterministic); synchronises the stream.
 * Returns GPLBM_E_NONFINITE (with *out filled) if some phi or c is not
 * finite. */
int gplbm_diagnostics(gplbm_ctx* ctx, gplbm_diag* out);

/* For callers that cannot allocate device memory at all (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * diagnostics, bit-identical to gplbm_diagnostics, with the reduction
 * partials in a static device array of the library instead of the context's
 * buffer.  That array holds 8 * 1024 + 8 doubles (65.6 KB) per device, taken
 * when the first context is created on the device and kept until the process
 * ends; its size does not depend on the grid (the reduction grid is fixed),
 * so every grid gplbm_create accepts fits and larger ones are rejected with
 * GPLBM_E_SIZE.  Calls no allocating routine.  All calls on one device share
 * the array: calls that overlap on one device (other threads, other streams)
 * race and must be serialised by the caller.  Synchronises the stream;
 * GPLBM_E_DEVICE if the array's device address could not be taken. */
int gplbm_diagnostics_noalloc(gplbm_ctx* ctx, gplbm_diag* out);

/* Copy the complete state (gplbm_checkpoint_bytes bytes) to / from device
 * memory; together with the step count it determines every later step
 * exactly.  Asynchronous on the context's stream. */
int gplbm_save_state(gplbm_ctx* ctx, void* dev_dst);
int gplbm_load_state(gplbm_ctx* ctx, const void* dev_src, int64_t step);

/* Adjoint (reverse mode) of gplbm_init_fields followed by K steps, for every
 * context: gradients of a scalar objective J(phi^K, c^K) with
 * respect to phi0, c0, lambda and D_l (gamma, M_phi, W and a_at held fixed;
 * D' = D_l - D_s and D(phi) follow D_l).  It differentiates the discrete map
 * of the step in FP64 arithmetic (every operation of the collisions,
 * sources, closure, normal, anti-trapping current, streaming and boundaries)
 * at the forward values recomputed from saved states; for an FP64 context
 * that is exactly the map gplbm_step computes, for an FP32 context the same
 * map taken at the FP32 states, for an FP16/BF16-deviation context the same
 * map taken at the decoded states (the reverse sweep and all accumulations
 * are FP64 in all).  The caller drives the reverse sweep (e.g. with sqrt(K)
 * checkpointing of gplbm_save_state snapshots).
 *
 * gplbm_adjoint_bytes: size of the FP64 device workspace (adjoint state,
 *   intermediates, per-node parameter accumulators).
 * gplbm_adjoint_begin: borrow the workspace (256-byte aligned) and seed the
 *   adjoint of the state at time K from dJ/dphi^K and dJ/dc^K (device arrays of
 *   N doubles; NULL means zero).  Zeroes the parameter accumulators.
 * gplbm_adjoint_step: one reverse step from time n+1 to n; state_n and
 *   state_np1 are the forward states at n and n+1 in the gplbm_save_state
 *   format (device).  Asynchronous.
 * gplbm_adjoint_finish: reverse of gplbm_init_fields at (phi0, c0) (device):
 *   writes dJ/dphi0 and dJ/dc0 (device, N doubles) and dJ/dlambda, dJ/dD_l into
 *   dJ_dparams (host, 2 doubles).  Parameter sums are reduced in a fixed
 *   order.  Synchronises the stream.
 * Every lattice combination, both h schemes, both free-energy forms (the
 * quadratic constants eps_s, eps_l, m_s, m_l, df_min held fixed) and the
 * deviation formats are supported.  Return GPLBM_E_INVALID for invalid
 * parameters or null pointers, GPLBM_E_SIZE for a short workspace,
 * GPLBM_E_STATE out of order. */
int gplbm_adjoint_bytes(const gplbm_params* p, uint64_t* bytes);
int gplbm_adjoint_begin(gplbm_ctx* ctx, void* work, uint64_t bytes, const double* phi_bar,
                        const double* c_bar);
int gplbm_adjoint_step(gplbm_ctx* ctx, const void* state_n, const void* state_np1);
/* gplbm_adjoint_segment: the reverse steps over a segment of forward states
 *   laid out as in gplbm_step_chain (states j = 0 .. n at states + j * stride):
 *   gplbm_adjoint_step(state j, state j+1) for j = n-1 down to 0, in one call.
 *   Asynchronous; GPLBM_E_INVALID for a null pointer, n < 0 or a bad stride,
 *   GPLBM_E_STATE before gplbm_adjoint_begin. */
int gplbm_adjoint_segment(gplbm_ctx* ctx, const void* states, uint64_t stride, int64_t n);
int gplbm_adjoint_finish(gplbm_ctx* ctx, const double* phi0, const double* c0, double* phi0_bar,
                         double* c0_bar, double* dJ_dparams);

/* Bandwidth reference of the device (not part of the method): copies bytes
 * (a multiple of 16, at most 2^31 - 1 blocks of 4 KiB) from src to dst
 * (device, 16-byte aligned, not overlapping), one 16-byte vector per thread
 * with non-temporal stores, asynchronously on stream.  Its rate is the
 * practical ceiling of a kernel that reads and writes the same amount, which
 * the step does.  GPLBM_E_INVALID for null or misaligned pointers or a size
 * that is not a multiple of 16. */
int gplbm_stream_copy(const void* src, void* dst, uint64_t bytes, void* stream);

/* Which schedule the context runs (GPLBM_SCHED_SPLIT or GPLBM_SCHED_FUSED). */
int gplbm_schedule(const gplbm_ctx* ctx);

const char* gplbm_last_error(const gplbm_ctx* ctx);
void gplbm_destroy(gplbm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
