// C ABI of the coupled phi / c lattice-Boltzmann library (declarations and
// contract in include/gplbm.h).
//
// Host side: validation, the carving of the borrowed device buffer, the
// per-run constants, and the dispatch of the kernels over the lattices of g
// and h and the precision.  No device allocation happens here.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>

#include "gplbm.h"
#include "kernels_adjoint.h"
#include "kernels_dev.h"
#include "kernels_fused2d.h"
#include "kernels_fused3d.h"
#include "kernels_split.h"
#include "stream_copy.h"

using namespace gplbm;

struct gplbm_ctx {
  gplbm_params p;
  int Q;             // populations of g
  int Qh;            // populations of h
  int64_t N;
  size_t elem;        // bytes per stored phi value
  size_t pop_bytes;   // the g distribution (rounded up)
  size_t hpop_bytes;  // the h distribution (rounded up)
  size_t mov_bytes;   // deviation formats: the 16-bit moving part of the g distribution
  size_t hmov_bytes;  // and of the h distribution
  size_t phi_bytes;   // N*elem rounded up
  size_t lam_bytes;   // deviation formats: the Lambda field
  char* G[2];
  char* H[2];
  char* PHI[2];
  char* LAM[2];
  double* red;        // reduction scratch: kDiagBlocks*kDiagVals + kDiagVals
  int cur;
  int64_t step;
  bool ready;
  int sched;
  hipStream_t stream;
  int device;
  std::string err;
  // adjoint (every context; FP64 reverse sweep)
  AdjWork adj;
  int adj_cur;
  bool adj_ready;
};

namespace {

constexpr size_t kAlign = 256;

size_t round_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int lattice_q(int lattice) {
  switch (lattice) {
    case GPLBM_D2Q9: return D2Q9::Q;
    case GPLBM_D3Q19: return D3Q19::Q;
    case GPLBM_D2Q5: return D2Q5::Q;
    default: return D3Q7::Q;
  }
}

bool two_d(int lattice) { return lattice == GPLBM_D2Q9 || lattice == GPLBM_D2Q5; }
bool light_g(int lattice) { return lattice == GPLBM_D2Q5 || lattice == GPLBM_D3Q7; }

// h on the light lattice: asked for under D2Q9 / D3Q19, always under D2Q5 / D3Q7
bool light_h(const gplbm_params& p) { return p.h_lattice == GPLBM_H_LIGHT || light_g(p.lattice); }

int lattice_qh(const gplbm_params* p) {
  if (light_h(*p)) return two_d(p->lattice) ? D2Q5::Q : D3Q7::Q;
  return lattice_q(p->lattice);
}

// xi_s^2 of the h lattice
double lattice_cs2h(const gplbm_params& p) {
  if (light_h(p)) return two_d(p.lattice) ? D2Q5::cs2 : D3Q7::cs2;
  return p.lattice == GPLBM_D2Q9 ? D2Q9::cs2 : D3Q19::cs2;
}

// 1 / xi_s^2 of the g lattice, written exactly
double lattice_inv_cs2g(int lattice) { return lattice == GPLBM_D3Q7 ? D3Q7::inv_cs2 : D3Q19::inv_cs2; }

// Returns an error text, or nullptr when the parameters are acceptable.
const char* check_params(const gplbm_params* p) {
  if (!p) return "null parameters";
  if (p->lattice < GPLBM_D2Q9 || p->lattice > GPLBM_D3Q7) return "unknown lattice";
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return "grid sizes must be >= 1";
  if (two_d(p->lattice) && p->nz != 1) return "2-D lattices need nz == 1";
  for (int a = 0; a < 3; ++a)
    if (p->bc[a] != GPLBM_PERIODIC && p->bc[a] != GPLBM_ZERO_FLUX) return "unknown boundary";
  if (p->precision < GPLBM_FP64 || p->precision > GPLBM_BF16_DEV) return "unknown precision";
  if (p->schedule < GPLBM_SCHED_AUTO || p->schedule > GPLBM_SCHED_FUSED) return "unknown schedule";
  if (p->h_lattice != GPLBM_H_FULL && p->h_lattice != GPLBM_H_LIGHT) return "unknown h lattice";
  if (p->h_scheme != GPLBM_H_SOURCE && p->h_scheme != GPLBM_H_EQ_ALT) return "unknown h scheme";
  if (p->free_energy != GPLBM_FE_EQUAL && p->free_energy != GPLBM_FE_QUADRATIC)
    return "unknown free energy";
  if (p->free_energy == GPLBM_FE_QUADRATIC) {
    if (!(p->eps_s > 0.0) || !(p->eps_l > 0.0) || !std::isfinite(p->eps_s) || !std::isfinite(p->eps_l))
      return "eps_s and eps_l must be > 0";
    if (!std::isfinite(p->m_s) || !std::isfinite(p->m_l) || !std::isfinite(p->df_min))
      return "non-finite parameter";
  }
  if (!(p->W > 0.0) || !std::isfinite(p->W)) return "W must be > 0";
  if (!(p->M_phi > 0.0) || !std::isfinite(p->M_phi)) return "M_phi must be > 0 (omega_g in (0,2))";
  if (!(p->gamma > 0.0) || !std::isfinite(p->gamma)) return "gamma must be > 0 (omega_h in (0,2))";
  const double vals[] = {p->lambda, p->D_l, p->D_s, p->a_at, p->c_s_co, p->c_l_co, p->mu_eq, p->eps_n};
  for (double v : vals)
    if (!std::isfinite(v)) return "non-finite parameter";
  const int64_t N = (int64_t)p->nx * p->ny * p->nz;
  if (N > (int64_t)1 << 40) return "grid too large";
  return nullptr;
}

// Borrowed buffer: G[0], G[1], H[0], H[1], PHI[0], PHI[1], LAM[0], LAM[1],
// reduction scratch.  A saved state: G, H, PHI, LAM.
struct Layout {
  size_t elem, pop, hpop, mov, hmov, phi, lam, red, total, ckpt;
};

Layout layout(const gplbm_params* p) {
  Layout l{};
  const int64_t N = (int64_t)p->nx * p->ny * p->nz;
  const int Q = lattice_q(p->lattice);
  if (p->precision >= GPLBM_FP16_DEV) {
    l.elem = 4;
    l.mov = round_up((size_t)(Q - 1) * N * 2);
    l.pop = l.mov + round_up((size_t)N * 4);
    l.hmov = round_up((size_t)(lattice_qh(p) - 1) * N * 2);
    l.hpop = l.hmov + round_up((size_t)N * 4);
    l.lam = round_up((size_t)N * 4);
  } else {
    l.elem = p->precision == GPLBM_FP64 ? 8 : 4;
    l.mov = 0;
    l.hmov = 0;
    l.pop = round_up((size_t)Q * N * l.elem);
    l.hpop = round_up((size_t)lattice_qh(p) * N * l.elem);
    l.lam = 0;
  }
  l.phi = round_up((size_t)N * l.elem);
  l.red = round_up(sizeof(double) * (kDiagBlocks * kDiagVals + kDiagVals));
  l.total = 2 * l.pop + 2 * l.hpop + 2 * l.phi + 2 * l.lam + l.red;
  l.ckpt = l.pop + l.hpop + l.phi + l.lam;
  return l;
}

int fail(gplbm_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

int check_launch(gplbm_ctx* ctx, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return fail(ctx, GPLBM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return GPLBM_OK;
}

ClosureK closure_k(const gplbm_params& p) {
  ClosureK q{};
  q.quad = p.free_energy == GPLBM_FE_QUADRATIC ? 1 : 0;
  q.cl = p.c_l_co;
  q.cs = p.c_s_co;
  q.mueq = p.mu_eq;
  if (q.quad) {
    q.efac = std::sqrt(p.eps_s * p.eps_l);
    q.eps_s = p.eps_s;
    q.eps_l = p.eps_l;
    q.m_s = p.m_s;
    q.m_l = p.m_l;
  }
  return q;
}

template <class C>
Coef<C> make_coef(const gplbm_params& p) {
  Coef<C> K{};
  const double dc = p.c_s_co - p.c_l_co;
  // tau_g = M_phi / xi_s^2 (3 M_phi, or 4 M_phi on D3Q7)
  K.omega_g_d = 1.0 / (lattice_inv_cs2g(p.lattice) * p.M_phi + 0.5);
  K.omega_g = C(K.omega_g_d);
  // tau_h = 1 / (gamma xi_s^2): the diffusivity of the c-LBE is D(phi) on
  // every h lattice
  K.omega_h = C(1.0 / (1.0 / (p.gamma * lattice_cs2h(p)) + 0.5));
  K.dc = C(dc);
  K.kst = C(-((p.lambda * p.M_phi) / (p.W * p.W)));
  K.k4w = C(4.0 / p.W);
  K.kdw = C(-((8.0 * p.M_phi) / (p.W * p.W)));
  K.jfac = C((p.a_at * p.W) * dc);
  K.Dp = C(p.D_l - p.D_s);
  K.Dl = C(p.D_l);
  K.Ds = C(p.D_s);
  K.gamma = C(p.gamma);
  K.eps2 = C(p.eps_n * p.eps_n);
  K.mueq_c = C(p.mu_eq);
  K.counter_term = p.counter_term ? 1 : 0;
  K.anti_trapping = p.anti_trapping ? 1 : 0;
  K.h_alt = p.h_scheme == GPLBM_H_EQ_ALT ? 1 : 0;
  K.fe_quad = p.free_energy == GPLBM_FE_QUADRATIC ? 1 : 0;
  K.q = closure_k(p);
  if (K.fe_quad) {
    K.k2 = C((p.eps_l - p.eps_s) / std::sqrt(p.eps_l * p.eps_s));
    K.dml = C(p.m_l - p.m_s);
    K.dfm = C(p.df_min);
    K.ks = C(-((p.eps_s - p.eps_l) / std::sqrt(p.eps_s * p.eps_l)));
    K.ms = C(p.m_s);
    K.ml = C(p.m_l);
    K.aW = C(p.a_at * p.W);
  }
  return K;
}

Geo make_geo(const gplbm_params& p) {
  Geo g;
  g.nx = p.nx;
  g.ny = p.ny;
  g.nz = p.nz;
  g.bcx = p.bc[0];
  g.bcy = p.bc[1];
  g.bcz = two_d(p.lattice) ? GPLBM_PERIODIC : p.bc[2];
  g.N = (int64_t)p.nx * p.ny * p.nz;
  return g;
}

// Typed operations for the lattices L (g) and LH (h) and the storage /
// arithmetic types S, C.
template <class L, class LH, class S, class C>
struct Ops {
  static dim3 block() { return dim3(64, 4, 1); }
  static dim3 grid(const gplbm_ctx* ctx) {
    return dim3((ctx->p.nx + 63) / 64, (ctx->p.ny + 3) / 4, ctx->p.nz);
  }
  static Coef<C> coef(const gplbm_ctx* ctx) { return make_coef<C>(ctx->p); }
  // the alternative h scheme or the general free energies
  static bool general(const gplbm_ctx* ctx) {
    return ctx->p.h_scheme != GPLBM_H_SOURCE || ctx->p.free_energy != GPLBM_FE_EQUAL;
  }

  static int init(gplbm_ctx* ctx, const double* phi0, const double* c0) {
    const Geo g = make_geo(ctx->p);
    const int a = ctx->cur;
    hipLaunchKernelGGL((k_init<L, LH, S, C>), grid(ctx), block(), 0, ctx->stream, g, coef(ctx), phi0,
                       c0, (S*)ctx->G[a], (S*)ctx->H[a], (S*)ctx->PHI[a]);
    return check_launch(ctx, "init");
  }

  static int step_split(gplbm_ctx* ctx, int64_t nsteps) {
    const Geo g = make_geo(ctx->p);
    const Coef<C> K = coef(ctx);
    for (int64_t s = 0; s < nsteps; ++s) {
      const int a = ctx->cur, b = 1 - a;
      StepBufs<S> bufs{(const S*)ctx->G[a], (const S*)ctx->H[a], (const S*)ctx->PHI[a],
                       (S*)ctx->H[b],       (S*)ctx->PHI[b],       (S*)ctx->G[b]};
      if (general(ctx)) {
        hipLaunchKernelGGL((k_split_h<L, LH, S, C, true>), grid(ctx), block(), 0, ctx->stream, g, K,
                           bufs);
        hipLaunchKernelGGL((k_split_g<L, LH, S, C, true>), grid(ctx), block(), 0, ctx->stream, g, K,
                           bufs);
      } else {
        hipLaunchKernelGGL((k_split_h<L, LH, S, C, false>), grid(ctx), block(), 0, ctx->stream, g,
                           K, bufs);
        hipLaunchKernelGGL((k_split_g<L, LH, S, C, false>), grid(ctx), block(), 0, ctx->stream, g,
                           K, bufs);
      }
      int rc = check_launch(ctx, "split step");
      if (rc) return rc;
      ctx->cur = b;
      ctx->step += 1;
    }
    return GPLBM_OK;
  }

  static int step_fused(gplbm_ctx* ctx, int64_t nsteps) {
    const Geo g = make_geo(ctx->p);
    const Coef<C> K = coef(ctx);
    for (int64_t s = 0; s < nsteps; ++s) {
      const int a = ctx->cur, b = 1 - a;
      StepBufs<S> bufs{(const S*)ctx->G[a], (const S*)ctx->H[a], (const S*)ctx->PHI[a],
                       (S*)ctx->H[b],       (S*)ctx->PHI[b],       (S*)ctx->G[b]};
      int rc = general(ctx) ? FusedLaunch<L, LH, S, C, true>::launch(g, K, bufs, ctx->stream)
                            : FusedLaunch<L, LH, S, C, false>::launch(g, K, bufs, ctx->stream);
      if (rc) return fail(ctx, GPLBM_E_DEVICE, "fused step launch failed");
      rc = check_launch(ctx, "fused step");
      if (rc) return rc;
      ctx->cur = b;
      ctx->step += 1;
    }
    return GPLBM_OK;
  }

  static int fields(gplbm_ctx* ctx, double* phi, double* c, double* mu) {
    const Geo g = make_geo(ctx->p);
    const int a = ctx->cur;
    hipLaunchKernelGGL((k_fields<LH, S>), grid(ctx), block(), 0, ctx->stream, g,
                       closure_k(ctx->p), (const S*)ctx->H[a], (const S*)ctx->PHI[a], phi, c, mu);
    return check_launch(ctx, "read fields");
  }

  static int diag(gplbm_ctx* ctx, double* red) {
    const Geo g = make_geo(ctx->p);
    const int a = ctx->cur;
    double* part = red;
    double* out = red + kDiagBlocks * kDiagVals;
    hipLaunchKernelGGL((k_diag_partial<LH, S>), dim3(kDiagBlocks), dim3(kDiagThreads), 0,
                       ctx->stream, g, (const S*)ctx->H[a], (const S*)ctx->PHI[a], part);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kDiagThreads), 0, ctx->stream,
                       (const double*)part, kDiagBlocks, out);
    return check_launch(ctx, "diagnostics");
  }
};

// Operations in the deviation storage formats (every lattice combination;
// the fused schedules are the 3-D z-march and the 2-D tile kernel).
template <class Codec, class L, class LH>
struct DevOps {
  static dim3 block() { return dim3(64, 4, 1); }
  static dim3 grid(const gplbm_ctx* ctx) {
    return dim3((ctx->p.nx + 63) / 64, (ctx->p.ny + 3) / 4, ctx->p.nz);
  }
  static DevState state(const gplbm_ctx* ctx, int a) {
    DevState s;
    s.G.mov = (uint16_t*)ctx->G[a];
    s.G.rest = (float*)(ctx->G[a] + ctx->mov_bytes);
    s.H.mov = (uint16_t*)ctx->H[a];
    s.H.rest = (float*)(ctx->H[a] + ctx->hmov_bytes);
    s.PHI = (float*)ctx->PHI[a];
    s.LAM = (float*)ctx->LAM[a];
    return s;
  }
  static int init(gplbm_ctx* ctx, const double* phi0, const double* c0) {
    const Geo g = make_geo(ctx->p);
    const Coef<float> K = make_coef<float>(ctx->p);
    const DevState s = state(ctx, ctx->cur);
    hipLaunchKernelGGL(k_dev_init_fields, grid(ctx), block(), 0, ctx->stream, g, K, phi0, c0, s);
    hipLaunchKernelGGL((k_dev_init<Codec, L, LH>), grid(ctx), block(), 0, ctx->stream, g, K, c0, s);
    return check_launch(ctx, "init");
  }
  static int step(gplbm_ctx* ctx, int64_t nsteps) {
    const Geo g = make_geo(ctx->p);
    const Coef<float> K = make_coef<float>(ctx->p);
    for (int64_t n = 0; n < nsteps; ++n) {
      const int a = ctx->cur, b = 1 - a;
      const DevStep st{state(ctx, a), state(ctx, b)};
      if (ctx->sched == GPLBM_SCHED_FUSED) {
        // the general instantiation only for h^eq,alt or eps_s != eps_l
        const bool gen = ctx->p.h_scheme != GPLBM_H_SOURCE || ctx->p.free_energy != GPLBM_FE_EQUAL;
        int rc;
        if constexpr (L::D == 3)
          rc = gen ? DevFused3D<Codec, L, LH, true>::launch(g, K, st, ctx->stream)
                   : DevFused3D<Codec, L, LH, false>::launch(g, K, st, ctx->stream);
        else
          rc = gen ? DevFused2D<Codec, L, LH, true>::launch(g, K, st, ctx->stream)
                   : DevFused2D<Codec, L, LH, false>::launch(g, K, st, ctx->stream);
        if (rc) return fail(ctx, GPLBM_E_DEVICE, "fused step launch failed");
      } else {
        hipLaunchKernelGGL((k_dev_split_h<Codec, L, LH>), grid(ctx), block(), 0, ctx->stream, g, K, st);
        hipLaunchKernelGGL((k_dev_split_g<Codec, L, LH>), grid(ctx), block(), 0, ctx->stream, g, K, st);
      }
      int rc = check_launch(ctx, "step");
      if (rc) return rc;
      ctx->cur = b;
      ctx->step += 1;
    }
    return GPLBM_OK;
  }
  static int fields(gplbm_ctx* ctx, double* phi, double* c, double* mu) {
    const Geo g = make_geo(ctx->p);
    hipLaunchKernelGGL((k_dev_fields<Codec, LH>), grid(ctx), block(), 0, ctx->stream, g,
                       closure_k(ctx->p), state(ctx, ctx->cur), phi, c, mu);
    return check_launch(ctx, "read fields");
  }
  static int diag(gplbm_ctx* ctx, double* red) {
    const Geo g = make_geo(ctx->p);
    double* part = red;
    double* out = red + kDiagBlocks * kDiagVals;
    hipLaunchKernelGGL((k_dev_diag_partial<Codec, LH>), dim3(kDiagBlocks), dim3(kDiagThreads), 0,
                       ctx->stream, g, state(ctx, ctx->cur), part);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kDiagThreads), 0, ctx->stream,
                       (const double*)part, kDiagBlocks, out);
    return check_launch(ctx, "diagnostics");
  }
};

template <class Codec, class L, class LH>
struct DevAdapter {
  using Ops = DevOps<Codec, L, LH>;
  static int init(gplbm_ctx* c, const double* a, const double* b) { return Ops::init(c, a, b); }
  static int step(gplbm_ctx* c, int64_t n) { return Ops::step(c, n); }
  static int fields(gplbm_ctx* c, double* a, double* b, double* d) { return Ops::fields(c, a, b, d); }
  static int diag(gplbm_ctx* c, double* r) { return Ops::diag(c, r); }
};

template <template <class, class, class, class> class Fn, class L, class LH, class... Args>
int dispatch_prec(gplbm_ctx* ctx, Args... args) {
  if (ctx->p.precision == GPLBM_FP64) return Fn<L, LH, double, double>::run(ctx, args...);
  return Fn<L, LH, float, float>::run(ctx, args...);
}

// deviation formats: the lattice combinations of the other precisions
template <template <class, class, class, class> class Fn, class Codec, class... Args>
int dispatch_dev(gplbm_ctx* ctx, Args... args) {
  const bool light = ctx->p.h_lattice == GPLBM_H_LIGHT;
  switch (ctx->p.lattice) {
    case GPLBM_D2Q9:
      return light ? Fn<DevAdapter<Codec, D2Q9, D2Q5>, void, void, void>::run(ctx, args...)
                   : Fn<DevAdapter<Codec, D2Q9, D2Q9>, void, void, void>::run(ctx, args...);
    case GPLBM_D3Q19:
      return light ? Fn<DevAdapter<Codec, D3Q19, D3Q7>, void, void, void>::run(ctx, args...)
                   : Fn<DevAdapter<Codec, D3Q19, D3Q19>, void, void, void>::run(ctx, args...);
    case GPLBM_D2Q5:
      return Fn<DevAdapter<Codec, D2Q5, D2Q5>, void, void, void>::run(ctx, args...);
    default:
      return Fn<DevAdapter<Codec, D3Q7, D3Q7>, void, void, void>::run(ctx, args...);
  }
}

template <template <class, class, class, class> class Fn, class... Args>
int dispatch(gplbm_ctx* ctx, Args... args) {
  const bool light = ctx->p.h_lattice == GPLBM_H_LIGHT;
  if (ctx->p.precision >= GPLBM_FP16_DEV)
    return ctx->p.precision == GPLBM_FP16_DEV ? dispatch_dev<Fn, F16Codec>(ctx, args...)
                                              : dispatch_dev<Fn, BF16Codec>(ctx, args...);
  switch (ctx->p.lattice) {
    case GPLBM_D2Q9:
      return light ? dispatch_prec<Fn, D2Q9, D2Q5>(ctx, args...)
                   : dispatch_prec<Fn, D2Q9, D2Q9>(ctx, args...);
    case GPLBM_D3Q19:
      return light ? dispatch_prec<Fn, D3Q19, D3Q7>(ctx, args...)
                   : dispatch_prec<Fn, D3Q19, D3Q19>(ctx, args...);
    case GPLBM_D2Q5:
      return dispatch_prec<Fn, D2Q5, D2Q5>(ctx, args...);
    default:
      return dispatch_prec<Fn, D3Q7, D3Q7>(ctx, args...);
  }
}

template <class L, class LH, class S, class C>
struct InitFn {
  static int run(gplbm_ctx* c, const double* a, const double* b) {
    return Ops<L, LH, S, C>::init(c, a, b);
  }
};
template <class A>
struct InitFn<A, void, void, void> {
  static int run(gplbm_ctx* c, const double* a, const double* b) { return A::init(c, a, b); }
};
template <class L, class LH, class S, class C>
struct StepFn {
  static int run(gplbm_ctx* c, int64_t n) {
    return c->sched == GPLBM_SCHED_FUSED ? Ops<L, LH, S, C>::step_fused(c, n)
                                         : Ops<L, LH, S, C>::step_split(c, n);
  }
};
template <class A>
struct StepFn<A, void, void, void> {
  static int run(gplbm_ctx* c, int64_t n) { return A::step(c, n); }
};
template <class L, class LH, class S, class C>
struct FieldsFn {
  static int run(gplbm_ctx* c, double* a, double* b, double* d) {
    return Ops<L, LH, S, C>::fields(c, a, b, d);
  }
};
template <class A>
struct FieldsFn<A, void, void, void> {
  static int run(gplbm_ctx* c, double* a, double* b, double* d) { return A::fields(c, a, b, d); }
};
template <class L, class LH, class S, class C>
struct DiagFn {
  static int run(gplbm_ctx* c, double* r) { return Ops<L, LH, S, C>::diag(c, r); }
};
template <class A>
struct DiagFn<A, void, void, void> {
  static int run(gplbm_ctx* c, double* r) { return A::diag(c, r); }
};

int choose_schedule(const gplbm_params& p) {
  const bool fused_ok = p.precision >= GPLBM_FP16_DEV
                            ? (two_d(p.lattice) || dev_fused_supported(p.nx, p.ny, p.nz, p.bc))
                        : two_d(p.lattice)           ? fused2d_supported(p.nx, p.ny)
                                                     : fused3d_supported(p.nx, p.ny, p.nz, p.bc);
  if (p.schedule == GPLBM_SCHED_SPLIT) return GPLBM_SCHED_SPLIT;
  if (p.schedule == GPLBM_SCHED_FUSED) return fused_ok ? GPLBM_SCHED_FUSED : -1;
  return fused_ok ? GPLBM_SCHED_FUSED : GPLBM_SCHED_SPLIT;
}

int use_device(gplbm_ctx* ctx) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(ctx, GPLBM_E_DEVICE, "hipGetDevice failed");
  if (dev != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
    return fail(ctx, GPLBM_E_DEVICE, "hipSetDevice failed");
  return GPLBM_OK;
}

// The reduction scratch of gplbm_diagnostics_noalloc: the partials of the
// fixed reduction grid and the final values, the same amount the borrowed
// buffer reserves for gplbm_diagnostics.  Every device holds its own copy for
// the life of the process; its device address is taken once per device (with
// that device current) when a context is created there, and only that address
// is handed to kernels.
constexpr int kMaxDevices = 64;
constexpr size_t kScratchDoubles = (size_t)kDiagBlocks * kDiagVals + kDiagVals;
std::mutex scratch_mu;
double* scratch_ptr[kMaxDevices] = {};
hipError_t scratch_err[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

// Device address of scratch on the current device `dev` (taken on the first
// call per device); nullptr with the HIP error in *err when it cannot be had.
double* scratch_on(int dev, hipError_t* err) {
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev] && scratch_err[dev] == hipSuccess) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      scratch_err[dev] = e != hipSuccess ? e : hipErrorInvalidSymbol;
    else
      scratch_ptr[dev] = (double*)ptr;
  }
  *err = scratch_err[dev];
  return scratch_ptr[dev];
}

// Copy the final reduction values from device memory and fill *out
// (synchronises the stream).
int finish_diagnostics(gplbm_ctx* ctx, const double* red, gplbm_diag* out) {
  double v[kDiagVals];
  hipError_t e = hipMemcpyAsync(v, red + kDiagBlocks * kDiagVals, sizeof(v),
                                hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return fail(ctx, GPLBM_E_DEVICE, std::string("diagnostics copy: ") + hipGetErrorString(e));
  out->step = ctx->step;
  out->total_mass = v[0];
  out->solid_fraction = v[1] / (double)ctx->N;
  out->solid_fraction_count = v[2] / (double)ctx->N;
  out->sum_phi = v[3];
  out->phi_min = v[4];
  out->phi_max = v[5];
  out->nonfinite = v[6] != 0.0 ? 1 : 0;
  out->reserved = 0;
  if (out->nonfinite) return fail(ctx, GPLBM_E_NONFINITE, "non-finite phi or c");
  return GPLBM_OK;
}

}  // namespace

extern "C" {

int gplbm_state_bytes(const gplbm_params* p, uint64_t* bytes) {
  if (check_params(p) || !bytes) return GPLBM_E_INVALID;
  *bytes = layout(p).total;
  return GPLBM_OK;
}

int gplbm_checkpoint_bytes(const gplbm_params* p, uint64_t* bytes) {
  if (check_params(p) || !bytes) return GPLBM_E_INVALID;
  *bytes = layout(p).ckpt;
  return GPLBM_OK;
}

int gplbm_create(const gplbm_params* p, void* dev_buf, uint64_t bytes, void* stream,
                 gplbm_ctx** out) {
  if (!out) return GPLBM_E_INVALID;
  *out = nullptr;
  if (check_params(p) || !dev_buf) return GPLBM_E_INVALID;
  if (((uintptr_t)dev_buf) % kAlign) return GPLBM_E_INVALID;
  const Layout lay = layout(p);
  if (bytes < lay.total) return GPLBM_E_SIZE;
  const int sched = choose_schedule(*p);
  if (sched < 0) return GPLBM_E_INVALID;
  gplbm_ctx* ctx = new gplbm_ctx();
  ctx->p = *p;
  if (two_d(ctx->p.lattice)) ctx->p.bc[2] = GPLBM_PERIODIC;
  ctx->Q = lattice_q(p->lattice);
  ctx->Qh = lattice_qh(p);
  ctx->N = (int64_t)p->nx * p->ny * p->nz;
  ctx->elem = lay.elem;
  ctx->pop_bytes = lay.pop;
  ctx->hpop_bytes = lay.hpop;
  ctx->mov_bytes = lay.mov;
  ctx->hmov_bytes = lay.hmov;
  ctx->phi_bytes = lay.phi;
  ctx->lam_bytes = lay.lam;
  char* b = (char*)dev_buf;
  const size_t pop = lay.pop, hpop = lay.hpop, phi = lay.phi, lam = lay.lam;
  const size_t pops = 2 * pop + 2 * hpop;
  ctx->G[0] = b;
  ctx->G[1] = b + pop;
  ctx->H[0] = b + 2 * pop;
  ctx->H[1] = b + 2 * pop + hpop;
  ctx->PHI[0] = b + pops;
  ctx->PHI[1] = b + pops + phi;
  ctx->LAM[0] = lam ? b + pops + 2 * phi : nullptr;
  ctx->LAM[1] = lam ? b + pops + 2 * phi + lam : nullptr;
  ctx->red = (double*)(b + pops + 2 * phi + 2 * lam);
  ctx->cur = 0;
  ctx->step = 0;
  ctx->ready = false;
  ctx->sched = sched;
  ctx->stream = (hipStream_t)stream;
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    delete ctx;
    return GPLBM_E_DEVICE;
  }
  // set-up of gplbm_diagnostics_noalloc on this device (a failure is
  // reported by that call, not here)
  hipError_t serr;
  (void)scratch_on(ctx->device, &serr);
  *out = ctx;
  return GPLBM_OK;
}

int gplbm_set_stream(gplbm_ctx* ctx, void* stream) {
  if (!ctx) return GPLBM_E_INVALID;
  ctx->stream = (hipStream_t)stream;
  return GPLBM_OK;
}

int gplbm_init_fields(gplbm_ctx* ctx, const double* phi0, const double* c0) {
  if (!ctx) return GPLBM_E_INVALID;
  if (!phi0 || !c0) return fail(ctx, GPLBM_E_INVALID, "null field pointer");
  if (int rc = use_device(ctx)) return rc;
  ctx->cur = 0;
  ctx->step = 0;
  int rc = dispatch<InitFn>(ctx, phi0, c0);
  ctx->ready = rc == GPLBM_OK;
  return rc;
}

int gplbm_step(gplbm_ctx* ctx, int64_t nsteps) {
  if (!ctx) return GPLBM_E_INVALID;
  if (nsteps < 0) return fail(ctx, GPLBM_E_INVALID, "negative step count");
  if (!ctx->ready) return fail(ctx, GPLBM_E_STATE, "step before init");
  if (int rc = use_device(ctx)) return rc;
  return dispatch<StepFn>(ctx, nsteps);
}

int gplbm_step_to(gplbm_ctx* ctx, const void* src_state, void* dst_state) {
  if (!ctx || !src_state || !dst_state || src_state == dst_state) return GPLBM_E_INVALID;
  if (int rc = use_device(ctx)) return rc;
  // run one step with the context's buffers pointed at the two saved states
  char* G0[2] = {ctx->G[0], ctx->G[1]};
  char* H0[2] = {ctx->H[0], ctx->H[1]};
  char* P0[2] = {ctx->PHI[0], ctx->PHI[1]};
  char* L0[2] = {ctx->LAM[0], ctx->LAM[1]};
  const int cur = ctx->cur;
  const int64_t step = ctx->step;
  const bool ready = ctx->ready;
  char* s = (char*)src_state;
  char* d = (char*)dst_state;
  const size_t pp = ctx->pop_bytes, hp = ctx->hpop_bytes, ph = ctx->phi_bytes;
  ctx->G[cur] = s;
  ctx->H[cur] = s + pp;
  ctx->PHI[cur] = s + pp + hp;
  ctx->LAM[cur] = ctx->lam_bytes ? s + pp + hp + ph : nullptr;
  ctx->G[1 - cur] = d;
  ctx->H[1 - cur] = d + pp;
  ctx->PHI[1 - cur] = d + pp + hp;
  ctx->LAM[1 - cur] = ctx->lam_bytes ? d + pp + hp + ph : nullptr;
  ctx->ready = true;
  const int rc = dispatch<StepFn>(ctx, 1);
  for (int a = 0; a < 2; ++a) {
    ctx->G[a] = G0[a];
    ctx->H[a] = H0[a];
    ctx->PHI[a] = P0[a];
    ctx->LAM[a] = L0[a];
  }
  ctx->cur = cur;
  ctx->step = step;
  ctx->ready = ready;
  return rc;
}

int64_t gplbm_step_count(const gplbm_ctx* ctx) { return ctx ? ctx->step : -1; }

int gplbm_read_fields(gplbm_ctx* ctx, double* phi, double* c, double* mu) {
  if (!ctx) return GPLBM_E_INVALID;
  if (!ctx->ready) return fail(ctx, GPLBM_E_STATE, "read before init");
  if (int rc = use_device(ctx)) return rc;
  return dispatch<FieldsFn>(ctx, phi, c, mu);
}

int gplbm_diagnostics(gplbm_ctx* ctx, gplbm_diag* out) {
  if (!ctx || !out) return GPLBM_E_INVALID;
  if (!ctx->ready) return fail(ctx, GPLBM_E_STATE, "diagnostics before init");
  if (int rc = use_device(ctx)) return rc;
  int rc = dispatch<DiagFn>(ctx, ctx->red);
  if (rc) return rc;
  return finish_diagnostics(ctx, ctx->red, out);
}

int gplbm_diagnostics_noalloc(gplbm_ctx* ctx, gplbm_diag* out) {
  if (!ctx || !out) return GPLBM_E_INVALID;
  if (!ctx->ready) return fail(ctx, GPLBM_E_STATE, "diagnostics before init");
  if (int rc = use_device(ctx)) return rc;
  // the reduction grid is fixed, so the scratch fits every grid
  // gplbm_create accepts; the check guards the layout it was sized for
  static_assert(kScratchDoubles == (size_t)kDiagBlocks * kDiagVals + kDiagVals,
                "scratch sized for the reduction grid");
  if (ctx->N > ((int64_t)1 << 40))
    return fail(ctx, GPLBM_E_SIZE, "diagnostics scratch: grid larger than 2^40 nodes");
  hipError_t serr = hipSuccess;
  double* red = scratch_on(ctx->device, &serr);
  if (!red)
    return fail(ctx, GPLBM_E_DEVICE,
                std::string("diagnostics scratch address: ") + hipGetErrorString(serr));
  // every partial and final value is written before it is read, so nothing
  // left by an earlier call needs clearing
  int rc = dispatch<DiagFn>(ctx, red);
  if (rc) return rc;
  return finish_diagnostics(ctx, red, out);
}

int gplbm_save_state(gplbm_ctx* ctx, void* dev_dst) {
  if (!ctx || !dev_dst) return GPLBM_E_INVALID;
  if (!ctx->ready) return fail(ctx, GPLBM_E_STATE, "save before init");
  if (int rc = use_device(ctx)) return rc;
  const int a = ctx->cur;
  char* d = (char*)dev_dst;
  const size_t pp = ctx->pop_bytes, hp = ctx->hpop_bytes, ph = ctx->phi_bytes;
  hipError_t e = hipMemcpyAsync(d, ctx->G[a], pp, hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d + pp, ctx->H[a], hp, hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d + pp + hp, ctx->PHI[a], ph, hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess && ctx->lam_bytes)
    e = hipMemcpyAsync(d + pp + hp + ph, ctx->LAM[a], ctx->lam_bytes, hipMemcpyDeviceToDevice,
                       ctx->stream);
  if (e != hipSuccess) return fail(ctx, GPLBM_E_DEVICE, std::string("save: ") + hipGetErrorString(e));
  return GPLBM_OK;
}

int gplbm_load_state(gplbm_ctx* ctx, const void* dev_src, int64_t step) {
  if (!ctx || !dev_src || step < 0) return GPLBM_E_INVALID;
  if (int rc = use_device(ctx)) return rc;
  const int a = ctx->cur;
  const char* s = (const char*)dev_src;
  const size_t pp = ctx->pop_bytes, hp = ctx->hpop_bytes, ph = ctx->phi_bytes;
  hipError_t e = hipMemcpyAsync(ctx->G[a], s, pp, hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctx->H[a], s + pp, hp, hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctx->PHI[a], s + pp + hp, ph, hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess && ctx->lam_bytes)
    e = hipMemcpyAsync(ctx->LAM[a], s + pp + hp + ph, ctx->lam_bytes, hipMemcpyDeviceToDevice,
                       ctx->stream);
  if (e != hipSuccess) return fail(ctx, GPLBM_E_DEVICE, std::string("load: ") + hipGetErrorString(e));
  ctx->step = step;
  ctx->ready = true;
  return GPLBM_OK;
}

int gplbm_schedule(const gplbm_ctx* ctx) { return ctx ? ctx->sched : GPLBM_E_INVALID; }

int gplbm_stream_copy(const void* src, void* dst, uint64_t bytes, void* stream) {
  if (!src || !dst || bytes % 16 || ((uintptr_t)src) % 16 || ((uintptr_t)dst) % 16)
    return GPLBM_E_INVALID;
  if (bytes == 0) return GPLBM_OK;
  const uint64_t n = bytes / 16, blocks = (n + kStreamThreads - 1) / kStreamThreads;
  if (blocks > 0x7fffffffull) return GPLBM_E_INVALID;
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(kStreamThreads), 0,
                     (hipStream_t)stream, (const StreamVec*)src, (StreamVec*)dst, n);
  return hipGetLastError() == hipSuccess ? GPLBM_OK : GPLBM_E_DEVICE;
}

const char* gplbm_last_error(const gplbm_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void gplbm_destroy(gplbm_ctx* ctx) { delete ctx; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Adjoint: FP64 reverse sweep over FP64, FP32 or deviation-format forward
// states.

namespace {

struct AdjLayout {
  size_t pop, hpop, fld, vec, red, total;
};

AdjLayout adj_layout(const gplbm_params* p) {
  AdjLayout l{};
  const int64_t N = (int64_t)p->nx * p->ny * p->nz;
  l.pop = round_up((size_t)lattice_q(p->lattice) * N * 8);  // A1: g populations
  l.hpop = round_up((size_t)lattice_qh(p) * N * 8);         // B1: h populations
  l.fld = round_up((size_t)N * 8);
  l.vec = round_up((size_t)3 * N * 8);
  l.red = round_up(sizeof(double) * (2 * kDiagBlocks + 2));
  // two sets (A1, B1, B2, B3, B4), A2..A4, two accumulators, reduction
  l.total = 2 * (l.pop + l.hpop + 2 * l.fld + l.vec) + (l.vec + 2 * l.fld) + 2 * l.fld + l.red;
  return l;
}

// A saved state (gplbm_save_state layout: G | H | PHI | LAM) as the forward
// state type FS of the reverse kernels.
template <class FS>
struct FwdFromState;
template <class S>
struct FwdFromState<FwdState<S>> {
  static FwdState<S> get(const gplbm_ctx* ctx, const void* ck) {
    const char* b = (const char*)ck;
    return FwdState<S>{(const S*)b, (const S*)(b + ctx->pop_bytes),
                       (const S*)(b + ctx->pop_bytes + ctx->hpop_bytes)};
  }
};
template <class Codec>
struct FwdFromState<DevFwdState<Codec>> {
  static DevFwdState<Codec> get(const gplbm_ctx* ctx, const void* ck) {
    char* b = (char*)const_cast<void*>(ck);
    DevFwdState<Codec> f;
    f.H.mov = (uint16_t*)(b + ctx->pop_bytes);
    f.H.rest = (float*)(b + ctx->pop_bytes + ctx->hmov_bytes);
    f.PHI = (const float*)(b + ctx->pop_bytes + ctx->hpop_bytes);
    f.LAM = (const float*)(b + ctx->pop_bytes + ctx->hpop_bytes + ctx->phi_bytes);
    return f;
  }
};

template <class L, class LH, class FS>
struct AdjOps {
  static dim3 block() { return dim3(64, 4, 1); }
  static dim3 grid(const gplbm_ctx* ctx) {
    return dim3((ctx->p.nx + 63) / 64, (ctx->p.ny + 3) / 4, ctx->p.nz);
  }
  static double lam_M_W2(const gplbm_ctx* ctx) { return ctx->p.M_phi / (ctx->p.W * ctx->p.W); }
  static int seed(gplbm_ctx* ctx, const double* phib, const double* cb) {
    const Geo g = make_geo(ctx->p);
    hipLaunchKernelGGL((k_adj_seed<L, LH>), grid(ctx), block(), 0, ctx->stream, g, phib, cb,
                       ctx->adj.set[ctx->adj_cur], ctx->adj);
    return check_launch(ctx, "adjoint seed");
  }
  static int step(gplbm_ctx* ctx, const void* s0, const void* s1) {
    const Geo g = make_geo(ctx->p);
    const Coef<double> K = make_coef<double>(ctx->p);
    const int a = ctx->adj_cur, b = 1 - a;
    const FS S0 = FwdFromState<FS>::get(ctx, s0), S1 = FwdFromState<FS>::get(ctx, s1);
    // the general reverse kernels only for h^eq,alt or eps_s != eps_l; the
    // periodic addressing when no axis has walls
    const bool gen = ctx->p.h_scheme != GPLBM_H_SOURCE || ctx->p.free_energy != GPLBM_FE_EQUAL;
    const bool per = !ctx->p.bc[0] && !ctx->p.bc[1] && !ctx->p.bc[2];
    auto launch = [&](auto kgen, auto kper) {
      constexpr bool G = decltype(kgen)::value, Pr = decltype(kper)::value;
      hipLaunchKernelGGL((k_adj_ra<L, LH, FS, G, Pr>), grid(ctx), block(), 0, ctx->stream, g, K,
                         lam_M_W2(ctx), S1, ctx->adj.set[a], ctx->adj.set[b], ctx->adj);
      hipLaunchKernelGGL((k_adj_rb<L, LH, FS, G, Pr>), grid(ctx), block(), 0, ctx->stream, g, K,
                         lam_M_W2(ctx), S0, S1, ctx->adj.set[a], ctx->adj.set[b], ctx->adj);
    };
    using T = std::true_type;
    using F = std::false_type;
    if (gen)
      per ? launch(T{}, T{}) : launch(T{}, F{});
    else
      per ? launch(F{}, T{}) : launch(F{}, F{});
    int rc = check_launch(ctx, "adjoint step");
    if (rc) return rc;
    ctx->adj_cur = b;
    return GPLBM_OK;
  }
  static int finish(gplbm_ctx* ctx, const double* phi0, const double* c0, double* phi0b,
                    double* c0b) {
    const Geo g = make_geo(ctx->p);
    const Coef<double> K = make_coef<double>(ctx->p);
    const int a = ctx->adj_cur, b = 1 - a;
    hipLaunchKernelGGL((k_adj_init_a<L, LH>), grid(ctx), block(), 0, ctx->stream, g, K, lam_M_W2(ctx),
                       phi0, c0, ctx->adj.set[a], ctx->adj.set[b], ctx->adj, c0b);
    hipLaunchKernelGGL((k_adj_init_b<L>), grid(ctx), block(), 0, ctx->stream, g, ctx->adj.set[b],
                       phi0b);
    hipLaunchKernelGGL(k_adj_reduce, dim3(kDiagBlocks), dim3(kDiagThreads), 0, ctx->stream,
                       (const double*)ctx->adj.lamb, (const double*)ctx->adj.dlb, g.N, ctx->adj.red);
    hipLaunchKernelGGL(k_adj_reduce_final, dim3(1), dim3(64), 0, ctx->stream,
                       (const double*)ctx->adj.red, kDiagBlocks, ctx->adj.red + 2 * kDiagBlocks);
    return check_launch(ctx, "adjoint finish");
  }
};

template <template <class, class, class> class Fn, class L, class LH, class... Args>
int adj_dispatch_prec(gplbm_ctx* ctx, Args... args) {
  switch (ctx->p.precision) {
    case GPLBM_FP64:
      return Fn<L, LH, FwdState<double>>::run(ctx, args...);
    case GPLBM_FP32:
      return Fn<L, LH, FwdState<float>>::run(ctx, args...);
    case GPLBM_FP16_DEV:
      return Fn<L, LH, DevFwdState<F16Codec>>::run(ctx, args...);
    default:
      return Fn<L, LH, DevFwdState<BF16Codec>>::run(ctx, args...);
  }
}

template <template <class, class, class> class Fn, class... Args>
int adj_dispatch(gplbm_ctx* ctx, Args... args) {
  const bool light = ctx->p.h_lattice == GPLBM_H_LIGHT;
  switch (ctx->p.lattice) {
    case GPLBM_D2Q9:
      return light ? adj_dispatch_prec<Fn, D2Q9, D2Q5>(ctx, args...)
                   : adj_dispatch_prec<Fn, D2Q9, D2Q9>(ctx, args...);
    case GPLBM_D3Q19:
      return light ? adj_dispatch_prec<Fn, D3Q19, D3Q7>(ctx, args...)
                   : adj_dispatch_prec<Fn, D3Q19, D3Q19>(ctx, args...);
    case GPLBM_D2Q5:
      return adj_dispatch_prec<Fn, D2Q5, D2Q5>(ctx, args...);
    default:
      return adj_dispatch_prec<Fn, D3Q7, D3Q7>(ctx, args...);
  }
}
template <class L, class LH, class FS>
struct AdjSeedFn {
  static int run(gplbm_ctx* c, const double* a, const double* b) {
    return AdjOps<L, LH, FS>::seed(c, a, b);
  }
};
template <class L, class LH, class FS>
struct AdjStepFn {
  static int run(gplbm_ctx* c, const void* a, const void* b) {
    return AdjOps<L, LH, FS>::step(c, a, b);
  }
};
template <class L, class LH, class FS>
struct AdjFinishFn {
  static int run(gplbm_ctx* c, const double* a, const double* b, double* d, double* e) {
    return AdjOps<L, LH, FS>::finish(c, a, b, d, e);
  }
};

// The adjoint covers every context the parameters allow: every precision
// (FP64, FP32, FP16 / BF16 deviations), every lattice combination, both h
// schemes and both free-energy forms.
bool adjoint_supported(const gplbm_params& p) { return check_params(&p) == nullptr; }

}  // namespace

extern "C" {

int gplbm_adjoint_bytes(const gplbm_params* p, uint64_t* bytes) {
  if (check_params(p) || !bytes || !adjoint_supported(*p)) return GPLBM_E_INVALID;
  *bytes = adj_layout(p).total;
  return GPLBM_OK;
}

int gplbm_adjoint_begin(gplbm_ctx* ctx, void* work, uint64_t bytes, const double* phi_bar,
                        const double* c_bar) {
  if (!ctx || !work || ((uintptr_t)work) % kAlign) return GPLBM_E_INVALID;
  if (!adjoint_supported(ctx->p)) {
    const char* why = check_params(&ctx->p);
    return fail(ctx, GPLBM_E_INVALID, std::string("adjoint: ") + (why ? why : "invalid parameters"));
  }
  const AdjLayout l = adj_layout(&ctx->p);
  if (bytes < l.total) return fail(ctx, GPLBM_E_SIZE, "adjoint workspace too small");
  if (int rc = use_device(ctx)) return rc;
  char* b = (char*)work;
  AdjWork& w = ctx->adj;
  for (int a = 0; a < 2; ++a) {
    w.set[a].A1 = (double*)b; b += l.pop;
    w.set[a].B1 = (double*)b; b += l.hpop;
    w.set[a].B2 = (double*)b; b += l.fld;
    w.set[a].B3 = (double*)b; b += l.vec;
    w.set[a].B4 = (double*)b; b += l.fld;
  }
  w.A2 = (double*)b; b += l.vec;
  w.A3 = (double*)b; b += l.fld;
  w.A4 = (double*)b; b += l.fld;
  w.lamb = (double*)b; b += l.fld;
  w.dlb = (double*)b; b += l.fld;
  w.red = (double*)b;
  ctx->adj_cur = 0;
  int rc = adj_dispatch<AdjSeedFn>(ctx, phi_bar, c_bar);
  ctx->adj_ready = rc == GPLBM_OK;
  return rc;
}

int gplbm_step_chain(gplbm_ctx* ctx, void* states, uint64_t stride, int64_t n) {
  if (!ctx || !states || n < 0 || stride % kAlign || (uintptr_t)states % kAlign)
    return GPLBM_E_INVALID;
  uint64_t need = 0;
  if (gplbm_checkpoint_bytes(&ctx->p, &need) || stride < need) return GPLBM_E_INVALID;
  char* s = (char*)states;
  for (int64_t j = 0; j < n; ++j)
    if (int rc = gplbm_step_to(ctx, s + j * stride, s + (j + 1) * stride)) return rc;
  return GPLBM_OK;
}

int gplbm_adjoint_segment(gplbm_ctx* ctx, const void* states, uint64_t stride, int64_t n) {
  if (!ctx || !states || n < 0 || stride % kAlign || (uintptr_t)states % kAlign)
    return GPLBM_E_INVALID;
  uint64_t need = 0;
  if (gplbm_checkpoint_bytes(&ctx->p, &need) || stride < need) return GPLBM_E_INVALID;
  if (!ctx->adj_ready) return fail(ctx, GPLBM_E_STATE, "adjoint segment before adjoint begin");
  const char* s = (const char*)states;
  for (int64_t j = n - 1; j >= 0; --j)
    if (int rc = gplbm_adjoint_step(ctx, s + j * stride, s + (j + 1) * stride)) return rc;
  return GPLBM_OK;
}

int gplbm_adjoint_step(gplbm_ctx* ctx, const void* state_n, const void* state_np1) {
  if (!ctx || !state_n || !state_np1) return GPLBM_E_INVALID;
  if (!ctx->adj_ready) return fail(ctx, GPLBM_E_STATE, "adjoint step before adjoint begin");
  if (int rc = use_device(ctx)) return rc;
  return adj_dispatch<AdjStepFn>(ctx, state_n, state_np1);
}

int gplbm_adjoint_finish(gplbm_ctx* ctx, const double* phi0, const double* c0, double* phi0_bar,
                         double* c0_bar, double* dJ_dparams) {
  if (!ctx || !phi0 || !c0 || !phi0_bar || !c0_bar || !dJ_dparams) return GPLBM_E_INVALID;
  if (!ctx->adj_ready) return fail(ctx, GPLBM_E_STATE, "adjoint finish before adjoint begin");
  if (int rc = use_device(ctx)) return rc;
  int rc = adj_dispatch<AdjFinishFn>(ctx, phi0, c0, phi0_bar, c0_bar);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(dJ_dparams, ctx->adj.red + 2 * kDiagBlocks, 2 * sizeof(double),
                                hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return fail(ctx, GPLBM_E_DEVICE, std::string("adjoint finish: ") + hipGetErrorString(e));
  ctx->adj_ready = false;
  return GPLBM_OK;
}

}  // extern "C"
