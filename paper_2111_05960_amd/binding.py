"""ctypes binding of libgplbm.so (argument marshalling only).

Every function of the C ABI in include/gplbm.h has a Python function of the
same name here.  Device memory and streams come from PyTorch: pointers are
``tensor.data_ptr()`` and the stream is ``torch.cuda.current_stream()``.  No
arithmetic of the method runs in Python; if the library is missing this
module raises instead of falling back to anything else.

``Simulation`` is a convenience owner of one context: it allocates the
borrowed state buffer as a torch uint8 tensor on the current device and
exposes the C calls as methods.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GPLBM_LIBRARY") or os.path.join(HERE, "libgplbm.so")

GPLBM_OK = 0
GPLBM_E_INVALID = -1
GPLBM_E_SIZE = -2
GPLBM_E_DEVICE = -3
GPLBM_E_NONFINITE = -4
GPLBM_E_STATE = -5

GPLBM_D2Q9, GPLBM_D3Q19, GPLBM_D2Q5, GPLBM_D3Q7 = 0, 1, 2, 3
GPLBM_H_FULL, GPLBM_H_LIGHT = 0, 1
GPLBM_H_SOURCE, GPLBM_H_EQ_ALT = 0, 1
GPLBM_FE_EQUAL, GPLBM_FE_QUADRATIC = 0, 1
GPLBM_PERIODIC, GPLBM_ZERO_FLUX = 0, 1
GPLBM_FP64, GPLBM_FP32, GPLBM_FP16_DEV, GPLBM_BF16_DEV = 0, 1, 2, 3
GPLBM_SCHED_AUTO, GPLBM_SCHED_SPLIT, GPLBM_SCHED_FUSED = 0, 1, 2

PRECISIONS = {"fp64": GPLBM_FP64, "fp32": GPLBM_FP32, "fp16dev": GPLBM_FP16_DEV,
              "bf16dev": GPLBM_BF16_DEV}
SCHEDULES = {"auto": GPLBM_SCHED_AUTO, "split": GPLBM_SCHED_SPLIT, "fused": GPLBM_SCHED_FUSED}

# exported symbols of the C ABI (checked by the tests against the header)
SYMBOLS = ("gplbm_state_bytes", "gplbm_checkpoint_bytes", "gplbm_create", "gplbm_set_stream",
           "gplbm_init_fields", "gplbm_step", "gplbm_step_count", "gplbm_read_fields",
           "gplbm_diagnostics", "gplbm_save_state", "gplbm_load_state", "gplbm_schedule",
           "gplbm_last_error", "gplbm_destroy", "gplbm_adjoint_bytes", "gplbm_adjoint_begin",
           "gplbm_adjoint_step", "gplbm_adjoint_finish", "gplbm_step_to",
           "gplbm_diagnostics_noalloc", "gplbm_stream_copy", "gplbm_step_chain",
           "gplbm_adjoint_segment")


class gplbm_params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 3),
        ("precision", ctypes.c_int32),
        ("counter_term", ctypes.c_int32),
        ("anti_trapping", ctypes.c_int32),
        ("schedule", ctypes.c_int32),
        ("h_lattice", ctypes.c_int32),
        ("h_scheme", ctypes.c_int32),
        ("free_energy", ctypes.c_int32),
        ("W", ctypes.c_double), ("M_phi", ctypes.c_double), ("lam", ctypes.c_double),
        ("D_l", ctypes.c_double), ("D_s", ctypes.c_double), ("gamma", ctypes.c_double),
        ("a_at", ctypes.c_double), ("c_s_co", ctypes.c_double), ("c_l_co", ctypes.c_double),
        ("mu_eq", ctypes.c_double), ("eps_n", ctypes.c_double),
        ("eps_s", ctypes.c_double), ("eps_l", ctypes.c_double),
        ("m_s", ctypes.c_double), ("m_l", ctypes.c_double), ("df_min", ctypes.c_double),
    ]


class gplbm_diag(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64),
        ("total_mass", ctypes.c_double),
        ("solid_fraction", ctypes.c_double),
        ("solid_fraction_count", ctypes.c_double),
        ("sum_phi", ctypes.c_double),
        ("phi_min", ctypes.c_double),
        ("phi_max", ctypes.c_double),
        ("nonfinite", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


_lib = None


def load():
    """Load libgplbm.so (after torch, so both use the same HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(there is no fallback path)")
    try:
        import torch  # noqa: F401  (binds the process to torch's HIP runtime first)
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64
    P = ctypes.POINTER
    lib.gplbm_state_bytes.argtypes = [P(gplbm_params), P(u64)]
    lib.gplbm_checkpoint_bytes.argtypes = [P(gplbm_params), P(u64)]
    lib.gplbm_create.argtypes = [P(gplbm_params), vp, u64, vp, P(vp)]
    lib.gplbm_set_stream.argtypes = [vp, vp]
    lib.gplbm_init_fields.argtypes = [vp, vp, vp]
    lib.gplbm_step.argtypes = [vp, i64]
    lib.gplbm_step_count.argtypes = [vp]
    lib.gplbm_step_count.restype = i64
    lib.gplbm_read_fields.argtypes = [vp, vp, vp, vp]
    lib.gplbm_diagnostics.argtypes = [vp, P(gplbm_diag)]
    lib.gplbm_diagnostics_noalloc.argtypes = [vp, P(gplbm_diag)]
    lib.gplbm_stream_copy.argtypes = [vp, vp, u64, vp]
    lib.gplbm_step_chain.argtypes = [vp, vp, u64, i64]
    lib.gplbm_adjoint_segment.argtypes = [vp, vp, u64, i64]
    lib.gplbm_save_state.argtypes = [vp, vp]
    lib.gplbm_load_state.argtypes = [vp, vp, i64]
    lib.gplbm_schedule.argtypes = [vp]
    lib.gplbm_last_error.argtypes = [vp]
    lib.gplbm_last_error.restype = ctypes.c_char_p
    lib.gplbm_destroy.argtypes = [vp]
    lib.gplbm_destroy.restype = None
    lib.gplbm_step_to.argtypes = [vp, vp, vp]
    lib.gplbm_step_to.restype = ctypes.c_int
    lib.gplbm_adjoint_bytes.argtypes = [P(gplbm_params), P(u64)]
    lib.gplbm_adjoint_begin.argtypes = [vp, vp, u64, vp, vp]
    lib.gplbm_adjoint_step.argtypes = [vp, vp, vp]
    lib.gplbm_adjoint_finish.argtypes = [vp, vp, vp, vp, vp, P(ctypes.c_double)]
    for name in ("gplbm_state_bytes", "gplbm_checkpoint_bytes", "gplbm_create",
                 "gplbm_set_stream", "gplbm_init_fields", "gplbm_step", "gplbm_read_fields",
                 "gplbm_diagnostics", "gplbm_diagnostics_noalloc", "gplbm_save_state",
                 "gplbm_load_state", "gplbm_schedule", "gplbm_stream_copy",
                 "gplbm_adjoint_bytes", "gplbm_adjoint_begin", "gplbm_adjoint_step",
                 "gplbm_adjoint_finish"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def make_params(cfg, precision="fp64", schedule="auto") -> gplbm_params:
    """C parameter struct from a mapping with the keys lattice, shape
    (nz, ny, nx), bc, counter_term, anti_trapping, W, M_phi, lam, D_l, D_s,
    gamma, a_at, c_s_co, c_l_co, mu_eq, eps_n, and optionally h_lattice
    (0: h on the lattice of g, the default; 1: h on D2Q5 / D3Q7), h_scheme
    (0: source H_k, the default; 1: h^eq,alt) and free_energy (0: equal
    curvatures, the default; 1: general quadratic, with eps_s, eps_l, m_s,
    m_l, df_min)."""
    p = gplbm_params()
    nz, ny, nx = cfg["shape"]
    p.lattice = int(cfg["lattice"])
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    for a in range(3):
        p.bc[a] = int(cfg["bc"][a])
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.counter_term = int(cfg["counter_term"])
    p.anti_trapping = int(cfg["anti_trapping"])
    p.schedule = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
    p.h_lattice = int(cfg.get("h_lattice", 0))
    p.h_scheme = int(cfg.get("h_scheme", 0))
    p.free_energy = int(cfg.get("free_energy", 0))
    for key, default in (("eps_s", 1.0), ("eps_l", 1.0), ("m_s", 0.0), ("m_l", 0.0),
                         ("df_min", 0.0)):
        setattr(p, key, float(cfg.get(key, default)))
    for key in ("W", "M_phi", "lam", "D_l", "D_s", "gamma", "a_at", "c_s_co", "c_l_co",
                "mu_eq", "eps_n"):
        setattr(p, key, float(cfg[key]))
    return p


class GplbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gplbm error {code}: {msg}")
        self.code = code


# ---- thin wrappers with the C names --------------------------------------


def gplbm_state_bytes(p: gplbm_params) -> int:
    out = ctypes.c_uint64()
    rc = load().gplbm_state_bytes(ctypes.byref(p), ctypes.byref(out))
    if rc:
        raise GplbmError(rc, "invalid parameters")
    return out.value


def gplbm_checkpoint_bytes(p: gplbm_params) -> int:
    out = ctypes.c_uint64()
    rc = load().gplbm_checkpoint_bytes(ctypes.byref(p), ctypes.byref(out))
    if rc:
        raise GplbmError(rc, "invalid parameters")
    return out.value


def gplbm_create(p: gplbm_params, dev_buf: int, nbytes: int, stream: int):
    h = ctypes.c_void_p()
    rc = load().gplbm_create(ctypes.byref(p), ctypes.c_void_p(dev_buf), nbytes,
                             ctypes.c_void_p(stream), ctypes.byref(h))
    if rc:
        raise GplbmError(rc, "gplbm_create rejected the request")
    return h


def _check(ctx, rc):
    if rc:
        raise GplbmError(rc, load().gplbm_last_error(ctx).decode())


def gplbm_set_stream(ctx, stream: int):
    _check(ctx, load().gplbm_set_stream(ctx, ctypes.c_void_p(stream)))


def gplbm_init_fields(ctx, phi0_ptr: int, c0_ptr: int):
    _check(ctx, load().gplbm_init_fields(ctx, ctypes.c_void_p(phi0_ptr), ctypes.c_void_p(c0_ptr)))


def gplbm_step(ctx, nsteps: int):
    _check(ctx, load().gplbm_step(ctx, int(nsteps)))


def gplbm_step_count(ctx) -> int:
    return int(load().gplbm_step_count(ctx))


def gplbm_read_fields(ctx, phi_ptr, c_ptr, mu_ptr):
    _check(ctx, load().gplbm_read_fields(ctx, ctypes.c_void_p(phi_ptr or None),
                                         ctypes.c_void_p(c_ptr or None),
                                         ctypes.c_void_p(mu_ptr or None)))


def gplbm_diagnostics(ctx, allow_nonfinite: bool = False) -> dict:
    d = gplbm_diag()
    rc = load().gplbm_diagnostics(ctx, ctypes.byref(d))
    if rc and not (rc == GPLBM_E_NONFINITE and allow_nonfinite):
        _check(ctx, rc)
    return {"step": d.step, "total_mass": d.total_mass, "solid_fraction": d.solid_fraction,
            "solid_fraction_count": d.solid_fraction_count, "sum_phi": d.sum_phi,
            "phi_min": d.phi_min, "phi_max": d.phi_max, "nonfinite": bool(d.nonfinite)}


def gplbm_diagnostics_noalloc(ctx, allow_nonfinite: bool = False) -> dict:
    d = gplbm_diag()
    rc = load().gplbm_diagnostics_noalloc(ctx, ctypes.byref(d))
    if rc and not (rc == GPLBM_E_NONFINITE and allow_nonfinite):
        _check(ctx, rc)
    return {"step": d.step, "total_mass": d.total_mass, "solid_fraction": d.solid_fraction,
            "solid_fraction_count": d.solid_fraction_count, "sum_phi": d.sum_phi,
            "phi_min": d.phi_min, "phi_max": d.phi_max, "nonfinite": bool(d.nonfinite)}


def gplbm_stream_copy(src_ptr: int, dst_ptr: int, nbytes: int, stream: int):
    rc = load().gplbm_stream_copy(ctypes.c_void_p(src_ptr), ctypes.c_void_p(dst_ptr),
                                  int(nbytes), ctypes.c_void_p(stream))
    if rc:
        raise GplbmError(rc, "gplbm_stream_copy rejected the request")


def gplbm_save_state(ctx, dst_ptr: int):
    _check(ctx, load().gplbm_save_state(ctx, ctypes.c_void_p(dst_ptr)))


def gplbm_load_state(ctx, src_ptr: int, step: int):
    _check(ctx, load().gplbm_load_state(ctx, ctypes.c_void_p(src_ptr), int(step)))


def gplbm_schedule(ctx) -> int:
    return int(load().gplbm_schedule(ctx))


def gplbm_last_error(ctx) -> str:
    return load().gplbm_last_error(ctx).decode()


def gplbm_destroy(ctx):
    load().gplbm_destroy(ctx)


def gplbm_step_to(ctx, src_ptr: int, dst_ptr: int):
    _check(ctx, load().gplbm_step_to(ctx, ctypes.c_void_p(src_ptr), ctypes.c_void_p(dst_ptr)))


def gplbm_step_chain(ctx, states_ptr: int, stride: int, n: int):
    _check(ctx, load().gplbm_step_chain(ctx, ctypes.c_void_p(states_ptr), stride, n))


def gplbm_adjoint_segment(ctx, states_ptr: int, stride: int, n: int):
    _check(ctx, load().gplbm_adjoint_segment(ctx, ctypes.c_void_p(states_ptr), stride, n))


def gplbm_adjoint_bytes(p: gplbm_params) -> int:
    out = ctypes.c_uint64()
    rc = load().gplbm_adjoint_bytes(ctypes.byref(p), ctypes.byref(out))
    if rc:
        raise GplbmError(rc, "gplbm_adjoint_bytes rejected the parameters (see "
                         "gplbm_state_bytes for the checks they must pass)")
    return out.value


def gplbm_adjoint_begin(ctx, work_ptr: int, nbytes: int, phi_bar_ptr, c_bar_ptr):
    _check(ctx, load().gplbm_adjoint_begin(ctx, ctypes.c_void_p(work_ptr), nbytes,
                                           ctypes.c_void_p(phi_bar_ptr or None),
                                           ctypes.c_void_p(c_bar_ptr or None)))


def gplbm_adjoint_step(ctx, state_n_ptr: int, state_np1_ptr: int):
    _check(ctx, load().gplbm_adjoint_step(ctx, ctypes.c_void_p(state_n_ptr),
                                          ctypes.c_void_p(state_np1_ptr)))


def gplbm_adjoint_finish(ctx, phi0_ptr, c0_ptr, phi0_bar_ptr, c0_bar_ptr):
    out = (ctypes.c_double * 2)()
    _check(ctx, load().gplbm_adjoint_finish(ctx, ctypes.c_void_p(phi0_ptr), ctypes.c_void_p(c0_ptr),
                                            ctypes.c_void_p(phi0_bar_ptr),
                                            ctypes.c_void_p(c0_bar_ptr), out))
    return out[0], out[1]


# ---- convenience owner ----------------------------------------------------


class Simulation:
    """One context with its state buffer allocated by torch on the current
    device and ordered on torch's current stream."""

    def __init__(self, cfg, precision="fp64", schedule="auto", device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("gplbm needs a HIP device")
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.cfg = dict(cfg)
        self.params = make_params(cfg, precision, schedule)
        self.shape = tuple(int(s) for s in cfg["shape"])
        self.N = self.shape[0] * self.shape[1] * self.shape[2]
        lat = self.params.lattice
        self.Q = {GPLBM_D2Q9: 9, GPLBM_D3Q19: 19, GPLBM_D2Q5: 5, GPLBM_D3Q7: 7}[lat]
        if self.params.h_lattice == GPLBM_H_LIGHT or lat in (GPLBM_D2Q5, GPLBM_D3Q7):
            self.Qh = 5 if lat in (GPLBM_D2Q9, GPLBM_D2Q5) else 7
        else:
            self.Qh = self.Q
        nbytes = gplbm_state_bytes(self.params)
        with torch.cuda.device(self.device):
            self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.buf.data_ptr()
            aligned = (base + 255) // 256 * 256
            self.stream = torch.cuda.current_stream(self.device)
            self.ctx = gplbm_create(self.params, aligned, nbytes, self.stream.cuda_stream)

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx:
            gplbm_destroy(ctx)
            self.ctx = None

    @property
    def schedule(self) -> str:
        return {GPLBM_SCHED_SPLIT: "split", GPLBM_SCHED_FUSED: "fused"}[gplbm_schedule(self.ctx)]

    @property
    def step_count(self) -> int:
        return gplbm_step_count(self.ctx)

    def init(self, phi0, c0):
        torch = self.torch
        phi0 = torch.as_tensor(phi0, dtype=torch.float64).reshape(-1).to(self.device).contiguous()
        c0 = torch.as_tensor(c0, dtype=torch.float64).reshape(-1).to(self.device).contiguous()
        assert phi0.numel() == self.N and c0.numel() == self.N
        gplbm_init_fields(self.ctx, phi0.data_ptr(), c0.data_ptr())
        self._keep = (phi0, c0)  # keep alive until the stream has consumed them
        return self

    def step(self, n: int = 1):
        gplbm_step(self.ctx, n)
        return self

    def fields_device(self):
        torch = self.torch
        out = [torch.empty(self.N, dtype=torch.float64, device=self.device) for _ in range(3)]
        gplbm_read_fields(self.ctx, out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr())
        return tuple(t.view(self.shape) for t in out)

    def fields(self):
        """(phi, c, mu) at the current time as numpy arrays (nz, ny, nx)."""
        return tuple(t.cpu().numpy() for t in self.fields_device())

    def diagnostics(self, allow_nonfinite=False) -> dict:
        return gplbm_diagnostics(self.ctx, allow_nonfinite)

    def checkpoint(self):
        t = self.torch.empty(gplbm_checkpoint_bytes(self.params), dtype=self.torch.uint8,
                             device=self.device)
        gplbm_save_state(self.ctx, t.data_ptr())
        return t, self.step_count

    def restore(self, ckpt):
        t, step = ckpt
        gplbm_load_state(self.ctx, t.data_ptr(), step)
        return self
