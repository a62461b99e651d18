"""FP64 CPU oracle of the coupled phi / c lattice-Boltzmann step (arXiv:2111.05960).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke entry point and by
the CPU-baseline leg of bench.py.  The GPU library never imports it and shares
no code with it.  What it computes (and the readings of the paper it applies)
is stated in oracle.c.

Parameters are passed as a plain mapping with the keys of ``PARAM_KEYS``
(lattice units); fields are numpy float64 arrays of shape (nz, ny, nx).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# A prebuilt oracle library to load instead (the mutation check of the pins
# runs them against deliberately broken copies of oracle.c).
_LIB_OVERRIDE = os.environ.get("GPLBM_ORACLE_LIB")

D2Q9, D3Q19 = 0, 1
D2Q5, D3Q7 = 2, 3  # g (and h) on the light lattices
PERIODIC, ZERO_FLUX = 0, 1

PARAM_KEYS = ("W", "M_phi", "lam", "D_l", "D_s", "gamma", "a_at",
              "c_s_co", "c_l_co", "mu_eq", "eps_n")
# general quadratic free energies (free_energy = 1), with their defaults
QUADRATIC_KEYS = (("eps_s", 1.0), ("eps_l", 1.0), ("m_s", 0.0), ("m_l", 0.0), ("df_min", 0.0))


class _Params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 3),
        ("counter_term", ctypes.c_int32),
        ("anti_trapping", ctypes.c_int32),
        ("h_lattice", ctypes.c_int32),
        ("h_scheme", ctypes.c_int32),
        ("free_energy", ctypes.c_int32),
        ("W", ctypes.c_double), ("M_phi", ctypes.c_double),
        ("lam", ctypes.c_double), ("D_l", ctypes.c_double),
        ("D_s", ctypes.c_double), ("gamma", ctypes.c_double),
        ("a_at", ctypes.c_double), ("c_s_co", ctypes.c_double),
        ("c_l_co", ctypes.c_double), ("mu_eq", ctypes.c_double),
        ("eps_n", ctypes.c_double),
        ("eps_s", ctypes.c_double), ("eps_l", ctypes.c_double),
        ("m_s", ctypes.c_double), ("m_l", ctypes.c_double),
        ("df_min", ctypes.c_double),
    ]


def compile_library(src: str, out: str, quiet: bool = False) -> None:
    """gcc, FP contraction off, OpenMP on."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-I", _HERE, "-o", out, src, "-lm"]
    subprocess.run(cmd, check=True, capture_output=quiet)


def build(force: bool = True) -> str:
    """Compile liboracle.so (unless a library override is set)."""
    if _LIB_OVERRIDE:
        return _LIB_OVERRIDE
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        compile_library(_SRC, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            path = _LIB_OVERRIDE
        else:
            path = build(force=False)
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        lib.orc_create.restype = ctypes.c_void_p
        lib.orc_create.argtypes = [P(_Params)]
        lib.orc_destroy.argtypes = [ctypes.c_void_p]
        lib.orc_q.argtypes = [ctypes.c_void_p]
        lib.orc_qh.argtypes = [ctypes.c_void_p]
        lib.orc_nodes.restype = ctypes.c_int64
        lib.orc_nodes.argtypes = [ctypes.c_void_p]
        lib.orc_step_count.restype = ctypes.c_int64
        lib.orc_step_count.argtypes = [ctypes.c_void_p]
        lib.orc_init.argtypes = [ctypes.c_void_p, dp, dp]
        lib.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        lib.orc_fields.argtypes = [ctypes.c_void_p, dp, dp, dp]
        lib.orc_gradient.argtypes = [ctypes.c_void_p, dp, dp]
        lib.orc_get_state.argtypes = [ctypes.c_void_p, dp, dp, dp]
        lib.orc_set_state.argtypes = [ctypes.c_void_p, dp, dp, dp, ctypes.c_int64]
        lib.orc_diagnostics.argtypes = [ctypes.c_void_p, dp]
        lib.orc_local.argtypes = [P(_Params), ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def threads() -> int:
    return int(_load().orc_threads())


def _params(cfg) -> _Params:
    nz, ny, nx = cfg["shape"]
    p = _Params()
    p.lattice = int(cfg["lattice"])
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    for a in range(3):
        p.bc[a] = int(cfg["bc"][a])
    p.counter_term = int(cfg["counter_term"])
    p.anti_trapping = int(cfg["anti_trapping"])
    p.h_lattice = int(cfg.get("h_lattice", 0))
    p.h_scheme = int(cfg.get("h_scheme", 0))
    p.free_energy = int(cfg.get("free_energy", 0))
    for key in PARAM_KEYS:
        setattr(p, key, float(cfg[key]))
    for key, default in QUADRATIC_KEYS:
        setattr(p, key, float(cfg.get(key, default)))
    return p


def local(cfg, phi: float, c: float, mu: float):
    """The oracle's local forms at one point: (closure mu(c, phi), bracket
    of S_phi at mu, composition jump of the anti-trapping current at mu)."""
    out = np.empty(3)
    _load().orc_local(ctypes.byref(_params(cfg)), float(phi), float(c), float(mu), _ptr(out))
    return float(out[0]), float(out[1]), float(out[2])


class Oracle:
    """One simulation on the CPU oracle.

    ``cfg`` is a mapping with ``lattice`` (0 D2Q9, 1 D3Q19), ``shape``
    (nz, ny, nx), ``bc`` (per axis x, y, z: 0 periodic, 1 zero flux),
    ``counter_term``, ``anti_trapping``, the scalar keys of PARAM_KEYS and
    optionally ``h_lattice`` (0: h on the lattice of g, 1: h on D2Q5 / D3Q7),
    ``h_scheme`` (0: source H_k, 1: h^eq,alt) and ``free_energy`` (0: equal
    curvatures, 1: general quadratic with the keys of QUADRATIC_KEYS).
    """

    def __init__(self, cfg):
        lib = _load()
        nz, ny, nx = cfg["shape"]
        p = _params(cfg)
        self._p = p
        self.shape = (nz, ny, nx)
        self._h = lib.orc_create(ctypes.byref(p))
        if not self._h:
            raise ValueError("oracle rejected the parameters")
        self.Q = lib.orc_q(self._h)
        self.Qh = lib.orc_qh(self._h)
        self.N = nx * ny * nz
        self._lib = lib

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    def init(self, phi0, c0):
        phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(-1)
        c0 = np.ascontiguousarray(c0, dtype=np.float64).reshape(-1)
        assert phi0.size == self.N and c0.size == self.N
        self._lib.orc_init(self._h, _ptr(phi0), _ptr(c0))
        return self

    def step(self, n: int = 1):
        rc = self._lib.orc_step(self._h, int(n))
        if rc != 0:
            raise RuntimeError(f"oracle step failed ({rc})")
        return self

    @property
    def step_count(self) -> int:
        return int(self._lib.orc_step_count(self._h))

    def fields(self):
        """(phi, c, mu) at the current time, each of shape (nz, ny, nx)."""
        phi = np.empty(self.N)
        c = np.empty(self.N)
        mu = np.empty(self.N)
        self._lib.orc_fields(self._h, _ptr(phi), _ptr(c), _ptr(mu))
        return tuple(a.reshape(self.shape) for a in (phi, c, mu))

    def gradient(self):
        """(grad, normal) of the current phi, each of shape (nz, ny, nx, 3)."""
        g = np.empty(3 * self.N)
        n = np.empty(3 * self.N)
        self._lib.orc_gradient(self._h, _ptr(g), _ptr(n))
        return g.reshape(self.shape + (3,)), n.reshape(self.shape + (3,))

    def state(self):
        """Natural state (g, h, phi): populations of shape (Q, nz, ny, nx)."""
        g = np.empty(self.Q * self.N)
        h = np.empty(self.Qh * self.N)
        phi = np.empty(self.N)
        self._lib.orc_get_state(self._h, _ptr(g), _ptr(h), _ptr(phi))
        return (g.reshape((self.Q,) + self.shape), h.reshape((self.Qh,) + self.shape),
                phi.reshape(self.shape))

    def set_state(self, g, h, phi, step: int = 0):
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1)
        h = np.ascontiguousarray(h, dtype=np.float64).reshape(-1)
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1)
        self._lib.orc_set_state(self._h, _ptr(g), _ptr(h), _ptr(phi), int(step))
        return self

    def diagnostics(self) -> dict:
        out = np.empty(8)
        self._lib.orc_diagnostics(self._h, _ptr(out))
        return {"total_mass": out[0], "solid_fraction": out[1],
                "solid_fraction_count": out[2], "sum_phi": out[3],
                "phi_min": out[4], "phi_max": out[5],
                "nonfinite": bool(out[6]), "step": int(out[7])}
