"""Seeded synthetic inputs and workload recipes for the coupled phi / c step.

This module is shared by the GPU path's tests and benchmark and by the CPU
oracle's tests.  It holds no arithmetic of the lattice-Boltzmann scheme: it
builds initial fields (phi0, c0) as float64 numpy arrays of shape
(nz, ny, nx), x fastest, and parameter mappings in lattice units
(dx = dt = 1).

Parameter mappings carry the keys ``lattice`` (0 D2Q9, 1 D3Q19, 2 D2Q5, 3 D3Q7), ``shape``
(nz, ny, nx), ``bc`` (x, y, z; 0 periodic, 1 zero flux), ``counter_term``,
``anti_trapping`` and the scalars W, M_phi, lam, D_l, D_s, gamma, a_at,
c_s_co, c_l_co, mu_eq, eps_n.
"""
from __future__ import annotations

import math

import numpy as np

D2Q9, D3Q19 = 0, 1
D2Q5, D3Q7 = 2, 3  # g (and h) on the light lattices
PERIODIC, ZERO_FLUX = 0, 1

# Integrals of the thin-interface analysis as printed in Table 3 of the
# paper (q_s = 0, h = phi, a = 1/4): I, K and F.
TABLE3_I = 2.0 / 3.0
TABLE3_K = (31.0 - 30.0 * math.log(2.0)) / 150.0
TABLE3_F = math.log(2.0) / 4.0


def lambda_star(D_l: float, M_phi: float, dc: float,
                I: float = TABLE3_I, K: float = TABLE3_K, F: float = TABLE3_F) -> float:
    """Coupling that cancels the kinetic coefficient, Eq. (Lambda-Star):
    lambda* = D_l / (M_phi dc^2) * I / (K + F)."""
    return D_l / (M_phi * dc * dc) * I / (K + F)


def base_params(**over) -> dict:
    """Lattice-unit parameters shared by the workloads below.

    W = 2.5, M_phi = 0.05, D_l = 0.1, D_s = 0 with anti-trapping (a = 1/4),
    c_s^co = 1.0, c_l^co = 0.1, mu_eq = 0, gamma = 1/D_l, eps_n = 1e-2,
    lambda = lambda* from the printed Table 3 constants.
    """
    p = dict(lattice=D2Q9, shape=(1, 8, 512), bc=(ZERO_FLUX, PERIODIC, PERIODIC),
             counter_term=1, anti_trapping=1,
             W=2.5, M_phi=0.05, D_l=0.1, D_s=0.0, a_at=0.25,
             c_s_co=1.0, c_l_co=0.1, mu_eq=0.0, eps_n=1e-2)
    p["gamma"] = 1.0 / p["D_l"]
    p["lam"] = lambda_star(p["D_l"], p["M_phi"], p["c_s_co"] - p["c_l_co"])
    p.update(over)
    if "D_l" in over and "gamma" not in over:
        p["gamma"] = 1.0 / p["D_l"]
    return p


# --------------------------------------------------------------------------
# Initial fields


def tanh_profile(d, W):
    """Equilibrium phase-field profile phi0 = (1 + tanh(2 d / W)) / 2 as a
    function of the signed distance d (liquid side d > 0)."""
    return 0.5 * (1.0 + np.tanh(2.0 * np.asarray(d, dtype=np.float64) / W))


def planar(nx: int, ny: int, W: float, x0: float, c_solid: float, c_liquid: float):
    """Flat interface at x = x0: solid (phi = 0) for x < x0, liquid beyond.
    c0 = c_solid (1 - phi0) + c_liquid phi0."""
    x = np.arange(nx, dtype=np.float64)
    phi_row = tanh_profile(x - x0, W)
    phi0 = np.broadcast_to(phi_row, (1, ny, nx)).copy()
    c0 = c_solid * (1.0 - phi0) + c_liquid * phi0
    return phi0, c0


def disc(nx: int, ny: int, R: float, W: float, c_solid: float, c_liquid: float,
         center=None):
    """Solid disc of radius R (phi = 0 inside) in liquid."""
    if center is None:
        center = ((nx - 1) / 2.0, (ny - 1) / 2.0)
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    r = np.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2)
    phi0 = tanh_profile(r - R, W)[None]
    c0 = c_solid * (1.0 - phi0) + c_liquid * phi0
    return phi0, c0


def sphere(n: int, R: float, W: float, c_solid: float, c_liquid: float):
    """Solid ball of radius R centred in an n^3 box."""
    ctr = (n - 1) / 2.0
    a = np.arange(n, dtype=np.float64) - ctr
    r = np.sqrt(a[None, None, :] ** 2 + a[None, :, None] ** 2 + a[:, None, None] ** 2)
    phi0 = tanh_profile(r - R, W)
    c0 = c_solid * (1.0 - phi0) + c_liquid * phi0
    return phi0, c0


def gaussian_random_field(shape, seed: int, ell: float) -> np.ndarray:
    """Periodic Gaussian random field with covariance exp(-r^2 / (2 ell^2)),
    zero mean and unit variance (float32).  White noise from
    numpy.random.default_rng(seed), filtered in Fourier space by
    exp(-|k|^2 ell^2 / 4)."""
    import scipy.fft as sfft
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal(size=shape, dtype=np.float32)
    spec = sfft.rfftn(noise, workers=-1)
    del noise
    ks = [np.fft.fftfreq(n).astype(np.float32) * np.float32(2 * np.pi) for n in shape[:-1]]
    ks.append(np.fft.rfftfreq(shape[-1]).astype(np.float32) * np.float32(2 * np.pi))
    fac = np.float32(ell * ell / 4.0)
    filt = None
    for ax, k in enumerate(ks):
        sh = [1] * len(shape)
        sh[ax] = k.size
        term = np.exp(-fac * k.reshape(sh) ** 2)
        filt = term if filt is None else filt * term
    spec *= filt
    f = sfft.irfftn(spec, s=shape, workers=-1).astype(np.float32)
    del spec
    f -= f.mean(dtype=np.float64)
    f /= np.float32(f.std(dtype=np.float64))
    return f


def porous(shape, seed: int, ell: float, porosity: float, W: float,
           c_solid: float, c_liquid: float):
    """Porous medium from a thresholded Gaussian random field.

    Pores (liquid, phi = 1) are the points where the field exceeds its
    (1 - porosity) quantile.  The interface is smoothed to the equilibrium
    profile with the level-set distance d = (f - t) / |grad f| (periodic
    central differences), so phi0 = (1 + tanh(2 d / W)) / 2.
    ``shape`` is (ny, nx) or (nz, ny, nx); the result has 3 axes.
    """
    shape = tuple(int(s) for s in shape)
    f = gaussian_random_field(shape, seed, ell)
    flat = f.reshape(-1)
    k = int(round((1.0 - porosity) * flat.size))
    k = min(max(k, 0), flat.size - 1)
    thr = np.partition(flat, k)[k]
    g2 = np.zeros(shape, dtype=np.float32)
    for ax in range(len(shape)):
        d = (np.roll(f, -1, axis=ax) - np.roll(f, 1, axis=ax)) * np.float32(0.5)
        g2 += d * d
        del d
    gn = np.sqrt(g2)
    del g2
    np.maximum(gn, np.float32(1e-3), out=gn)
    dist = (f - thr) / gn
    del gn, f
    phi0 = tanh_profile(dist, W)
    del dist
    c0 = c_solid * (1.0 - phi0) + c_liquid * phi0
    if phi0.ndim == 2:
        phi0, c0 = phi0[None], c0[None]
    return phi0, c0


# --------------------------------------------------------------------------
# Workload recipes (lattice units)


def config0(counter_term: int = 1, lam=None):
    """Planar dissolution, D2Q9, 512 x 8, zero flux in x, periodic in y,
    interface at x = 100 (solid on the left), liquid c = 0 (undersaturated),
    4000 steps."""
    p = base_params(lattice=D2Q9, shape=(1, 8, 512), bc=(ZERO_FLUX, PERIODIC, PERIODIC),
                    counter_term=counter_term)
    if lam is not None:
        p["lam"] = lam
    phi0, c0 = planar(512, 8, p["W"], 100.0, p["c_s_co"], 0.0)
    return p, phi0, c0, 4000


def config1(counter_term: int = 1, lam=None, n: int = 1024, R: float = 200.0):
    """Circular grain (radius 200, centred) in a periodic 1024^2 D2Q9 box, at
    equilibrium composition c0 = c_co(phi0), 20000 steps."""
    p = base_params(lattice=D2Q9, shape=(1, n, n), bc=(PERIODIC, PERIODIC, PERIODIC),
                    counter_term=counter_term)
    if lam is not None:
        p["lam"] = lam
    phi0, c0 = disc(n, n, R, p["W"], p["c_s_co"], p["c_l_co"])
    return p, phi0, c0, 20000


def config_porous3d(n: int, seed: int = 0, ell: float = 8.0, porosity: float = 0.40):
    """3-D porous medium, D3Q19, periodic n^3 box, counter term and
    anti-trapping on, liquid c = 0 (configs at n = 256 and n = 512)."""
    p = base_params(lattice=D3Q19, shape=(n, n, n), bc=(PERIODIC, PERIODIC, PERIODIC),
                    counter_term=1)
    phi0, c0 = porous((n, n, n), seed, ell, porosity, p["W"], p["c_s_co"], 0.0)
    return p, phi0, c0


def crop_zero_flux(p: dict, phi0, c0, size: int = 64):
    """Crop [0, size)^d of a periodic workload, run with zero flux on every
    face."""
    q = dict(p)
    if q["lattice"] in (D3Q19, D3Q7):
        q["shape"] = (size, size, size)
        q["bc"] = (ZERO_FLUX, ZERO_FLUX, ZERO_FLUX)
        return q, phi0[:size, :size, :size].copy(), c0[:size, :size, :size].copy()
    q["shape"] = (1, size, size)
    q["bc"] = (ZERO_FLUX, ZERO_FLUX, PERIODIC)
    return q, phi0[:, :size, :size].copy(), c0[:, :size, :size].copy()


def config_porous2d(n: int = 512, seed: int = 1, ell: float = 6.0, porosity: float = 0.45):
    """2-D porous medium, D2Q9, periodic n^2 box (the differentiation
    workload, 4000 steps)."""
    p = base_params(lattice=D2Q9, shape=(1, n, n), bc=(PERIODIC, PERIODIC, PERIODIC),
                    counter_term=1)
    phi0, c0 = porous((n, n), seed, ell, porosity, p["W"], p["c_s_co"], 0.0)
    return p, phi0, c0, 4000


def random_state_fields(shape, seed: int, smooth: bool = True):
    """Small random but smooth-ish (phi0, c0) pair for parity tests: a
    porous field at correlation length 3 with porosity 0.5, W = 2.5, and c0
    perturbed by seeded noise of amplitude 0.05."""
    nz, ny, nx = shape
    sh = (ny, nx) if nz == 1 else (nz, ny, nx)
    phi0, c0 = porous(sh, seed, 3.0, 0.5, 2.5, 1.0, 0.0)
    rng = np.random.default_rng(seed + 1000)
    c0 = c0 + 0.05 * rng.standard_normal(c0.shape)
    return phi0.reshape(shape), c0.reshape(shape)


# --------------------------------------------------------------------------
# The paper's one-dimensional validation runs (Sec. 4.2) at its own
# parameters: domain [-0.25, 0.25] x [0, 0.0036], 5000 x 36 D2Q9 nodes,
# dx = 1e-4, dt = 5e-9, bounce-back walls at x = +-0.25, periodic in y.
# Diffusivities and mobilities scale by dt / dx^2 = 0.5, lengths by 1 / dx.

PAPER_DX, PAPER_DT = 1e-4, 5e-9


def paper_x(nx: int = 5000) -> np.ndarray:
    """Physical x of the node centres (walls half a cell beyond the ends)."""
    return -0.25 + (np.arange(nx) + 0.5) * PAPER_DX


def paper_validation(kind: str):
    """(params, phi0, c0) of the dissolution (D_s = 0, anti-trapping,
    W = 5e-3, lambda* = 230) or precipitation (D_s = 0.9, D_l = 1, no
    anti-trapping, W = 1.2e-3, lambda* = 277) validation; c^co = (0.6, 0.5),
    mu_eq = 0.4, M_phi = 1.2, D_l = 1 in physical units."""
    s = PAPER_DT / PAPER_DX ** 2
    if kind == "dissolution":
        W, lam, D_s, at, cs_inf, cl_inf = 5e-3, 230.0, 0.0, 1, 0.6, 0.4
    elif kind == "precipitation":
        W, lam, D_s, at, cs_inf, cl_inf = 1.2e-3, 277.0, 0.9, 0, 0.75, 0.4
    else:
        raise ValueError(kind)
    D_l = 1.0 * s
    p = base_params(lattice=D2Q9, shape=(1, 36, 5000), bc=(ZERO_FLUX, PERIODIC, PERIODIC),
                    counter_term=1, anti_trapping=at, W=W / PAPER_DX, M_phi=1.2 * s,
                    D_l=D_l, D_s=D_s * s, a_at=0.25 * (1.0 - D_s / 1.0), lam=lam,
                    c_s_co=0.6, c_l_co=0.5, mu_eq=0.4)
    x = paper_x()
    t = np.tanh(2.0 * x / W)
    phi1 = 0.5 * (1.0 + t)
    c1 = 0.5 * (cl_inf + cs_inf + (cl_inf - cs_inf) * t)
    phi0 = np.broadcast_to(phi1, (1, 36, 5000)).copy()
    c0 = np.broadcast_to(c1, (1, 36, 5000)).copy()
    return p, phi0, c0
