"""Physical units to the lattice units the C ABI takes (dx = dt = 1).

Sec. 4.2 states its runs in physical units with a space step dx and a time
step dt.  Mobility and diffusivities scale as length^2 / time, the interface
width as a length, and gamma (whose inverse multiplies the diffusivity in
the c equilibrium) as time / length^2; lambda, a_at, the compositions, the
chemical potentials, the free-energy parameters and eps_n are dimensionless.
"""
from __future__ import annotations

_DIFFUSIVE = ("M_phi", "D_l", "D_s")


def to_lattice_units(phys: dict, dx: float, dt: float) -> dict:
    """A parameter mapping in physical units -> the same mapping in lattice
    units.  M_phi, D_l, D_s -> x dt / dx^2; W -> W / dx; gamma -> gamma dx^2 /
    dt (if absent: 1 / D_l in lattice units, the relaxation control of
    Sec. 3.3 that gives both LBEs the same stability margin when M and D are
    close); every other key is copied."""
    if not (dx > 0.0 and dt > 0.0):
        raise ValueError("dx and dt must be > 0")
    s = dt / (dx * dx)
    lat = dict(phys)
    for k in _DIFFUSIVE:
        if k in phys:
            lat[k] = phys[k] * s
    if "W" in phys:
        lat["W"] = phys["W"] / dx
    if "gamma" in phys:
        lat["gamma"] = phys["gamma"] / s
    elif "D_l" in lat:
        lat["gamma"] = 1.0 / lat["D_l"]
    return lat


def lattice_steps(t: float, dt: float) -> int:
    """Number of steps that reach the physical time t."""
    n = t / dt
    k = int(round(n))
    if abs(n - k) > 1e-9 * max(1.0, n):
        raise ValueError(f"t = {t} is not a whole number of steps of {dt}")
    return k
