"""FP16 / BF16 deviation storage of the D3Q19 and D2Q9 states, through the
C ABI.

Bars:
  - the fused and the split schedule give identical bits (same float
    arithmetic on the same decoded values; the D3Q19 z-march and the D2Q9
    tile kernel);
  - against the FP64 oracle, the interface-position error d_int (the
    displacement |phi_dev - phi_ref| / |grad phi_ref| over the interface
    nodes 0.1 < phi_ref < 0.9 whose gradient is at least 1 / (4 W),
    tests/metrics.py) stays below 1e-3 lattice units with FP16 storage.  BF16 keeps 8
    significand bits against the 11 of FP16 (whose deviations are also scaled
    into the normal range), so its rounding is 8x coarser; its bound is 1e-2
    (8x the FP16 bar, plus margin) and its error is reported;
  - the solute mass is conserved to the FP32 rounding of one rest population
    per node and step (relative drift below 1e-6 over the run).
"""
import numpy as np
import pytest

import workloads as wl
from tests import metrics

pytestmark = pytest.mark.gpu

PRECS = ["fp16dev", "bf16dev"]


@pytest.fixture(scope="module")
def gp():
    import torch
    assert torch.cuda.is_available()
    from paper_2111_05960_amd import binding
    binding.load()
    return binding


def interface_error(phi_a, phi_b, grad_b, W=2.5):
    return metrics.interface_error(phi_a, phi_b, grad_b, W)[0]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("shape,lat", [((40, 30, 70), "full"), ((70, 30, 70), "full"),
                                       ((140, 14, 70), "full"), ((140, 14, 70), "gh")])
def test_dev_fused_equals_split(gp, prec, shape, lat):
    """Periodic z-march (z chunks of 128 planes): one chunk with a ragged
    tile row, and two chunks (128 planes and a ragged 12) over two tile
    columns, D3Q19 and g and h on D3Q7."""
    p = wl.base_params(lattice=wl.D3Q19 if lat == "full" else wl.D3Q7, shape=shape, bc=(0, 0, 0))
    print(f"case dev fused=split {prec} {shape} {lat}", flush=True)
    phi0, c0 = wl.random_state_fields(shape, seed=21)
    a = gp.Simulation(p, prec, "split").init(phi0, c0).step(12)
    b = gp.Simulation(p, prec, "fused").init(phi0, c0).step(12)
    assert b.schedule == "fused" and a.schedule == "split"
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)


def _lattice(shape):
    return wl.D2Q9 if shape[0] == 1 else wl.D3Q19


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", [((32, 32, 32), (0, 0, 0), 23), ((24, 20, 28), (1, 1, 1), 23),
                                  ((1, 96, 128), (0, 0, 0), 23), ((1, 70, 90), (1, 1, 0), 23),
                                  ((1, 70, 90), (1, 1, 0), 29)])
def test_dev_against_oracle(gp, oracle_mod, prec, case):
    """Seed 29 on the walled 70 x 90 grid is the instance on which the
    unfloored interface measure read 1.9e-3 in FP16 (a degenerate interface
    node with a vanishing gradient)."""
    shape, bc, seed = case
    p = wl.base_params(lattice=_lattice(shape), shape=shape, bc=bc)
    phi0, c0 = wl.random_state_fields(shape, seed=seed)
    steps = 300
    sim = gp.Simulation(p, prec).init(phi0, c0)
    m0 = sim.diagnostics()["total_mass"]
    sim.step(steps)
    m1 = sim.diagnostics()["total_mass"]
    ref = oracle_mod.Oracle(p).init(phi0, c0).step(steps)
    phi_r, c_r, mu_r = ref.fields()
    grad_r, _ = ref.gradient()
    phi_d, c_d, mu_d = sim.fields()
    dint = interface_error(phi_d, phi_r, grad_r)
    linf_phi = float(np.max(np.abs(phi_d - phi_r)))
    drift = abs(m1 - m0) / abs(m0)
    print(f"{prec} {shape} bc={bc}: d_int={dint:.3e} Linf(phi)={linf_phi:.3e} "
          f"Linf(c)={np.max(np.abs(c_d - c_r)):.3e} mass drift={drift:.3e} "
          f"schedule={sim.schedule}", flush=True)
    assert dint <= (1e-3 if prec == "fp16dev" else 1e-2)
    assert drift <= 1e-6


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", [((1, 70, 150), (0, 0, 0)), ((1, 53, 91), (1, 1, 0)),
                                  ((1, 40, 130), (1, 0, 0)), ((1, 33, 64), (0, 1, 0))])
def test_dev_d2q9_fused_equals_split(gp, prec, case):
    """D2Q9 deviation storage: the fused tile kernel (walls handled in the
    block) and the split kernels give identical bits; ragged tiles."""
    shape, bc = case
    p = wl.base_params(lattice=wl.D2Q9, shape=shape, bc=bc)
    phi0, c0 = wl.random_state_fields(shape, seed=27)
    a = gp.Simulation(p, prec, "split").init(phi0, c0).step(15)
    b = gp.Simulation(p, prec, "fused").init(phi0, c0).step(15)
    assert b.schedule == "fused" and a.schedule == "split"
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("shape", [(16, 20, 24), (1, 40, 52)])
def test_dev_checkpoint_resume(gp, prec, shape):
    p = wl.base_params(lattice=_lattice(shape), shape=shape, bc=(0, 0, 0))
    phi0, c0 = wl.random_state_fields(shape, seed=25)
    a = gp.Simulation(p, prec).init(phi0, c0).step(5)
    ck = a.checkpoint()
    a.step(7)
    b = gp.Simulation(p, prec).init(phi0, c0).restore(ck).step(7)
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)


# the scheme variants in the deviation formats: h^eq,alt (Eqs. LBE_Concent_Alt,
# Seq_Concent_Alt) and general quadratic free energies (Eqs. Closure,
# SourceTerm, Anti-Trapping_Quadratic), eps_l / eps_s = 2.3; same bars and the
# same seeded instance as the base-scheme test (seed 23).  The interface metric
# divides by |grad phi| over 0.1 < phi < 0.9 and is ill-conditioned on some
# geometries: on the 70 x 90 walled case with seed 29 the base scheme itself
# reads 1.9e-3 in FP16 and FP32 reads 1.3e-4 (4x its value elsewhere), with
# every variant at or below the base scheme there.
QUAD = dict(free_energy=1, eps_s=1.0, eps_l=2.3, m_s=0.9, m_l=0.12, df_min=0.02)
VARIANTS = {"alt": dict(h_scheme=1), "quad": QUAD, "alt+quad": dict(QUAD, h_scheme=1)}


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", [((32, 32, 32), (0, 0, 0)), ((1, 70, 90), (1, 1, 0))])
@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_dev_variants_against_oracle(gp, oracle_mod, prec, case, variant):
    shape, bc = case
    p = wl.base_params(lattice=_lattice(shape), shape=shape, bc=bc, **VARIANTS[variant])
    phi0, c0 = wl.random_state_fields(shape, seed=23)
    steps = 300
    sim = gp.Simulation(p, prec).init(phi0, c0)
    m0 = sim.diagnostics()["total_mass"]
    sim.step(steps)
    m1 = sim.diagnostics()["total_mass"]
    ref = oracle_mod.Oracle(p).init(phi0, c0).step(steps)
    phi_r, _, _ = ref.fields()
    grad_r, _ = ref.gradient()
    phi_d, _, _ = sim.fields()
    dint = interface_error(phi_d, phi_r, grad_r)
    drift = abs(m1 - m0) / abs(m0)
    print(f"{variant} {prec} {shape} bc={bc}: d_int={dint:.3e} "
          f"Linf(phi)={np.max(np.abs(phi_d - phi_r)):.3e} mass drift={drift:.3e} "
          f"schedule={sim.schedule}", flush=True)
    assert dint <= (1e-3 if prec == "fp16dev" else 1e-2)
    assert drift <= 1e-6


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", [((24, 30, 70), (0, 0, 0)), ((1, 53, 91), (1, 1, 0))])
@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_dev_variants_fused_equals_split(gp, prec, case, variant):
    shape, bc = case
    p = wl.base_params(lattice=_lattice(shape), shape=shape, bc=bc, **VARIANTS[variant])
    phi0, c0 = wl.random_state_fields(shape, seed=31)
    a = gp.Simulation(p, prec, "split").init(phi0, c0).step(12)
    b = gp.Simulation(p, prec, "fused").init(phi0, c0).step(12)
    assert b.schedule == "fused" and a.schedule == "split"
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)


# the light lattices in the deviation formats: h on D3Q7 under D3Q19 / D2Q5
# under D2Q9 ("h"), or g and h both on D3Q7 / D2Q5 ("gh"); same bars and
# instances as the base scheme
def _light(shape, bc, which):
    if which == "h":
        return wl.base_params(lattice=_lattice(shape), shape=shape, bc=bc, h_lattice=1)
    return wl.base_params(lattice=wl.D2Q5 if shape[0] == 1 else wl.D3Q7, shape=shape, bc=bc)


@pytest.mark.parametrize("which", ["h", "gh"])
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", [((32, 32, 32), (0, 0, 0)), ((24, 20, 28), (1, 1, 1)),
                                  ((1, 96, 128), (0, 0, 0)), ((1, 70, 90), (1, 1, 0))])
def test_dev_light_h_against_oracle(gp, oracle_mod, prec, case, which):
    shape, bc = case
    p = _light(shape, bc, which)
    phi0, c0 = wl.random_state_fields(shape, seed=23)
    steps = 300
    sim = gp.Simulation(p, prec).init(phi0, c0)
    assert sim.Qh == (5 if shape[0] == 1 else 7)
    m0 = sim.diagnostics()["total_mass"]
    sim.step(steps)
    m1 = sim.diagnostics()["total_mass"]
    ref = oracle_mod.Oracle(p).init(phi0, c0).step(steps)
    phi_r, _, _ = ref.fields()
    grad_r, _ = ref.gradient()
    phi_d, _, _ = sim.fields()
    dint = interface_error(phi_d, phi_r, grad_r)
    drift = abs(m1 - m0) / abs(m0)
    print(f"light {which} {prec} {shape} bc={bc}: d_int={dint:.3e} "
          f"Linf(phi)={np.max(np.abs(phi_d - phi_r)):.3e} mass drift={drift:.3e} "
          f"schedule={sim.schedule}", flush=True)
    assert dint <= (1e-3 if prec == "fp16dev" else 1e-2)
    assert drift <= 1e-6


@pytest.mark.parametrize("which", ["h", "gh"])
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", [((24, 30, 70), (0, 0, 0)), ((1, 53, 91), (1, 1, 0)),
                                  ((1, 70, 150), (0, 0, 0)), ((70, 14, 64), (0, 0, 0))])
def test_dev_light_h_fused_equals_split(gp, prec, case, which):
    shape, bc = case
    p = _light(shape, bc, which)
    phi0, c0 = wl.random_state_fields(shape, seed=33)
    a = gp.Simulation(p, prec, "split").init(phi0, c0).step(12)
    b = gp.Simulation(p, prec, "fused").init(phi0, c0).step(12)
    assert b.schedule == "fused" and a.schedule == "split"
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("which", ["h", "gh"])
@pytest.mark.parametrize("prec", PRECS)
def test_dev_light_h_checkpoint_resume(gp, prec, which):
    shape = (16, 20, 24)
    p = _light(shape, (0, 0, 0), which)
    phi0, c0 = wl.random_state_fields(shape, seed=35)
    a = gp.Simulation(p, prec).init(phi0, c0).step(5)
    ck = a.checkpoint()
    a.step(7)
    b = gp.Simulation(p, prec).init(phi0, c0).restore(ck).step(7)
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)


# both variants on the light lattices in the deviation formats (h alone or g
# and h on D3Q7 / D2Q5); h^eq,alt alone on the base scheme's instances and
# bars.  With the general free energy these instances amplify perturbations:
# an FP64 run from phi0 + 1e-6 noise ends 9.4e-4 (phi) and 9e-3 (c) away from
# the unperturbed one after 300 steps with g and h on D3Q7 (25x less with the
# D3Q7 h alone), although every form's error after one step is the same as on
# the base scheme (2e-5 in FP16).  There the check stops at 20 steps, where
# the same perturbation has grown to 1.1e-6 (phi) and 3e-5 (c), against the
# maximum norm of phi and c.
@pytest.mark.parametrize("which", ["h", "gh"])
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", [((32, 32, 32), (0, 0, 0)), ((1, 70, 90), (1, 1, 0))])
@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_dev_light_variants_against_oracle(gp, oracle_mod, prec, case, variant, which):
    shape, bc = case
    p = dict(_light(shape, bc, which), **VARIANTS[variant])
    phi0, c0 = wl.random_state_fields(shape, seed=23)
    short = "quad" in variant
    steps = 20 if short else 300
    sim = gp.Simulation(p, prec).init(phi0, c0)
    assert sim.Qh == (5 if shape[0] == 1 else 7)
    m0 = sim.diagnostics()["total_mass"]
    sim.step(steps)
    m1 = sim.diagnostics()["total_mass"]
    ref = oracle_mod.Oracle(p).init(phi0, c0).step(steps)
    phi_r, _, _ = ref.fields()
    grad_r, _ = ref.gradient()
    phi_d, _, _ = sim.fields()
    dint = interface_error(phi_d, phi_r, grad_r)
    drift = abs(m1 - m0) / abs(m0)
    c_d, c_r = sim.fields()[1], ref.fields()[1]
    e_phi, e_c = np.max(np.abs(phi_d - phi_r)), np.max(np.abs(c_d - c_r))
    print(f"light {which} {variant} {prec} {shape} bc={bc} steps={steps}: d_int={dint:.3e} "
          f"Linf(phi)={e_phi:.3e} Linf(c)={e_c:.3e} mass drift={drift:.3e} "
          f"schedule={sim.schedule}", flush=True)
    scale = 1.0 if prec == "fp16dev" else 8.0      # BF16 keeps 3 fewer mantissa bits
    if short:
        assert e_phi <= 1e-4 * scale and e_c <= 5e-4 * scale
    else:
        assert dint <= (1e-3 if prec == "fp16dev" else 1e-2)
    assert drift <= 1e-6


@pytest.mark.parametrize("which", ["h", "gh"])
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", [((24, 30, 70), (0, 0, 0)), ((1, 53, 91), (1, 1, 0))])
@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_dev_light_variants_fused_equals_split(gp, prec, case, variant, which):
    shape, bc = case
    p = dict(_light(shape, bc, which), **VARIANTS[variant])
    phi0, c0 = wl.random_state_fields(shape, seed=31)
    a = gp.Simulation(p, prec, "split").init(phi0, c0).step(12)
    b = gp.Simulation(p, prec, "fused").init(phi0, c0).step(12)
    assert b.schedule == "fused" and a.schedule == "split"
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)


# zero-flux walls in the deviation z-march: on every lattice combination and
# in the general instantiation, with several z chunks (32 planes each) and
# ragged tiles, the fused kernel gives the bits of the split kernels
WALL_CASES_3D = [((40, 30, 70), (1, 1, 1)), ((33, 20, 130), (1, 0, 1)),
                 ((20, 27, 64), (0, 1, 0)), ((70, 13, 66), (0, 0, 1)),
                 ((5, 14, 128), (1, 1, 0))]


@pytest.mark.parametrize("variant", ["base", "alt+quad"])
@pytest.mark.parametrize("which", ["full", "h", "gh"])
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", WALL_CASES_3D)
def test_dev_walls_fused_equals_split(gp, prec, case, which, variant):
    shape, bc = case
    p = (wl.base_params(lattice=wl.D3Q19, shape=shape, bc=bc) if which == "full"
         else _light(shape, bc, which))
    if variant != "base":
        p = dict(p, **VARIANTS[variant])
    phi0, c0 = wl.random_state_fields(shape, seed=37)
    print(f"case walls {which} {variant} {prec} {shape} bc={bc}", flush=True)
    a = gp.Simulation(p, prec, "split").init(phi0, c0).step(9)
    b = gp.Simulation(p, prec, "fused").init(phi0, c0).step(9)
    assert b.schedule == "fused" and a.schedule == "split"
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)
