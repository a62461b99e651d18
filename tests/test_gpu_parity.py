"""GPU path against the CPU oracle, element by element, through the C ABI.

FP64: the norm err(a, b) = max|a - b| / max(max|b|, s), s = 1 for phi and c
and s = dc for mu - mu_eq, must stay below 1e-11.  Both sides evaluate the
same expressions in the same order, so the FP64 path is expected to be
bit-identical; the count of differing values is printed.

FP32 (float storage and collision, double moments and closure): the
tolerance follows from the arithmetic.  A step applies O(10) float operations
per value, each with relative rounding 2^-24 = 6e-8, to values of order 1;
rounding errors add up like a random walk over the steps, damped by the
relaxation, so after n steps the deviation stays within about
n^(1/2) * 1e-6.  The tests use 200 steps and a bound of 2e-5.
"""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _norm(a, b, s):
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), s))


def compare(p, got, exp):
    dc = p["c_s_co"] - p["c_l_co"]
    (phi_g, c_g, mu_g), (phi_e, c_e, mu_e) = got, exp
    errs = {"phi": _norm(phi_g, phi_e, 1.0), "c": _norm(c_g, c_e, 1.0),
            "mu": _norm(mu_g - p["mu_eq"], mu_e - p["mu_eq"], dc)}
    ndiff = int(sum(np.count_nonzero(a != b) for a, b in zip(got, exp)))
    return errs, ndiff


@pytest.fixture(scope="module")
def gp():
    import torch
    assert torch.cuda.is_available()
    from paper_2111_05960_amd import binding
    binding.load()
    return binding


CASES_2D = [
    # shape, bc, counter_term, anti_trapping
    ((1, 40, 72), (1, 0, 0), 1, 1),
    ((1, 37, 61), (0, 0, 0), 1, 1),
    ((1, 33, 70), (1, 1, 0), 0, 1),
    ((1, 24, 130), (0, 1, 0), 1, 0),
    ((1, 17, 9), (1, 1, 0), 0, 0),
    ((1, 3, 5), (0, 0, 0), 1, 1),
    ((1, 7, 200), (0, 1, 0), 0, 1),
]
CASES_3D = [
    ((12, 10, 14), (0, 0, 0), 1, 1),
    ((9, 13, 70), (1, 0, 1), 1, 1),
    ((10, 11, 12), (1, 1, 1), 0, 1),
    ((8, 16, 66), (0, 1, 0), 1, 0),
    ((70, 9, 13), (0, 0, 0), 1, 1),
    ((3, 4, 5), (0, 0, 0), 0, 1),
    ((33, 20, 130), (0, 0, 0), 1, 0),
    # whole and ragged x-tiles of 64, y-tiles of 6 / 12 / 13, one z chunk
    ((32, 12, 64), (0, 0, 0), 1, 1),
    ((6, 27, 128), (0, 0, 0), 0, 1),
    ((5, 7, 1), (0, 0, 0), 1, 1),
]


def _run_pair(gp, oracle_mod, lattice, shape, bc, ct, at, precision, schedule, steps, seed):
    p = wl.base_params(lattice=lattice, shape=shape, bc=bc, counter_term=ct, anti_trapping=at)
    phi0, c0 = wl.random_state_fields(shape, seed=seed)
    print(f"case lattice={lattice} shape={shape} bc={bc} ct={ct} at={at} "
          f"prec={precision} sched={schedule} steps={steps}", flush=True)
    sim = gp.Simulation(p, precision, schedule).init(phi0, c0)
    ref = oracle_mod.Oracle(p).init(phi0, c0)
    out = []
    for n in steps:
        sim.step(n - sim.step_count)
        ref.step(n - ref.step_count)
        out.append((n, compare(p, sim.fields(), ref.fields())))
    return sim, out


@pytest.mark.parametrize("schedule", ["split", "auto"])
@pytest.mark.parametrize("case", CASES_2D + CASES_3D)
def test_fp64_parity(gp, oracle_mod, case, schedule):
    shape, bc, ct, at = case
    lattice = wl.D2Q9 if shape[0] == 1 else wl.D3Q19
    sim, res = _run_pair(gp, oracle_mod, lattice, shape, bc, ct, at, "fp64", schedule,
                         (0, 1, 7, 60), seed=sum(shape))
    for n, (errs, ndiff) in res:
        print(f"  step {n}: schedule={sim.schedule} errs={errs} differing={ndiff}", flush=True)
        for k, e in errs.items():
            assert e <= 1e-11, (n, k, e)


@pytest.mark.parametrize("case", [CASES_2D[0], CASES_2D[1], CASES_3D[0], CASES_3D[1]])
def test_fp32_parity(gp, oracle_mod, case):
    shape, bc, ct, at = case
    lattice = wl.D2Q9 if shape[0] == 1 else wl.D3Q19
    sim, res = _run_pair(gp, oracle_mod, lattice, shape, bc, ct, at, "fp32", "auto",
                         (0, 200), seed=7)
    for n, (errs, _) in res:
        print(f"  step {n}: errs={errs}", flush=True)
        for k, e in errs.items():
            assert e <= 2e-5, (n, k, e)


def test_diagnostics_match_oracle(gp, oracle_mod):
    shape = (1, 48, 80)
    p = wl.base_params(shape=shape, bc=(0, 0, 0))
    phi0, c0 = wl.random_state_fields(shape, seed=2)
    sim = gp.Simulation(p, "fp64").init(phi0, c0).step(30)
    ref = oracle_mod.Oracle(p).init(phi0, c0).step(30)
    d, e = sim.diagnostics(), ref.diagnostics()
    assert d["step"] == e["step"] == 30
    for k in ("total_mass", "solid_fraction", "sum_phi"):
        assert abs(d[k] - e[k]) <= 1e-13 * max(abs(e[k]), 1.0), k
    for k in ("solid_fraction_count", "phi_min", "phi_max"):
        assert d[k] == e[k], k
    assert not d["nonfinite"]


def test_nonfinite_detected(gp):
    shape = (1, 16, 16)
    p = wl.base_params(shape=shape, bc=(0, 0, 0))
    phi0, c0 = wl.random_state_fields(shape, seed=2)
    phi0[0, 3, 5] = np.nan
    sim = gp.Simulation(p, "fp64").init(phi0, c0)
    with pytest.raises(gp.GplbmError) as e:
        sim.diagnostics()
    assert e.value.code == gp.GPLBM_E_NONFINITE
    assert sim.diagnostics(allow_nonfinite=True)["nonfinite"]


def test_checkpoint_resume_is_bitwise(gp):
    shape = (8, 12, 20)
    p = wl.base_params(lattice=wl.D3Q19, shape=shape, bc=(0, 1, 0))
    phi0, c0 = wl.random_state_fields(shape, seed=4)
    a = gp.Simulation(p, "fp64").init(phi0, c0).step(10)
    ck = a.checkpoint()
    a.step(15)
    b = gp.Simulation(p, "fp64").init(np.zeros(shape), np.zeros(shape)).restore(ck).step(15)
    assert b.step_count == a.step_count == 25
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("shape", [(1, 70, 150), (40, 30, 70)])
def test_tile_shape_and_schedule_invariance(gp, shape):
    """The fused and split schedules give identical bits."""
    lattice = wl.D2Q9 if shape[0] == 1 else wl.D3Q19
    p = wl.base_params(lattice=lattice, shape=shape, bc=(0, 0, 0))
    phi0, c0 = wl.random_state_fields(shape, seed=9)
    a = gp.Simulation(p, "fp64", "split").init(phi0, c0).step(25)
    b = gp.Simulation(p, "fp64", "fused").init(phi0, c0).step(25)
    assert b.schedule == "fused"
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)


# zero-flux walls in the 3-D z-march (the gather form, FP64 on D3Q19 with the
# g carry in registers on 64 x 5 tiles): several z chunks of 32 planes,
# ragged tiles, every lattice combination and the general instantiation;
# fused = split bit for bit, and FP64 equal to the oracle
WALL_CASES = [((40, 30, 70), (1, 1, 1)), ((33, 20, 130), (1, 0, 1)),
              ((20, 27, 64), (0, 1, 0)), ((70, 13, 66), (0, 0, 1)),
              ((5, 14, 128), (1, 1, 0))]
WALL_LATTICES = {"full": dict(lattice=wl.D3Q19), "h": dict(lattice=wl.D3Q19, h_lattice=1),
                 "gh": dict(lattice=wl.D3Q7)}


@pytest.mark.parametrize("which", sorted(WALL_LATTICES))
@pytest.mark.parametrize("shape", [(70, 14, 70), (130, 12, 64)])
def test_fp32_periodic_chunks_fused_equals_split(gp, shape, which):
    """Periodic FP32 z-march in z chunks of 64 planes: two and three chunks
    (the last ragged) give the bits of the split kernels."""
    p = wl.base_params(shape=shape, bc=(0, 0, 0), **WALL_LATTICES[which])
    phi0, c0 = wl.random_state_fields(shape, seed=41)
    print(f"case fp32 periodic chunks {which} {shape}", flush=True)
    a = gp.Simulation(p, "fp32", "split").init(phi0, c0).step(9)
    b = gp.Simulation(p, "fp32", "fused").init(phi0, c0).step(9)
    assert b.schedule == "fused" and a.schedule == "split"
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)
QUAD = dict(free_energy=1, eps_s=1.0, eps_l=2.3, m_s=0.9, m_l=0.12, df_min=0.02)


@pytest.mark.parametrize("variant", ["base", "alt+quad"])
@pytest.mark.parametrize("which", sorted(WALL_LATTICES))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", WALL_CASES)
def test_walls_fused_equals_split(gp, oracle_mod, prec, case, which, variant):
    shape, bc = case
    over = dict(WALL_LATTICES[which])
    if variant != "base":
        over.update(QUAD, h_scheme=1)
    p = wl.base_params(shape=shape, bc=bc, **over)
    phi0, c0 = wl.random_state_fields(shape, seed=39)
    print(f"case walls {which} {variant} {prec} {shape} bc={bc}", flush=True)
    a = gp.Simulation(p, prec, "split").init(phi0, c0).step(9)
    b = gp.Simulation(p, prec, "fused").init(phi0, c0).step(9)
    assert b.schedule == "fused" and a.schedule == "split"
    fa, fb = a.fields(), b.fields()
    for x, y in zip(fa, fb):
        assert np.array_equal(x, y)
    if prec == "fp64" and variant == "base":
        errs, ndiff = compare(p, fb, oracle_mod.Oracle(p).init(phi0, c0).step(9).fields())
        print(f"  vs oracle: errs={errs} differing={ndiff}", flush=True)
        for k, e in errs.items():
            assert e <= 1e-11, (k, e)
