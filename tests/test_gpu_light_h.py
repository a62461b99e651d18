"""The light lattices on the GPU against the oracle, through the C ABI:
h on D2Q5 / D3Q7 under g on D2Q9 / D3Q19 ("h"), and g and h both on D2Q5 /
D3Q7 ("gh").

The composition LBE needs only the zeroth moment and an isotropic second
moment of its equilibrium (Sec. 3.3), which the light lattices carry; with
tau_h = 1 / (gamma xi_s^2) the diffusivity is unchanged, and with
tau_g = M_phi / xi_s^2 the mobility.  The same bars as for the full lattice
apply: FP64 bit-identical to the oracle (norm <= 1e-11, the count of
differing values printed), FP32 within 2e-5 after 200 steps.  The cases are
the full-lattice parity cases (walls, ragged tiles, both schedules), plus the
schedule invariance and a checkpoint round trip, which exercise the separate
sizes of the g and h distributions in the state.
"""
import numpy as np
import pytest

import workloads as wl
from tests.test_gpu_parity import CASES_2D, CASES_3D, compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gp():
    import torch
    assert torch.cuda.is_available()
    from paper_2111_05960_amd import binding
    binding.load()
    return binding


def _params(shape, bc, ct, at, which="h"):
    if which == "h":
        lattice = wl.D2Q9 if shape[0] == 1 else wl.D3Q19
        return wl.base_params(lattice=lattice, shape=shape, bc=bc, counter_term=ct,
                              anti_trapping=at, h_lattice=1)
    lattice = wl.D2Q5 if shape[0] == 1 else wl.D3Q7
    return wl.base_params(lattice=lattice, shape=shape, bc=bc, counter_term=ct, anti_trapping=at)


def _run_pair(gp, oracle_mod, case, precision, schedule, steps, seed, which="h"):
    shape, bc, ct, at = case
    p = _params(shape, bc, ct, at, which)
    phi0, c0 = wl.random_state_fields(shape, seed=seed)
    print(f"case light-{which} shape={shape} bc={bc} ct={ct} at={at} prec={precision} "
          f"sched={schedule} steps={steps}", flush=True)
    sim = gp.Simulation(p, precision, schedule).init(phi0, c0)
    assert sim.Qh == (5 if shape[0] == 1 else 7)
    assert sim.Q == (sim.Qh if which == "gh" else (9 if shape[0] == 1 else 19))
    ref = oracle_mod.Oracle(p).init(phi0, c0)
    out = []
    for n in steps:
        sim.step(n - sim.step_count)
        ref.step(n - ref.step_count)
        out.append((n, compare(p, sim.fields(), ref.fields())))
    return sim, out


@pytest.mark.parametrize("which", ["h", "gh"])
@pytest.mark.parametrize("schedule", ["split", "auto"])
@pytest.mark.parametrize("case", CASES_2D + CASES_3D)
def test_fp64_parity_light(gp, oracle_mod, case, schedule, which):
    sim, res = _run_pair(gp, oracle_mod, case, "fp64", schedule, (0, 1, 7, 60),
                         seed=sum(case[0]) + 1, which=which)
    for n, (errs, ndiff) in res:
        print(f"  step {n}: schedule={sim.schedule} errs={errs} differing={ndiff}", flush=True)
        for k, e in errs.items():
            assert e <= 1e-11, (n, k, e)


@pytest.mark.parametrize("which", ["h", "gh"])
@pytest.mark.parametrize("case", [CASES_2D[0], CASES_2D[2], CASES_3D[0], CASES_3D[7]])
def test_fp32_parity_light(gp, oracle_mod, case, which):
    sim, res = _run_pair(gp, oracle_mod, case, "fp32", "auto", (0, 200), seed=5, which=which)
    for n, (errs, _) in res:
        print(f"  step {n}: schedule={sim.schedule} errs={errs}", flush=True)
        for k, e in errs.items():
            assert e <= 2e-5, (n, k, e)


@pytest.mark.parametrize("which", ["h", "gh"])
@pytest.mark.parametrize("shape", [(1, 70, 150), (40, 30, 70)])
def test_schedule_invariance_light(gp, shape, which):
    """Fused and split schedules give identical bits on the light lattices."""
    p = _params(shape, (0, 0, 0), 1, 1, which)
    phi0, c0 = wl.random_state_fields(shape, seed=19)
    a = gp.Simulation(p, "fp64", "split").init(phi0, c0).step(25)
    b = gp.Simulation(p, "fp64", "fused").init(phi0, c0).step(25)
    assert b.schedule == "fused"
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("which", ["h", "gh"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_checkpoint_resume_light(gp, prec, which):
    shape = (8, 12, 20)
    p = _params(shape, (0, 1, 0), 1, 1, which)
    phi0, c0 = wl.random_state_fields(shape, seed=4)
    a = gp.Simulation(p, prec).init(phi0, c0).step(10)
    ck = a.checkpoint()
    a.step(15)
    b = gp.Simulation(p, prec).init(np.zeros(shape), np.zeros(shape)).restore(ck).step(15)
    assert b.step_count == a.step_count == 25
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("which", ["h", "gh"])
def test_diagnostics_light_match_oracle(gp, oracle_mod, which):
    shape = (10, 14, 70)
    p = _params(shape, (0, 0, 0), 1, 1, which)
    phi0, c0 = wl.random_state_fields(shape, seed=3)
    sim = gp.Simulation(p, "fp64").init(phi0, c0).step(30)
    ref = oracle_mod.Oracle(p).init(phi0, c0).step(30)
    d, e = sim.diagnostics(), ref.diagnostics()
    for k in ("total_mass", "solid_fraction", "sum_phi"):
        assert abs(d[k] - e[k]) <= 1e-13 * max(abs(e[k]), 1.0), k
    for k in ("solid_fraction_count", "phi_min", "phi_max"):
        assert d[k] == e[k], k
