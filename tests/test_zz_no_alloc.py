"""The allocation-free diagnostics entry point (gplbm_diagnostics_noalloc)
against gplbm_diagnostics, through the C ABI: bit-identical values on two
calls in a row, the second on a smaller grid (the static reduction array keeps
the first call's contents), for an FP64, an FP32 and an FP16-deviation
context, 2-D and 3-D."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

KEYS = ("step", "total_mass", "solid_fraction", "solid_fraction_count", "sum_phi",
        "phi_min", "phi_max", "nonfinite")


@pytest.fixture(scope="module")
def gp():
    import torch
    assert torch.cuda.is_available()
    from paper_2111_05960_amd import binding
    binding.load()
    return binding


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16dev"])
def test_noalloc_diagnostics_equal_the_buffered_ones(gp, prec):
    cases = [((24, 40, 70), wl.D3Q19, (0, 1, 0), 9), ((1, 30, 50), wl.D2Q9, (1, 0, 0), 4)]
    for shape, lattice, bc, steps in cases:
        print(f"case prec={prec} shape={shape} lattice={lattice} bc={bc} steps={steps}",
              flush=True)
        p = wl.base_params(lattice=lattice, shape=shape, bc=bc)
        phi0, c0 = wl.random_state_fields(shape, seed=sum(shape))
        sim = gp.Simulation(p, prec).init(phi0, c0).step(steps)
        a = gp.gplbm_diagnostics_noalloc(sim.ctx)
        b = gp.gplbm_diagnostics(sim.ctx)
        print("  noalloc", a, flush=True)
        for k in KEYS:
            assert a[k] == b[k], (k, a[k], b[k])
        assert a["step"] == steps


def test_noalloc_diagnostics_flag_nonfinite(gp):
    shape = (1, 16, 16)
    p = wl.base_params(shape=shape, bc=(0, 0, 0))
    phi0, c0 = wl.random_state_fields(shape, seed=2)
    phi0[0, 3, 5] = np.nan
    sim = gp.Simulation(p, "fp64").init(phi0, c0)
    with pytest.raises(gp.GplbmError) as e:
        gp.gplbm_diagnostics_noalloc(sim.ctx)
    assert e.value.code == gp.GPLBM_E_NONFINITE
    assert gp.gplbm_diagnostics_noalloc(sim.ctx, allow_nonfinite=True)["nonfinite"]
