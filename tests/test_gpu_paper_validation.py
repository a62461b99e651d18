"""The paper's one-dimensional validation runs at its own parameters
(Sec. 4.2: 5000 x 36 D2Q9 nodes, dx = 1e-4, dt = 5e-9, up to 1e5 steps), on
the GPU in FP64, against the analytic solutions, with the relative L2 errors
compared to the ones the paper prints for its own runs:

- dissolution, D_s = 0, anti-trapping, W = 50 cells, lambda* = 230: the
  liquid chemical potential against the one-sided Stefan solution (Eqs.
  x_i_Ds0, Analytical_muL_Ds0) over the liquid x_i(t) < x <= L_x at
  t = 5e-5, 2.5e-4, 5e-4 (printed: 1.6e-3, 7.2e-4, 5.4e-4);
- precipitation, D_s = 0.9, D_l = 1, no anti-trapping, W = 12 cells,
  lambda* = 277: the compositions against the two-sided solution (Eqs.
  x_i_Ds-Dl, Compos_Solid, Compos_Liq) over [-0.04, 0.04] at t = 2.5e-5 and
  5e-4 (printed: 4.8e-3 at both).

The errors depend on the reading of the paper's unstated details (the
regularisation eps_n, gamma, the initial populations, the plotted range of
the error norm), so the bar is the printed error times 2.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as wl
from tests import analytic

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


@pytest.fixture(scope="module")
def gp():
    import torch
    assert torch.cuda.is_available()
    from paper_2111_05960_amd import binding
    binding.load()
    return binding


def _l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_dissolution_with_anti_trapping_at_paper_parameters(gp):
    g = json.load(open(GOLDEN))["dissolution_validation"]
    p, phi0, c0 = wl.paper_validation("dissolution")
    alpha = analytic.stefan_alpha(g["mu_eq"], g["mu_inf"], p["c_s_co"] - p["c_l_co"])
    x = wl.paper_x()
    sim = gp.Simulation(p, "fp64").init(phi0, c0)
    n = 0
    errs = []
    for t, printed in zip(g["t"], g["L2_mu"]):
        steps = int(round(t / wl.PAPER_DT))
        print(f"case dissolution t={t} steps={steps}", flush=True)
        sim.step(steps - n)
        n = steps
        phi, c, mu = sim.fields()
        mu1 = mu[0].mean(axis=0)
        xi = analytic.stefan_front(alpha, g["D_l"], t)
        m = x > xi
        ref = analytic.stefan_mu_liquid(x[m], t, alpha, g["D_l"], g["mu_eq"], g["mu_inf"])
        e = _l2(mu1[m], ref)
        xf = -0.25 + (1.0 - phi[0]).sum(axis=-1).mean() * wl.PAPER_DX
        print(f"  L2(mu_l) = {e:.3e} (printed {printed:.1e}); front {xf:.6e} "
              f"analytic {xi:.6e}", flush=True)
        errs.append((e, printed))
    for e, printed in errs:
        assert e <= 2.0 * printed


def test_precipitation_two_sided_at_paper_parameters(gp):
    g = json.load(open(GOLDEN))["maugis_precipitation"]
    p, phi0, c0 = wl.paper_validation("precipitation")
    alpha = analytic.maugis_alpha(g["cs_inf"], g["cl_inf"], g["m_s"], g["m_l"], g["df_min"],
                                  g["D_s"], g["D_l"])
    x = wl.paper_x()
    m = np.abs(x) <= 0.04
    sim = gp.Simulation(p, "fp64").init(phi0, c0)
    n = 0
    errs = []
    for t, printed in zip(g["t"], g["L2_c"]):
        steps = int(round(t / wl.PAPER_DT))
        print(f"case precipitation t={t} steps={steps}", flush=True)
        sim.step(steps - n)
        n = steps
        phi, c, mu = sim.fields()
        c1 = c[0].mean(axis=0)
        ref = analytic.maugis_composition(x[m], t, alpha, g["cs_inf"], g["cl_inf"], 0.6, 0.5,
                                          g["D_s"], g["D_l"])
        e = _l2(c1[m], ref)
        xf = -0.25 + (1.0 - phi[0]).sum(axis=-1).mean() * wl.PAPER_DX
        print(f"  L2(c) = {e:.3e} (printed {printed:.1e}); front {xf:.6e} "
              f"analytic {alpha * math.sqrt(t):.6e}", flush=True)
        errs.append((e, printed))
    for e, printed in errs:
        assert e <= 2.0 * printed
