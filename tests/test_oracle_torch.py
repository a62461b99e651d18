"""Pins of the oracle adjoint (the PyTorch-CPU restatement of the step,
differentiated by autograd): its forward equals the C oracle, and its
gradients equal central finite differences of that forward."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import torch_step as ts

# general quadratic free energies for the variant cases: eps_l / eps_s = 2.3
QUAD = dict(free_energy=1, eps_s=1.0, eps_l=2.3, m_s=0.9, m_l=0.12, df_min=0.02)


def _variant(v):
    """h_lattice as an int, or a variant name: alt (h^eq,alt), quad, alt+quad."""
    if not isinstance(v, str):
        return {"h_lattice": v}
    over = {}
    if "alt" in v:
        over["h_scheme"] = 1
    if "quad" in v:
        over.update(QUAD)
    return over


@pytest.mark.parametrize("lattice,shape,bc,ct,at,hl", [
    (0, (1, 20, 30), (1, 0, 0), 1, 1, 0),
    (0, (1, 17, 23), (0, 0, 0), 0, 1, 0),
    (0, (1, 12, 14), (1, 1, 0), 1, 0, 0),
    (1, (8, 9, 10), (1, 0, 1), 1, 1, 0),
    (1, (7, 8, 9), (0, 0, 0), 0, 0, 0),
    (0, (1, 20, 30), (1, 0, 0), 1, 1, 1),
    (1, (8, 9, 10), (1, 0, 1), 1, 1, 1),
    (2, (1, 17, 23), (1, 1, 0), 1, 1, 0),
    (3, (8, 9, 10), (0, 1, 0), 0, 1, 0),
    (0, (1, 20, 30), (1, 0, 0), 1, 1, "alt"),
    (1, (8, 9, 10), (0, 0, 1), 1, 1, "quad"),
    (0, (1, 17, 23), (0, 1, 0), 0, 1, "alt+quad"),
])
def test_torch_restatement_equals_c_oracle(oracle_mod, lattice, shape, bc, ct, at, hl):
    """Also with h on D2Q5 / D3Q7 (hl = 1), with g and h on them (lattice 2,
    3), with h^eq,alt and with general quadratic free energies."""
    p = wl.base_params(lattice=lattice, shape=shape, bc=bc, counter_term=ct, anti_trapping=at,
                       **_variant(hl))
    phi0, c0 = wl.random_state_fields(shape, seed=4)
    o = oracle_mod.Oracle(p).init(phi0, c0).step(25)
    phiK, cK = ts.run(p, torch.from_numpy(phi0.ravel()), torch.from_numpy(c0.ravel()), 25)
    phi, c, _ = o.fields()
    assert np.max(np.abs(phiK.numpy() - phi.ravel())) < 1e-13
    assert np.max(np.abs(cK.numpy() - c.ravel())) < 1e-13


@pytest.mark.parametrize("lattice,shape,bc,hl", [(0, (1, 14, 16), (1, 0, 0), 0),
                                                (1, (6, 7, 8), (0, 0, 0), 0),
                                                (1, (6, 7, 8), (1, 0, 0), 1),
                                                (3, (6, 7, 8), (0, 0, 1), 0),
                                                (0, (1, 14, 16), (1, 0, 0), "alt+quad")])
def test_torch_adjoint_matches_finite_differences(lattice, shape, bc, hl):
    p = wl.base_params(lattice=lattice, shape=shape, bc=bc, **_variant(hl))
    phi0, c0 = wl.random_state_fields(shape, seed=8)
    K = 10
    t_lam = torch.tensor(p["lam"], dtype=torch.float64, requires_grad=True)
    t_dl = torch.tensor(p["D_l"], dtype=torch.float64, requires_grad=True)
    t_phi0 = torch.tensor(phi0.ravel(), requires_grad=True)
    c0t = torch.from_numpy(c0.ravel())
    phiK, _ = ts.run(p, t_phi0, c0t, K, lam=t_lam, D_l=t_dl)
    J = ts.objectives(p, t_phi0, phiK)[1]
    J.backward()
    # the phi0 direction of the differentiation workload: seeded noise times
    # 4 phi0 (1 - phi0), which vanishes where phi0 is exactly 0 or 1 -- there
    # the map has a kink (p' and q take phi limited to [0, 1]) and a central
    # difference does not measure a derivative
    base = phi0.ravel()
    v = np.random.default_rng(9).standard_normal(phi0.size) * 4.0 * base * (1.0 - base)

    def J2(lam, dl, ph):
        with torch.no_grad():
            ph = torch.from_numpy(ph)
            out, _ = ts.run(p, ph, c0t, K, lam=torch.tensor(lam, dtype=torch.float64),
                            D_l=torch.tensor(dl, dtype=torch.float64))
            return ts.objectives(p, ph, out)[1].item()

    h = 1e-6
    base = phi0.ravel()
    fd_lam = (J2(p["lam"] + h, p["D_l"], base) - J2(p["lam"] - h, p["D_l"], base)) / (2 * h)
    fd_dl = (J2(p["lam"], p["D_l"] + h, base) - J2(p["lam"], p["D_l"] - h, base)) / (2 * h)
    fd_v = (J2(p["lam"], p["D_l"], base + h * v) - J2(p["lam"], p["D_l"], base - h * v)) / (2 * h)
    assert abs(t_lam.grad.item() - fd_lam) <= 1e-6 * abs(fd_lam)
    assert abs(t_dl.grad.item() - fd_dl) <= 1e-6 * abs(fd_dl)
    assert abs(float((t_phi0.grad.numpy() * v).sum()) - fd_v) <= 1e-6 * abs(fd_v)
