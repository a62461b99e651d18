"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each checks a printed value, a
closed-form solution, a conservation law or a special case that reduces to a
textbook problem.  The mutation test (test_oracle_mutations.py) shows that
each of a list of plausible slips in the oracle breaks at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import expit

import workloads as wl
from tests import analytic

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def golden():
    with open(GOLDEN) as f:
        return json.load(f)


# --------------------------------------------------------------------------
# Printed values: Stefan root, lambda*, Table 3


def test_stefan_root_matches_printed():
    g = golden()["stefan_dissolution"]
    a = analytic.stefan_alpha(g["mu_eq"], g["mu_inf"], g["c_s_co"] - g["c_l_co"])
    assert abs(a - g["alpha"]) < 0.6 * 10 ** (-g["printed_digits"])


def test_lambda_star_matches_printed():
    g = golden()["lambda_star_porous"]
    lam = wl.lambda_star(g["D_l"], g["M_phi"], g["dc"])
    assert round(lam) == g["lambda_star"]
    assert abs(lam - 230.2115) < 1e-3


def _tanh_phi(xi):
    # (1 + tanh(2 xi)) / 2 written as the logistic function of 4 xi, which
    # keeps full relative accuracy in both tails
    return expit(4.0 * xi)


def test_table3_integrals_by_quadrature():
    ln2 = math.log(2.0)
    dphi = lambda xi: 4.0 * _tanh_phi(xi) * (1.0 - _tanh_phi(xi))
    I = quad(lambda x: dphi(x) ** 2, -20, 20, epsabs=1e-14, epsrel=1e-14)[0]
    assert abs(I - 2.0 / 3.0) < 1e-12
    # (h - a dphi)/q with h = q = phi, a = 1/4 reduces to phi
    ratio = lambda x: (_tanh_phi(x) - 0.25 * dphi(x)) / _tanh_phi(x)
    F_l = quad(lambda x: 1.0 - ratio(x), 0, 20, epsabs=1e-14)[0]
    F_s = quad(lambda x: ratio(x), -20, 0, epsabs=1e-14)[0]
    assert abs(F_l - ln2 / 4) < 1e-12 and abs(F_s - ln2 / 4) < 1e-12
    p = lambda f: f * f * (3.0 - 2.0 * f)
    Ft_l = quad(lambda x: 1.0 - p(_tanh_phi(x)) / _tanh_phi(x), 0, 20, epsabs=1e-14)[0]
    Ft_s = quad(lambda x: p(_tanh_phi(x)) / _tanh_phi(x), -20, 0, epsabs=1e-14)[0]
    assert abs(Ft_l - (ln2 - 1) / 4) < 1e-12 and abs(Ft_s - (ln2 + 1) / 4) < 1e-12
    H_l = quad(lambda x: 1.0 - _tanh_phi(x), 0, 20, epsabs=1e-14)[0]
    assert abs(H_l - ln2 / 4) < 1e-12
    assert abs(wl.TABLE3_I - 2.0 / 3.0) < 1e-15
    assert abs(wl.TABLE3_F - ln2 / 4) < 1e-15


def test_table3_K_printed_vs_integrand():
    """K printed as (31 - 30 ln2)/150 reproduces the printed lambda* = 230, but
    quadrature of its defining integral gives 5/24 - ln2/4.  The printed value
    is used (it is the one the paper's own lambda* follows)."""
    ln2 = math.log(2.0)
    pprime_dphi = lambda x: 6.0 * _tanh_phi(x) * (1 - _tanh_phi(x)) * 4.0 * _tanh_phi(x) * (1 - _tanh_phi(x))
    inner = lambda x: quad(lambda s: _tanh_phi(s), 0.0, x, epsabs=1e-14)[0]
    K = quad(lambda x: pprime_dphi(x) * inner(x), -12, 12, epsabs=1e-13, limit=200)[0]
    assert abs(K - (5.0 / 24.0 - ln2 / 4.0)) < 1e-9
    assert abs(wl.TABLE3_K - (31 - 30 * ln2) / 150) < 1e-15
    assert abs(K - wl.TABLE3_K) > 0.03


# --------------------------------------------------------------------------
# General quadratic free energies (eps_s != eps_l)


def _quadratic(eps_s, eps_l, m_s, m_l, mu_star, **over):
    """Parameters for free_energy = 1 whose equilibrium chemical potential is
    mu_star: df_min chosen so that the grand potentials of the two phases are
    equal at mu_star (Eq. Egalite_grand-potentiel)."""
    df = (analytic.quad_omega(mu_star, eps_l, eps_s, eps_l, m_l, 0.0)
          - analytic.quad_omega(mu_star, eps_s, eps_s, eps_l, m_s, 0.0))
    p = wl.base_params(free_energy=1, eps_s=eps_s, eps_l=eps_l, m_s=m_s, m_l=m_l, df_min=df,
                       **over)
    cl = analytic.quad_composition(1.0, mu_star, eps_s, eps_l, m_s, m_l)
    cs = analytic.quad_composition(0.0, mu_star, eps_s, eps_l, m_s, m_l)
    p["lam"] = wl.lambda_star(p["D_l"], p["M_phi"], cs - cl)
    return p, cs, cl


@pytest.mark.parametrize("eps_s,eps_l", [(1.0, 2.0), (2.0, 1.0), (0.7, 3.1)])
def test_quadratic_local_forms(oracle_mod, eps_s, eps_l):
    """The oracle's closure, coupling bracket and anti-trapping jump against
    other statements of the paper: the closure inverts the composition of the
    mixture, Eq. (Composition_Quadratic); the bracket of S_phi is the reduced
    grand-potential difference omega_l - omega_s of Eq.
    (Quadratic_grand-potential_Liquid), i.e. Eq. (Dimensionless_OmegaL-OmegaS);
    the composition jump of j_at is the mu-derivative of that difference,
    Eq. (Anti-trapping_Current), which equals c_s(mu) - c_l(mu), the bulk
    compositions stated after Eq. (SourceTerm_Equilibrium)."""
    m_s, m_l, df = 0.83, 0.12, 0.031
    p = wl.base_params(free_energy=1, eps_s=eps_s, eps_l=eps_l, m_s=m_s, m_l=m_l, df_min=df)
    E = math.sqrt(eps_s * eps_l)
    for phi in (0.0, 0.13, 0.5, 0.91, 1.0):
        for mu in (-0.37, -0.05, 0.0, 0.08, 0.61):
            c = analytic.quad_composition(phi, mu, eps_s, eps_l, m_s, m_l)
            got_mu, bracket, jump = oracle_mod.local(p, phi, c, mu)
            assert abs(got_mu - mu) < 1e-14, (phi, mu, got_mu)
            om_l = analytic.quad_omega(mu, eps_l, eps_s, eps_l, m_l, 0.0)
            om_s = analytic.quad_omega(mu, eps_s, eps_s, eps_l, m_s, df)
            assert abs(bracket - (om_l - om_s)) < 1e-14
            d = 1e-5
            dw = ((analytic.quad_omega(mu + d, eps_l, eps_s, eps_l, m_l, 0.0)
                   - analytic.quad_omega(mu + d, eps_s, eps_s, eps_l, m_s, df))
                  - (analytic.quad_omega(mu - d, eps_l, eps_s, eps_l, m_l, 0.0)
                     - analytic.quad_omega(mu - d, eps_s, eps_s, eps_l, m_s, df))) / (2 * d)
            assert abs(jump - dw) < 1e-9
            cs_mu = mu * math.sqrt(eps_l / eps_s) + m_s
            cl_mu = mu * math.sqrt(eps_s / eps_l) + m_l
            assert abs(jump - (cs_mu - cl_mu)) < 1e-14
    assert abs(E - math.sqrt(eps_s * eps_l)) == 0.0


# --------------------------------------------------------------------------
# Closed-form solutions


@pytest.mark.parametrize("lattice,h_lattice,h_scheme",
                         [(0, 0, 0), (0, 1, 0), (0, 0, 1), (0, 1, 1), (2, 0, 0)])
def test_stefan_dissolution_front_and_profile(oracle_mod, lattice, h_lattice, h_scheme):
    """Workload 0 (planar dissolution, D_s = 0, anti-trapping, lambda*)
    against the one-sided Stefan solution of Sec. 4.2, with h on D2Q9 and
    on D2Q5, with the source H_k or with the flux folded into h^eq,alt
    (Eqs. LBE_Concent_Alt, Seq_Concent_Alt), and with g and h on D2Q5."""
    p, phi0, c0, nsteps = wl.config0()
    p = dict(p, lattice=lattice, h_lattice=h_lattice, h_scheme=h_scheme)
    mu_inf = p["mu_eq"] + 0.0 - p["c_l_co"]
    alpha = analytic.stefan_alpha(p["mu_eq"], mu_inf, p["c_s_co"] - p["c_l_co"])
    assert abs(alpha - (-0.0586022)) < 1e-6
    o = oracle_mod.Oracle(p).init(phi0, c0)
    x0 = analytic.front_position(o.fields()[0][0])
    assert abs(x0 - 100.0) < 1e-6
    for t in (1000, 2000, 3000, 4000):
        o.step(t - o.step_count)
        phi, c, mu = o.fields()
        dx = analytic.front_position(phi[0]) - x0
        exact = analytic.stefan_front(alpha, p["D_l"], t)
        assert abs(dx - exact) < 0.01 * abs(exact), (t, dx, exact)
    x = np.arange(512) - 100.0
    xi = analytic.stefan_front(alpha, p["D_l"], 4000)
    m = x > xi + 5
    mua = analytic.stefan_mu_liquid(x, 4000, alpha, p["D_l"], p["mu_eq"], mu_inf)
    err = np.linalg.norm(mu[0, 0][m] - mua[m]) / np.linalg.norm(mua[m])
    assert err < 2e-3
    # solid keeps its coexistence composition (D_s = 0)
    assert np.all(np.abs(c[0, :, :80] - p["c_s_co"]) < 1e-3)


@pytest.mark.parametrize("lattice,counter_term", [(0, 0), (0, 1), (2, 0), (2, 1)])
def test_circle_curvature_flow(oracle_mod, lattice, counter_term):
    """lambda = 0: without the counter term the grain follows mean-curvature
    flow R^2 = R0^2 - 2 M t (Eq. ModelA_EqPhi); with it the radius stays put
    (Eq. ModelA_EqPhi_CounterTerm)."""
    W, M = 6.0, 0.05
    p = wl.base_params(lattice=lattice, shape=(1, 128, 128), bc=(0, 0, 0),
                       counter_term=counter_term, lam=0.0, W=W)
    phi0, c0 = wl.disc(128, 128, 30.0, W, 1.0, 0.1)
    o = oracle_mod.Oracle(p).init(phi0, c0)
    o.step(400)
    A1 = (1 - o.fields()[0]).sum() / math.pi
    o.step(1600)
    A2 = (1 - o.fields()[0]).sum() / math.pi
    rate = (A1 - A2) / 1600
    if counter_term:
        assert abs(A1 - A2) / A1 < 1e-8
    else:
        assert abs(rate / (2 * M) - 1.0) < 0.03, rate


@pytest.mark.parametrize("lattice,h_lattice,axis", [
    (0, 0, 2), (0, 1, 2), (0, 1, 1), (1, 0, 0), (1, 1, 0), (1, 1, 2), (2, 0, 1), (3, 0, 0)])
def test_ade_fourier_mode_decay(oracle_mod, lattice, h_lattice, axis):
    """phi = 1 everywhere: the c-LBE reduces to the textbook advection-free
    diffusion LBM, so a Fourier mode of c decays as exp(-D_l k^2 t) -- on
    the full lattices and on the light ones (D2Q5, D3Q7, whose xi_s^2 = 1/4
    sets tau_h = 4 / gamma), along x, y and z (axis 2, 1, 0 of the array)."""
    L = 128
    shape = [1 if analytic.lattice_dim(lattice) == 2 else 2, 2, 2]
    shape[axis] = L
    shape = tuple(shape)
    p = wl.base_params(lattice=lattice, shape=shape, bc=(0, 0, 0), h_lattice=h_lattice)
    k = 2 * np.pi / L
    idx = [None, None, None]
    idx[axis] = slice(None)
    mode = np.cos(k * np.arange(L))[tuple(idx)]
    phi0 = np.ones(shape)
    c0 = p["c_l_co"] + 0.01 * np.broadcast_to(mode, shape)
    o = oracle_mod.Oracle(p).init(phi0, c0)
    o.step(100)

    def amp():
        line = np.moveaxis(o.fields()[1], axis, -1).reshape(-1, L)[0]
        return 2 * np.abs(np.fft.rfft(line)[1]) / L
    a0 = amp()
    o.step(2000)
    a1 = amp()
    rate = -math.log(a1 / a0) / 2000
    assert abs(rate / (p["D_l"] * k * k) - 1.0) < 2e-3, rate
    assert np.max(np.abs(o.fields()[0] - 1.0)) < 1e-15


@pytest.mark.parametrize("lattice,axis", [(0, 2), (2, 2), (2, 1), (1, 0), (3, 0), (3, 2)])
def test_phase_field_fourier_mode_decay(oracle_mod, lattice, axis):
    """lambda = 0, counter term on, phi a perturbation of amplitude 1e-9 about
    0: the counter term phi (1 - phi) n is of second order in the amplitude
    (|grad phi| << eps_n), so the phi-LBE reduces to the textbook diffusion
    LBM and a Fourier mode decays as exp(-M_phi k^2 t) -- on D2Q9, D3Q19 and
    on D2Q5 / D3Q7 (xi_s^2 = 1/4 sets tau_g = 4 M_phi), along x, y and z."""
    L = 128
    three = analytic.lattice_dim(lattice) == 3
    shape = [2 if three else 1, 2, 2]
    shape[axis] = L
    shape = tuple(shape)
    p = wl.base_params(lattice=lattice, shape=shape, bc=(0, 0, 0), lam=0.0, counter_term=1)
    k = 2 * np.pi / L
    idx = [None, None, None]
    idx[axis] = slice(None)
    phi0 = 1e-9 * np.broadcast_to(np.cos(k * np.arange(L))[tuple(idx)], shape)
    o = oracle_mod.Oracle(p).init(phi0, np.full(shape, p["c_l_co"]))
    o.step(100)

    def amp():
        line = np.moveaxis(o.fields()[0], axis, -1).reshape(-1, L)[0]
        return 2 * np.abs(np.fft.rfft(line)[1]) / L
    a0 = amp()
    o.step(2000)
    a1 = amp()
    rate = -math.log(a1 / a0) / 2000
    assert abs(rate / (p["M_phi"] * k * k) - 1.0) < 2e-3, rate


# --------------------------------------------------------------------------
# Conservation laws and special cases


@pytest.mark.parametrize("lattice,shape,bc,h_lattice,h_scheme", [
    (0, (1, 24, 40), (1, 0, 0), 0, 0),
    (0, (1, 24, 40), (1, 1, 0), 0, 0),
    (0, (1, 24, 40), (0, 0, 0), 0, 0),
    (1, (10, 12, 14), (1, 0, 1), 0, 0),
    (1, (10, 12, 14), (0, 0, 0), 0, 0),
    (0, (1, 24, 40), (1, 1, 0), 1, 0),
    (1, (10, 12, 14), (1, 0, 1), 1, 0),
    (0, (1, 24, 40), (1, 1, 0), 0, 1),
    (1, (10, 12, 14), (1, 0, 1), 1, 1),
    (2, (1, 24, 40), (1, 1, 0), 0, 0),
    (3, (10, 12, 14), (1, 0, 1), 0, 0),
    (3, (10, 12, 14), (0, 0, 0), 0, 1),
])
def test_solute_mass_conserved(oracle_mod, lattice, shape, bc, h_lattice, h_scheme):
    """sum_k h^eq_k = c (also for h^eq,alt), sum_k H_k = 0 and streaming
    permutes populations, so the total solute is conserved to round-off
    (Eq. Moment0_LBM_Concent)."""
    p = wl.base_params(lattice=lattice, shape=shape, bc=bc, h_lattice=h_lattice,
                       h_scheme=h_scheme)
    phi0, c0 = wl.random_state_fields(shape, seed=3)
    o = oracle_mod.Oracle(p).init(phi0, c0)
    m0 = o.diagnostics()["total_mass"]
    o.step(200)
    m1 = o.diagnostics()["total_mass"]
    assert abs(m1 - m0) / abs(m0) < 1e-12


@pytest.mark.parametrize("lattice,shape", [(0, (1, 32, 32)), (1, (12, 12, 12)),
                                           (2, (1, 32, 32)), (3, (12, 12, 12))])
def test_phase_conserved_without_coupling(oracle_mod, lattice, shape):
    """lambda = 0 with the counter term: the phi equation is conservative
    (Eq. ModelA_EqPhi_CounterTerm, divergence form), so sum phi is kept."""
    p = wl.base_params(lattice=lattice, shape=shape, bc=(0, 0, 0), lam=0.0)
    phi0, c0 = wl.random_state_fields(shape, seed=5)
    o = oracle_mod.Oracle(p).init(phi0, c0)
    s0 = o.diagnostics()["sum_phi"]
    o.step(300)
    s1 = o.diagnostics()["sum_phi"]
    assert abs(s1 - s0) / s0 < 1e-12


def test_pure_solid_is_stationary(oracle_mod):
    """phi = 0, D_s = 0: no diffusion, no source; the state does not move."""
    shape = (1, 16, 20)
    p = wl.base_params(shape=shape, bc=(1, 0, 0))
    phi0 = np.zeros(shape)
    c0 = 1.0 + 0.1 * np.random.default_rng(0).standard_normal(shape)
    o = oracle_mod.Oracle(p).init(phi0, c0)
    g0, h0, f0 = o.state()
    o.step(50)
    g1, h1, f1 = o.state()
    assert np.array_equal(g0, g1) and np.array_equal(h0, h1) and np.array_equal(f0, f1)


@pytest.mark.parametrize("lattice", [0, 1, 2, 3])
def test_gradient_exact_on_linear_field(oracle_mod, lattice):
    """Directional derivatives (Eq. DerivDirec_Grad) combined by Eq. (Grad)
    are exact for a linear field at interior nodes (on D2Q5 / D3Q7 they are
    central differences)."""
    three = analytic.lattice_dim(lattice) == 3
    shape = (7, 9, 11) if three else (1, 9, 11)
    p = wl.base_params(lattice=lattice, shape=shape, bc=(1, 1, 1 if three else 0))
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    b = (0.013, -0.021, 0.017 if three else 0.0)
    phi = 0.4 + b[0] * x + b[1] * y + b[2] * z
    o = oracle_mod.Oracle(p).init(phi, np.zeros(shape))
    g, n = o.gradient()
    inner = (slice(1, -1) if three else slice(None), slice(1, -1), slice(1, -1))
    for a in range(3):
        assert np.max(np.abs(g[inner][..., a] - b[a])) < 1e-14
    bn = np.array(b) / math.sqrt(sum(v * v for v in b) + p["eps_n"] ** 2)
    assert np.max(np.abs(n[inner] - bn)) < 1e-12


def test_planar_front_independent_of_y(oracle_mod):
    """Workload 0 is one-dimensional: every y row evolves identically."""
    p, phi0, c0, _ = wl.config0()
    o = oracle_mod.Oracle(p).init(phi0, c0)
    o.step(300)
    phi, c, mu = o.fields()
    for f in (phi, c, mu):
        assert np.all(f[0] == f[0, :1])


def test_counter_term_irrelevant_in_1d(oracle_mod):
    """Sec. 4: in one dimension both phi equations give the same solution."""
    xs = []
    for ct in (0, 1):
        p, phi0, c0, _ = wl.config0(counter_term=ct)
        o = oracle_mod.Oracle(p).init(phi0, c0)
        traj = []
        for _ in range(10):
            o.step(200)
            traj.append(analytic.front_position(o.fields()[0][0]))
        xs.append(np.array(traj))
    # 0.025 cells: about 1% of the distance the front travels by t = 4000
    assert np.max(np.abs(xs[0] - xs[1])) < 2.5e-2


def test_flat_front_at_equilibrium_is_stationary(oracle_mod):
    """c0 = c_co(phi0) puts mu = mu_eq everywhere: with the counter term a
    flat front does not move, apart from the slow relaxation of the sampled
    tanh profile to the discrete one (below 1e-2 cells and dying out, to
    compare with the 2.3 cells an undersaturated liquid drives it in 4000
    steps)."""
    p = wl.base_params(shape=(1, 4, 256), bc=(1, 0, 0))
    phi0, _ = wl.planar(256, 4, p["W"], 120.0, 1.0, 0.0)
    c0 = p["c_l_co"] * phi0 + p["c_s_co"] * (1 - phi0)
    o = oracle_mod.Oracle(p).init(phi0, c0)
    xs = []
    for _ in range(8):
        o.step(1000)
        xs.append(analytic.front_position(o.fields()[0][0]))
    xs = np.array(xs)
    drift = np.abs(np.diff(xs))
    assert np.max(np.abs(xs - 120.0)) < 1e-2
    assert np.all(np.diff(drift) < 0) and drift[-1] < 5e-4
    assert np.max(np.abs(o.fields()[2] - p["mu_eq"])) < 1e-3


def test_closed_box_reaches_equal_chemical_potentials(oracle_mod):
    """A closed box relaxes to mu = mu_eq in both phases (abstract, Sec. 5):
    liquid at c_l^co, solid at c_s^co, solid fraction by the lever rule."""
    n = 24
    p = wl.base_params(shape=(1, n, n), bc=(1, 1, 0), D_l=0.2)
    phi0, _ = wl.disc(n, n, 7.0, p["W"], 1.0, 0.0)
    c0 = p["c_s_co"] * (1 - phi0) + 0.05 * phi0
    o = oracle_mod.Oracle(p).init(phi0, c0)
    mtot = o.diagnostics()["total_mass"]
    errs = []
    for _ in range(6):
        o.step(4000)
        errs.append(np.max(np.abs(o.fields()[2] - p["mu_eq"])))
    assert errs[-1] < 1e-4 and errs[-1] < errs[0]
    phi, c, mu = o.fields()
    dc = p["c_s_co"] - p["c_l_co"]
    lever = (mtot / (n * n) - p["c_l_co"]) / dc
    assert abs(o.diagnostics()["solid_fraction"] - lever) < 1e-3


@pytest.mark.parametrize("lattice,counter_term", [(0, 0), (0, 1), (3, 1)])
def test_uniform_fields_follow_the_source_recurrence(oracle_mod, lattice, counter_term):
    """Uniform phi and c: no gradient, no normal, no flux, so c stays c0, and
    the phi-LBE collapses to a scalar recurrence.  Summing the BGK collision
    with the trapezoidal source over k, with sum g~ = phi - S_prev / 2 carried
    from the previous step (the variable change, and Eq. Moment_Phi closed
    with the source of the step's own collision), gives
        phi^{n+1} = phi^n + S^n + (1 - omega_g) / 2 (S^n - S^{n-1}),
    S^{-1} = S^0 (initial shift), omega_g = 1 / (3 M_phi + 1/2): explicit
    Euler of d phi / dt = S plus a second-order difference.  S is the zeroth
    moment of the sources (Eqs. SourceG_ST with SourceTerm_Coexistence, plus
    SourceG_dw without the counter term, whose own moment vanishes)."""
    shape = (1, 3, 4) if analytic.lattice_dim(lattice) == 2 else (3, 3, 4)
    p = wl.base_params(lattice=lattice, shape=shape, bc=(0, 0, 0), counter_term=counter_term)
    phi, c0 = 0.3, 0.5
    o = oracle_mod.Oracle(p).init(np.full(shape, phi), np.full(shape, c0))
    dc = p["c_s_co"] - p["c_l_co"]
    M, W = p["M_phi"], p["W"]
    omega = 1.0 / (M / analytic.lattice_cs2(lattice) + 0.5)

    def source(phi):
        mu = p["mu_eq"] + c0 - (p["c_l_co"] * phi + p["c_s_co"] * (1.0 - phi))
        S = -(p["lam"] * M / W ** 2) * 6.0 * phi * (1.0 - phi) * dc * (mu - p["mu_eq"])
        if not counter_term:
            S += -(8.0 * M / W ** 2) * 2.0 * phi * (1.0 - phi) * (1.0 - 2.0 * phi)
        return S

    steps = 30
    s_prev = source(phi)
    for _ in range(steps):
        S = source(phi)
        phi = phi + S + 0.5 * (1.0 - omega) * (S - s_prev)
        s_prev = S
    assert abs(phi - 0.3) > 0.1  # the source moves phi well away from its start
    o.step(steps)
    f, c, _ = o.fields()
    assert np.max(np.abs(f - phi)) < 1e-13
    assert np.max(np.abs(c - c0)) < 1e-14


@pytest.mark.parametrize("lattice,h_lattice,h_scheme",
                         [(0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0), (0, 0, 1), (1, 1, 1),
                          (2, 0, 0), (3, 0, 0)])
def test_wall_is_a_mirror_plane_for_wall_normal_fields(oracle_mod, lattice, h_lattice,
                                                       h_scheme):
    """For fields that vary only across a zero-flux wall, halfway bounce-back
    (the oblique populations that bounce and those that would mirror are
    equal by symmetry) and the mirror ghost of the gradient stencil make the
    wall a symmetry plane: the run on [0, n) between two walls equals the
    first half of the periodic run on [0, 2n) from the mirrored fields."""
    n = 24
    shape = (1, 4, n) if analytic.lattice_dim(lattice) == 2 else (2, 2, n)
    p = wl.base_params(lattice=lattice, shape=shape, bc=(1, 0, 0), h_lattice=h_lattice,
                       h_scheme=h_scheme)
    p2 = dict(p, shape=shape[:2] + (2 * n,), bc=(0, 0, 0))
    x = np.arange(n, dtype=np.float64)
    phi1 = wl.tanh_profile(x - 5.0, p["W"])          # front two cells off the wall
    c1 = 0.3 + 0.2 * np.cos(np.pi * x / n) - 0.25 * (1.0 - phi1)
    phi0 = np.broadcast_to(phi1, shape).copy()
    c0 = np.broadcast_to(c1, shape).copy()

    def mirrored(f):
        return np.concatenate([f, f[..., ::-1]], axis=-1)

    a = oracle_mod.Oracle(p).init(phi0, c0).step(80).fields()
    b = oracle_mod.Oracle(p2).init(mirrored(phi0), mirrored(c0)).step(80).fields()
    assert np.max(np.abs(a[0] - phi0)) > 1e-3        # the fields did move
    for fa, fb in zip(a, b):
        assert np.max(np.abs(fa - fb[..., :n])) < 1e-12


@pytest.mark.parametrize("lattice,h_lattice,h_scheme",
                         [(0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0), (0, 0, 1), (1, 1, 1),
                          (2, 0, 0), (3, 0, 0)])
def test_initial_populations_are_shifted_equilibria(oracle_mod, lattice, h_lattice, h_scheme):
    """Reading (the paper does not give the initial populations): at t = 0
    the populations before the variable change, g~ + G/2 and h~ + H/2, are
    the equilibria, with no anti-trapping current.  Checked by moments at
    the interior nodes of linear phi0 and c0, where the gradient is exact:
    sum g~ = phi0 - S/2, sum h~ = c0, and the first moments
    sum e_k g~_k = -(1/2) sum_k e_k G_k = -(1/6)(4/W) phi (1 - phi) n and
    sum e_k h~_k = -(1/2) sum_k e_k H_k = -(gamma/6) F with
    F = mu (D_l - D_s) grad phi (Eqs. SourceG_CT, SourceTerm_LBE_h; the
    second moment of the weights is 1/3).  With h^eq,alt there is no source
    and no shift: sum e_k h~_k is the first moment of h^eq,alt, which is F
    itself (Eq. Seq_Concent_Alt: w_k e_k . F / xi_s^2 summed with e_k)."""
    three = analytic.lattice_dim(lattice) == 3
    shape = (7, 9, 11) if three else (1, 9, 11)
    p = wl.base_params(lattice=lattice, shape=shape, bc=(1, 1, 1 if three else 0),
                       D_s=0.02, h_lattice=h_lattice, h_scheme=h_scheme)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    b = np.array([0.031, -0.023, 0.019 if three else 0.0])
    phi0 = 0.45 + b[0] * (x - 5) + b[1] * (y - 4) + b[2] * (z - 3 if three else 0)
    c0 = 0.35 - 0.02 * x + 0.015 * y
    o = oracle_mod.Oracle(p).init(phi0, c0)
    g, h, _ = o.state()
    inner = (slice(1, -1) if three else slice(None), slice(1, -1), slice(1, -1))
    dc = p["c_s_co"] - p["c_l_co"]
    M, W = p["M_phi"], p["W"]
    mu = p["mu_eq"] + c0 - (p["c_l_co"] * phi0 + p["c_s_co"] * (1.0 - phi0))
    Sst = -(p["lam"] * M / W ** 2) * 6.0 * phi0 * (1.0 - phi0) * dc * (mu - p["mu_eq"])
    nrm = b / math.sqrt(float(b @ b) + p["eps_n"] ** 2)
    kphi = (4.0 / W) * phi0 * (1.0 - phi0)
    F = (mu * (p["D_l"] - p["D_s"]))[..., None] * b
    assert np.max(np.abs(g.sum(0) - (phi0 - 0.5 * Sst))[inner]) < 1e-14
    assert np.max(np.abs(h.sum(0) - c0)[inner]) < 1e-14
    m1g = analytic.first_moment(g, lattice)
    m1h = analytic.first_moment(h, lattice, light=bool(h_lattice))
    cs2h = 0.25 if (lattice == 1 and h_lattice) else analytic.lattice_cs2(lattice)
    want_g = -(kphi * analytic.lattice_cs2(lattice) / 2.0)[..., None] * nrm
    want_h = F if h_scheme else -(p["gamma"] * cs2h / 2.0) * F
    assert np.max(np.abs(m1g - want_g)[inner]) < 1e-14
    assert np.max(np.abs(m1h - want_h)[inner]) < 1e-14
    assert np.max(np.abs(want_h[inner])) > 5e-4 and np.max(np.abs(want_g[inner])) > 1e-2


def test_maugis_root_matches_printed():
    """The two-sided (precipitation) transcendental equation of Sec. 4.2
    gives the printed root; the composition profiles then take the
    coexistence values on both sides of the interface and the far-field
    values away from it (the analytic helper used by the GPU validation)."""
    g = golden()["maugis_precipitation"]
    a = analytic.maugis_alpha(g["cs_inf"], g["cl_inf"], g["m_s"], g["m_l"], g["df_min"],
                              g["D_s"], g["D_l"])
    assert abs(a - g["alpha"]) < 0.6 * 10 ** (-g["printed_digits"])
    t = 5e-4
    xi = a * math.sqrt(t)
    c = analytic.maugis_composition([xi - 1e-12, xi + 1e-12, -0.25, 0.25], t, a, g["cs_inf"],
                                    g["cl_inf"], 0.6, 0.5, g["D_s"], g["D_l"])
    assert abs(c[0] - 0.6) < 1e-9 and abs(c[1] - 0.5) < 1e-9
    assert abs(c[2] - g["cs_inf"]) < 1e-9 and abs(c[3] - g["cl_inf"]) < 1e-9


# --------------------------------------------------------------------------
# General quadratic free energies: runs


def test_quadratic_reduces_to_equal_curvature(oracle_mod):
    """eps_s = eps_l: the general closure, source and anti-trapping current
    are the equal-curvature ones once m_phi = c_phi^co - mu_eq and
    df_min = mu_eq (m_s - m_l) (Eqs. Equilibrium_Potchem, Cl_coexistence,
    Cs_coexistence); the runs agree to round-off."""
    shape = (1, 20, 30)
    base = wl.base_params(shape=shape, bc=(1, 0, 0), mu_eq=0.07, D_s=0.01)
    m_s, m_l = base["c_s_co"] - base["mu_eq"], base["c_l_co"] - base["mu_eq"]
    gen = dict(base, free_energy=1, eps_s=1.7, eps_l=1.7, m_s=m_s, m_l=m_l,
               df_min=base["mu_eq"] * (m_s - m_l))
    phi0, c0 = wl.random_state_fields(shape, seed=12)
    a = oracle_mod.Oracle(base).init(phi0, c0).step(200).fields()
    b = oracle_mod.Oracle(gen).init(phi0, c0).step(200).fields()
    assert np.max(np.abs(a[0] - phi0)) > 1e-2
    for fa, fb in zip(a, b):
        assert np.max(np.abs(fa - fb)) < 1e-12


@pytest.mark.parametrize("eps_s,eps_l", [(1.0, 2.0), (2.0, 1.0)])
def test_quadratic_closed_box_equilibrium(oracle_mod, eps_s, eps_l):
    """A closed box with eps_s != eps_l relaxes to the common-tangent state:
    mu = mu_eq everywhere, the root of omega_l(mu) = omega_s(mu) (here 0.05,
    chosen through df_min), and at every node the composition of the mixture
    at that mu, Eq. (Composition_Quadratic); that composition is linear in
    phi, so the solid fraction mean(1 - phi) follows the lever rule between
    c_l(mu_eq) and c_s(mu_eq) exactly.  D_s = D_l: with D' = 0 the scheme's
    split of the flux (grad^2(D mu) and mu D' grad phi, which do not cancel
    exactly for a uniform mu != 0 at a curved, 2.5-cell interface) is out of
    the way, and the equilibrium is reached to round-off."""
    n = 24
    p, cs, cl = _quadratic(eps_s, eps_l, 0.9, 0.1, 0.05, shape=(1, n, n), bc=(1, 1, 0),
                           D_l=0.2, D_s=0.2)
    mu_star = analytic.quad_mu_eq(eps_s, eps_l, 0.9, 0.1, p["df_min"], near=0.05)
    assert abs(mu_star - 0.05) < 1e-12
    phi0, _ = wl.disc(n, n, 7.0, p["W"], 1.0, 0.0)
    c0 = cs * (1 - phi0) + 0.05 * phi0
    o = oracle_mod.Oracle(p).init(phi0, c0)
    mtot = o.diagnostics()["total_mass"]
    errs = []
    for _ in range(6):
        o.step(4000)
        errs.append(np.max(np.abs(o.fields()[2] - mu_star)))
    assert errs[-1] < 1e-12 and errs[0] > 1e-8
    phi, c, mu = o.fields()
    want = analytic.quad_composition(phi, mu_star, eps_s, eps_l, 0.9, 0.1)
    assert np.max(np.abs(c - want)) < 1e-12
    assert np.max(phi) - np.min(phi) > 0.99  # a grain is still there
    lever = (mtot / (n * n) - cl) / (cs - cl)
    assert abs(o.diagnostics()["solid_fraction"] - lever) < 1e-12


@pytest.mark.parametrize("eps_s,eps_l", [(1.0, 2.0), (2.0, 1.0)])
def test_quadratic_stefan_front(oracle_mod, eps_s, eps_l):
    """Planar dissolution with eps_s != eps_l, D_s = 0 and anti-trapping:
    in the liquid c = c_l(mu) = mu sqrt(eps_s / eps_l) + m_l, so c obeys
    the diffusion equation with D_c = D_l / sqrt(eps_s / eps_l) (Eq.
    Mixed-Formulation), and the front follows the one-sided Stefan solution
    of Sec. 4.2 in composition units with D_c, the interface at the
    equilibrium compositions.  The equilibrium chemical potential is taken
    0 (df_min = 0): at a 2.5-cell interface the scheme's split of the flux
    into grad^2(D mu) and mu D' grad phi carries an error proportional to mu
    at the interface (a few percent on the front at mu_eq = 0.05 with equal
    curvatures as well)."""
    p, cs, cl = _quadratic(eps_s, eps_l, 1.0, 0.1, 0.0, lattice=0, shape=(1, 2, 512),
                           bc=(1, 0, 0))
    assert p["df_min"] == 0.0 and abs(cs - 1.0) < 1e-15 and abs(cl - 0.1) < 1e-15
    phi0, c0 = wl.planar(512, 2, p["W"], 100.0, cs, 0.0)
    kl = math.sqrt(eps_s / eps_l)
    Dc = p["D_l"] / kl
    alpha = analytic.stefan_alpha(cl, 0.0, cs - cl)
    o = oracle_mod.Oracle(p).init(phi0, c0)
    x0 = analytic.front_position(o.fields()[0][0])
    for t in (1000, 2000, 3000, 4000):
        o.step(t - o.step_count)
        dx = analytic.front_position(o.fields()[0][0]) - x0
        exact = analytic.stefan_front(alpha, Dc, t)
        assert abs(dx - exact) < 0.01 * abs(exact), (t, dx, exact)
    phi, c, mu = o.fields()
    x = np.arange(512) - 100.0
    m = x > analytic.stefan_front(alpha, Dc, 4000) + 5
    ca = analytic.stefan_mu_liquid(x, 4000, alpha, Dc, cl, 0.0)
    mua = (ca - 0.1) / kl
    assert np.linalg.norm(mu[0, 0][m] - mua[m]) / np.linalg.norm(mua[m]) < 2e-3
    assert np.all(np.abs(c[0, :, :80] - cs) < 1e-3)


# --------------------------------------------------------------------------
# Interpolation functions on [0, 1] (p' of S_phi, q of D)


@pytest.mark.parametrize("lattice", [0, 1])
@pytest.mark.parametrize("phi_u,c_u", [(-0.01, 0.0), (1.01, 1.0)])
def test_overshoot_is_not_driven_further(oracle_mod, lattice, phi_u, c_u):
    """A uniform phase field just outside [0, 1] (solid side undersaturated,
    liquid side supersaturated) with the counter term stays where it is, to
    the rounding of the weight sums: no gradient, so no counter term and no
    flux, and the coupling source vanishes because p'(phi) is the derivative
    of an interpolation function on [0, 1].  The unlimited 6 phi (1 - phi)
    has there the sign that drives phi further out of the range (by ~3e-3
    per step here)."""
    shape = (1, 6, 8) if lattice == 0 else (4, 5, 6)
    p = wl.base_params(lattice=lattice, shape=shape, bc=(0, 0, 0), counter_term=1)
    o = oracle_mod.Oracle(p).init(np.full(shape, phi_u), np.full(shape, c_u))
    phi0, c0, _ = o.fields()
    o.step(200)
    phi1, c1, _ = o.fields()
    assert np.max(np.abs(phi1 - phi0)) < 1e-13
    assert np.max(np.abs(c1 - c0)) < 1e-13


@pytest.mark.parametrize("lattice", [0, 1])
def test_no_diffusion_in_overshooting_solid(oracle_mod, lattice):
    """phi = -0.01 everywhere with D_s = 0: the diffusivity D_l q + D_s (1 - q)
    with q limited to [0, 1] is 0, so a composition mode does not move (the
    unlimited q would give D = -1e-3, an anti-diffusion that amplifies it)."""
    L = 32
    shape = (1, 2, L) if lattice == 0 else (2, 2, L)
    p = wl.base_params(lattice=lattice, shape=shape, bc=(0, 0, 0), counter_term=1)
    phi0 = np.full(shape, -0.01)
    c0 = (1.0 + 0.01 * np.cos(2 * np.pi * np.arange(L) / L))[None, None, :] + 0.0 * phi0
    o = oracle_mod.Oracle(p).init(phi0, c0)
    _, ca, _ = o.fields()
    o.step(400)
    _, cb, _ = o.fields()
    assert np.max(np.abs(cb - ca)) < 1e-14


def test_liquid_overshoot_diffuses_at_D_l(oracle_mod):
    """phi = 1.02 everywhere: q limited to 1, so a composition mode decays at
    exp(-D_l k^2 t) as in the liquid (the unlimited q = 1.02 would decay 2%
    faster)."""
    L = 128
    shape = (1, 2, L)
    p = wl.base_params(lattice=0, shape=shape, bc=(0, 0, 0))
    k = 2 * np.pi / L
    phi0 = np.full(shape, 1.02)
    c0 = (p["c_l_co"] + 0.01 * np.cos(k * np.arange(L)))[None, None, :] + 0.0 * phi0
    o = oracle_mod.Oracle(p).init(phi0, c0)
    o.step(100)

    def amp():
        line = o.fields()[1][0, 0]
        return 2 * np.abs(np.fft.rfft(line)[1]) / L
    a0 = amp()
    o.step(2000)
    rate = -math.log(amp() / a0) / 2000
    assert abs(rate / (p["D_l"] * k * k) - 1.0) < 2e-3, rate
    assert np.max(np.abs(o.fields()[0] - 1.02)) < 1e-13


# --------------------------------------------------------------------------
# Diagnostics on hand-computed fixtures


@pytest.mark.parametrize("lattice", [0, 1])
def test_diagnostics_hand_computed_fixture(oracle_mod, lattice):
    """The reported quantities at time 0, where phi^0 = phi0 and c^0 equals
    c0 up to the rounding of the equilibrium sums (the shifted equilibria
    of the initial populations sum to c0, Eq. Heq_Composition, and the
    source moments vanish): twelve phi0 values chosen by hand, dyadic so
    that every sum below is exact.

      phi0 = 0, 1/4, 1/2, 3/4, 1, 1/8, 7/8, 1/2 - 2^-20, 3/8, 5/8, 1/16, 1
      phi < 1/2 (strictly): 0, 1/4, 1/8, 1/2 - 2^-20, 3/8, 1/16  -> 6 of 12
      sum phi = 0 + 1/4 + 1/2 + 3/4 + 1 + 1/8 + 7/8 + (1/2 - 2^-20) + 3/8
        + 5/8 + 1/16 + 1 = 97/16 - 2^-20
      mean (1 - phi) = (12 - 97/16 + 2^-20) / 12 = (95/16 + 2^-20) / 12
      min 0, max 1; c0 = 1/2 + phi0 / 4 sums to 6 + (97/16 - 2^-20) / 4
    """
    vals = np.array([0.0, 0.25, 0.5, 0.75, 1.0, 0.125, 0.875, 0.5 - 2.0 ** -20,
                     0.375, 0.625, 0.0625, 1.0])
    shape = (1, 3, 4) if lattice == 0 else (3, 2, 2)
    p = wl.base_params(lattice=lattice, shape=shape, bc=(0, 0, 0))
    phi0 = vals.reshape(shape)
    c0 = 0.5 + 0.25 * phi0
    d = oracle_mod.Oracle(p).init(phi0, c0).diagnostics()
    assert d["step"] == 0 and not d["nonfinite"]
    assert d["solid_fraction_count"] == 6.0 / 12.0
    assert d["phi_min"] == 0.0 and d["phi_max"] == 1.0
    assert d["sum_phi"] == 97.0 / 16.0 - 2.0 ** -20
    assert d["solid_fraction"] == (95.0 / 16.0 + 2.0 ** -20) / 12.0
    assert abs(d["total_mass"] - (6.0 + (97.0 / 16.0 - 2.0 ** -20) / 4.0)) < 1e-14


def test_diagnostics_after_steps_and_nonfinite(oracle_mod):
    """Pure liquid (phi = 1) with uniform c is stationary up to the rounding
    of the weight sums: after 5 steps the diagnostics report step 5, no node
    below 1/2, solid fraction 0, min = max = 1, the N values of phi and the
    solute N c (to 1e-15 per node).  A NaN in phi0 or an infinite c0 raises
    the non-finite flag."""
    shape = (4, 3, 5)
    N = 60
    p = wl.base_params(lattice=1, shape=shape, bc=(1, 0, 1))
    o = oracle_mod.Oracle(p).init(np.ones(shape), np.full(shape, 0.125)).step(5)
    d = o.diagnostics()
    assert d["step"] == 5 and not d["nonfinite"]
    assert d["solid_fraction_count"] == 0.0 and abs(d["solid_fraction"]) < 1e-15
    assert abs(d["phi_min"] - 1.0) < 1e-15 and abs(d["phi_max"] - 1.0) < 1e-15
    assert d["phi_min"] <= d["phi_max"]
    assert abs(d["sum_phi"] - N) < N * 1e-15
    assert abs(d["total_mass"] - 0.125 * N) < N * 1e-15
    phi0 = np.full(shape, 0.5)
    phi0[1, 2, 3] = np.nan
    assert oracle_mod.Oracle(p).init(phi0, np.zeros(shape)).diagnostics()["nonfinite"]
    c0 = np.zeros(shape)
    c0[3, 0, 0] = np.inf
    assert oracle_mod.Oracle(p).init(np.full(shape, 0.5), c0).diagnostics()["nonfinite"]


# --------------------------------------------------------------------------
# Three-dimensional curvature flow (last: the slowest pins)


@pytest.mark.parametrize("lattice", [1, 3])
def test_sphere_curvature_flow(oracle_mod, lattice):
    """lambda = 0, no counter term, in 3-D on D3Q19 and D3Q7: a solid sphere
    follows mean-curvature flow, dR/dt = -2 M / R, i.e. R^2 = R0^2 - 4 M t
    (Eq. ModelA_EqPhi in three dimensions), with the radius taken from the
    solid volume sum(1 - phi).  The bar, 10%, covers the diffuse-interface
    correction at W / R = 1/4 ... 1/3 (7.7% on D3Q19, 3.6% on D3Q7
    measured); a wrong xi_s^2 in tau_g would be off by a third."""
    n, R0, W = 36, 12.0, 3.0
    p = wl.base_params(lattice=lattice, shape=(n, n, n), bc=(0, 0, 0), counter_term=0,
                       lam=0.0, W=W)
    phi0, c0 = wl.sphere(n, R0, W, 1.0, 0.1)
    o = oracle_mod.Oracle(p).init(phi0, c0)
    o.step(60)
    V1 = (1 - o.fields()[0]).sum()
    o.step(300)
    V2 = (1 - o.fields()[0]).sum()
    R1, R2 = (3 * V1 / (4 * math.pi)) ** (1 / 3), (3 * V2 / (4 * math.pi)) ** (1 / 3)
    rate = (R1 * R1 - R2 * R2) / 300
    assert R2 < R1 - 2.5
    assert abs(rate / (4 * p["M_phi"]) - 1.0) < 0.10, rate
