"""Closed-form solutions used to pin the oracle (independent of it).

One-sided Stefan problem (D_s = 0) of Sec. 4.2 of the paper, with the
chemical potential playing the role of the temperature:
  transcendental equation, Eq. (Cartesian_Transcendental):
      alpha exp(alpha^2) erfc(alpha) + (mu_eq - mu_inf) / (dc sqrt(pi)) = 0
  interface position, Eq. (x_i_Ds0):  x_i(t) = 2 alpha sqrt(D_l t)
  liquid chemical potential, Eq. (Analytical_muL_Ds0):
      mu_l(x, t) = mu_inf + (mu_eq - mu_inf) erfc(x / (2 sqrt(D_l t))) / erfc(alpha)
"""
import math

import numpy as np
from scipy.optimize import brentq
from scipy.special import erfc


def stefan_alpha(mu_eq: float, mu_inf: float, dc: float) -> float:
    rhs = (mu_eq - mu_inf) / (dc * math.sqrt(math.pi))
    f = lambda a: a * math.exp(a * a) * math.erfc(a) + rhs
    return brentq(f, -5.0, 5.0, xtol=1e-15, rtol=1e-15)


def stefan_front(alpha: float, D_l: float, t):
    return 2.0 * alpha * np.sqrt(D_l * np.asarray(t, dtype=np.float64))


def stefan_mu_liquid(x, t, alpha, D_l, mu_eq, mu_inf):
    x = np.asarray(x, dtype=np.float64)
    return mu_inf + (mu_eq - mu_inf) * erfc(x / (2.0 * math.sqrt(D_l * t))) / erfc(alpha)


def maugis_u(a: float, D: float) -> float:
    """u_Phi(alpha) of the two-sided solution (Sec. 4.2, Eq. solution_u)."""
    return math.sqrt(D / math.pi) * math.exp(-a * a / (4.0 * D)) / math.erfc(a / (2.0 * math.sqrt(D)))


def maugis_alpha(cs_inf, cl_inf, m_s, m_l, df_min, D_s, D_l) -> float:
    """Root of the binary transcendental equation of the two-sided diffusion
    problem (Sec. 4.2, Eq. Transcendental_Eq), with dm = m_s - m_l:
    -alpha dm^2 / 2 = df_min [u_s(-alpha) + u_l(alpha)]
                      + dm [(m_s - cs_inf) u_s(-alpha) + (m_l - cl_inf) u_l(alpha)]."""
    dm = m_s - m_l

    def f(a):
        us, ul = maugis_u(-a, D_s), maugis_u(a, D_l)
        return 0.5 * a * dm * dm + df_min * (us + ul) + dm * ((m_s - cs_inf) * us + (m_l - cl_inf) * ul)
    return brentq(f, -2.0, 2.0, xtol=1e-15, rtol=1e-15)


def maugis_composition(x, t, alpha, cs_inf, cl_inf, cs_co, cl_co, D_s, D_l):
    """Compositions of the two-sided solution (Eqs. x_i_Ds-Dl, Compos_Solid,
    Compos_Liq): solid for x < alpha sqrt(t), liquid beyond."""
    x = np.asarray(x, dtype=np.float64)
    xi = alpha * math.sqrt(t)
    cs = cs_inf + (cs_co - cs_inf) * erfc(-x / (2.0 * math.sqrt(D_s * t))) / erfc(-alpha / (2.0 * math.sqrt(D_s)))
    cl = cl_inf + (cl_co - cl_inf) * erfc(x / (2.0 * math.sqrt(D_l * t))) / erfc(alpha / (2.0 * math.sqrt(D_l)))
    return np.where(x < xi, cs, cl)


def front_position(phi):
    """Interface position of a planar front with solid on the left and the
    zero-flux wall at x = -1/2: -1/2 + mean over y of sum_x (1 - phi)."""
    phi = np.asarray(phi)
    return -0.5 + (1.0 - phi).sum(axis=-1).mean()


# Velocity sets in the population order of the oracle's state arrays: D2Q9 in
# the paper's numbering (Sec. 3.1); D3Q19 grouped by e_z (+1, 0, -1), the
# convention of this project (the paper does not number D3Q19).
D2Q9_E = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0],
                   [1, 1, 0], [-1, 1, 0], [-1, -1, 0], [1, -1, 0]], dtype=np.float64)
D3Q19_E = np.array([[0, 0, 1], [1, 0, 1], [-1, 0, 1], [0, 1, 1], [0, -1, 1],
                    [0, 0, 0],
                    [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0],
                    [1, 1, 0], [-1, 1, 0], [-1, -1, 0], [1, -1, 0],
                    [0, 0, -1], [-1, 0, -1], [1, 0, -1], [0, -1, -1], [0, 1, -1]],
                   dtype=np.float64)


# the light sets for h: D2Q5 = the first five vectors of D2Q9; D3Q7 grouped
# by e_z like D3Q19
D2Q5_E = D2Q9_E[:5]
D3Q7_E = np.array([[0, 0, 1], [0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0],
                   [0, 0, -1]], dtype=np.float64)


def first_moment(f, lattice, light=False):
    """sum_k e_k f_k for populations f of shape (Q, nz, ny, nx) -> (nz, ny, nx, 3);
    lattice 0 D2Q9, 1 D3Q19, 2 D2Q5, 3 D3Q7 (light: the light lattice of 0, 1)."""
    if light or lattice in (2, 3):
        e = D2Q5_E if lattice in (0, 2) else D3Q7_E
    else:
        e = D2Q9_E if lattice == 0 else D3Q19_E
    return np.einsum("ka,k...->...a", e, f)


# General quadratic free energies (eps_s != eps_l), Sec. 2.3, in the reduced
# variables of the paper (mu = mu_bar V_m E, omega = omega_bar E,
# E = sqrt(eps_s eps_l)).  Stated from the grand potentials of the two phases,
# Eq. (Quadratic_grand-potential_Liquid), and the composition of the mixture,
# Eq. (Composition_Quadratic), not from the closure or the source the oracle
# evaluates.


def quad_omega(mu, eps_phi, eps_s, eps_l, m_phi, f_min_bar):
    """Reduced grand potential of one phase: -(E / eps_phi) mu^2 / 2
    - m_phi mu + f_min_bar."""
    E = math.sqrt(eps_s * eps_l)
    return -(E / eps_phi) * mu * mu / 2.0 - m_phi * mu + f_min_bar


def quad_composition(phi, mu, eps_s, eps_l, m_s, m_l):
    """c(phi, mu) of Eq. (Composition_Quadratic) with h(phi) = phi, in reduced
    units: phi m_l + (1 - phi) m_s + (phi E / eps_l + (1 - phi) E / eps_s) mu."""
    E = math.sqrt(eps_s * eps_l)
    return phi * m_l + (1.0 - phi) * m_s + (phi * E / eps_l + (1.0 - phi) * E / eps_s) * mu


def quad_mu_eq(eps_s, eps_l, m_s, m_l, df_min, near=0.0):
    """Equilibrium chemical potential: equal grand potentials of the two
    phases, Eq. (Egalite_grand-potentiel), omega_l(mu) = omega_s(mu) with
    f_min_s - f_min_l = df_min; the root nearest to `near`."""
    f = lambda m: (quad_omega(m, eps_l, eps_s, eps_l, m_l, 0.0)
                   - quad_omega(m, eps_s, eps_s, eps_l, m_s, df_min))
    return brentq(f, near - 0.5, near + 0.5, xtol=1e-15, rtol=1e-15)


def lattice_cs2(lattice: int) -> float:
    """xi_s^2, the second moment of the weights: 1/4 on D3Q7, 1/3 otherwise."""
    return 0.25 if lattice == 3 else 1.0 / 3.0


def lattice_dim(lattice: int) -> int:
    return 2 if lattice in (0, 2) else 3
