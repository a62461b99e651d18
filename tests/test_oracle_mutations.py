"""Mutation check of the oracle's pins.

Each entry below plants one plausible slip in a copy of oracle.c (a dropped
term or factor, a flipped sign, a wrong index, a transposed operand, a wrong
table entry, for the full lattices and for the light h lattices), builds the
copy, and runs the pins of test_oracle_pins.py against it.  Every mutant must make at least one pin fail: a pin set that
lets one through does not pin that part of the oracle.  The shipped oracle
is never modified; the mutants live in a temporary directory.
"""
import concurrent.futures
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "oracle.c")

# (name, original text in oracle.c, replacement)
MUTANTS = [
    ("closure: phases swapped in c_co(phi)",
     "double cco = (p->c_l_co * phi) + (p->c_s_co * (1.0 - phi));",
     "double cco = (p->c_s_co * phi) + (p->c_l_co * (1.0 - phi));"),
    ("closure: sign of c - c_co",
     "return p->mu_eq + (c - cco);",
     "return p->mu_eq + (cco - c);"),
    ("gradient: factor 1/xi_s^2 dropped",
     "g3[a] = s->inv_cs2g * acc[a];",
     "g3[a] = acc[a];"),
    ("gradient: 3 instead of 1/xi_s^2 (D3Q7)",
     "g3[a] = s->inv_cs2g * acc[a];",
     "g3[a] = 3.0 * acc[a];"),
    ("gradient: central difference without 1/2",
     "double dk = 0.5 * (phi_at(",
     "double dk = 1.0 * (phi_at("),
    ("gradient: difference reversed",
     "(phi_at(s, f, x, y, z, s->e[k]) - phi_at(s, f, x, y, z, m))",
     "(phi_at(s, f, x, y, z, m) - phi_at(s, f, x, y, z, s->e[k]))"),
    ("gradient: weight w_k dropped",
     "acc[a] = acc[a] + (s->w[k] * (double)s->e[k][a]) * dk;",
     "acc[a] = acc[a] + ((double)s->e[k][a]) * dk;"),
    ("normal: not normalised",
     "n3[a] = g3[a] / den;",
     "n3[a] = g3[a];"),
    ("e_k . v: operand axes transposed",
     "r = r + (double)s->e[k][a] * v[a];",
     "r = r + (double)s->e[k][a] * v[s->D - 1 - a];"),
    ("p'(phi): factor 6 dropped",
     "double pprime = 6.0 * (pl * (1.0 - pl));",
     "double pprime = (pl * (1.0 - pl));"),
    ("G^st: sign flipped",
     "double Gst = -((p->lambda * p->M_phi) / (p->W * p->W)) * Sphi;",
     "double Gst = ((p->lambda * p->M_phi) / (p->W * p->W)) * Sphi;"),
    ("G^st: W instead of W^2",
     "double Gst = -((p->lambda * p->M_phi) / (p->W * p->W)) * Sphi;",
     "double Gst = -((p->lambda * p->M_phi) / (p->W)) * Sphi;"),
    ("counter term: sign flipped",
     "G[k] = s->w[k] * (Gst + kphi * edot(s, k, n3));",
     "G[k] = s->w[k] * (Gst - kphi * edot(s, k, n3));"),
    ("counter term: 1/W instead of 4/W",
     "double kphi = (4.0 / p->W) * (phi * (1.0 - phi));",
     "double kphi = (1.0 / p->W) * (phi * (1.0 - phi));"),
    ("double well: sign flipped",
     "double Gdw = -((8.0 * p->M_phi) / (p->W * p->W)) * wdw;",
     "double Gdw = ((8.0 * p->M_phi) / (p->W * p->W)) * wdw;"),
    ("phi moment: source moment dropped (counter term)",
     "*sbar = Gst;",
     "*sbar = 0.0;"),
    ("g collision: trapezoidal half source dropped",
     "double t = (gk - s->w[k] * phi) + 0.5 * G[k];",
     "double t = (gk - s->w[k] * phi);"),
    ("g collision: half instead of full source",
     "s->gs[k * N + i] = (gk - omega_g * t) + G[k];",
     "s->gs[k * N + i] = (gk - omega_g * t) + 0.5 * G[k];"),
    ("g relaxation: M = tau / xi_s^2 instead of xi_s^2 tau",
     "const double omega_g = 1.0 / (s->inv_cs2g * p->M_phi + 0.5);",
     "const double omega_g = 1.0 / (p->M_phi / s->inv_cs2g + 0.5);"),
    ("g relaxation: tau_g = 3 M on D3Q7",
     "const double omega_g = 1.0 / (s->inv_cs2g * p->M_phi + 0.5);",
     "const double omega_g = 1.0 / (3.0 * p->M_phi + 0.5);"),
    ("g lattice D3Q7: 1/xi_s^2 = 3",
     "    s->inv_cs2g = 4.0;",
     "    s->inv_cs2g = 3.0;"),
    ("g lattice D3Q7: h relaxed with the xi_s^2 of D3Q19",
     "s->cs2h = p->lattice == ORC_D3Q7 ? 1.0 / 4.0 : 1.0 / 3.0;",
     "s->cs2h = 1.0 / 3.0;"),
    ("h relaxation: tau_h = 1/gamma instead of 1/(gamma xi_s^2)",
     "const double omega_h = 1.0 / (1.0 / (p->gamma * s->cs2h) + 0.5);",
     "const double omega_h = 1.0 / (1.0 / p->gamma + 0.5);"),
    ("h relaxation: D3Q7 with the xi_s^2 of D3Q19",
     "    s->cs2h = 1.0 / 4.0;",
     "    s->cs2h = 1.0 / 3.0;"),
    ("phi^{n+1}: half source moment dropped",
     "s->phin[i] = sum + 0.5 * s->sbar[i];",
     "s->phin[i] = sum;"),
    ("anti-trapping: sign flipped",
     "j = (((p->a_at * p->W) * jump) * dtphi) * s->nrm[3 * i + a];",
     "j = -(((p->a_at * p->W) * jump) * dtphi) * s->nrm[3 * i + a];"),
    ("anti-trapping: d phi / dt taken as zero",
     "double dtphi = s->phin[i] - phi;",
     "double dtphi = 0.0;"),
    ("flux: mu D' grad phi term dropped",
     "F[a] = (mu * (p->D_l - p->D_s)) * s->grad[3 * i + a] + j;",
     "F[a] = j;"),
    ("D(phi): phases swapped",
     "double D = (p->D_l * q) + (p->D_s * (1.0 - q));",
     "double D = (p->D_s * q) + (p->D_l * (1.0 - q));"),
    ("h source: gamma dropped",
     "return (s->p.gamma * s->wh[k]) * r;",
     "return (s->wh[k]) * r;"),
    ("h equilibrium: rest population c - Lambda",
     "if (k == s->resth) return c - (1.0 - s->wh[k]) * lam;\n  return s->wh[k] * lam;",
     "if (k == s->resth) return c - lam;\n  return s->wh[k] * lam;"),
    ("h collision: trapezoidal half source dropped",
     "double t = (hk - h_equilibrium(s, k, c, lam)) + 0.5 * Hk;",
     "double t = (hk - h_equilibrium(s, k, c, lam));"),
    ("moment c: first population skipped",
     "for (int k = 0; k < Qh; ++k) c = c + s->h[k * N + i];",
     "for (int k = 1; k < Qh; ++k) c = c + s->h[k * N + i];"),
    ("g bounce-back: population not reversed",
     "s->g[k * N + i] = s->gs[s->opp[k] * N + i];",
     "s->g[k * N + i] = s->gs[k * N + i];"),
    ("h bounce-back: population not reversed",
     "s->h[k * N + i] = s->hs[s->opph[k] * N + i];",
     "s->h[k * N + i] = s->hs[k * N + i];"),
    ("D3Q7 table: rest and axis weights swapped",
     "static const double d3q7_w[7] = {1.0 / 8.0, 1.0 / 4.0, 1.0 / 8.0, 1.0 / 8.0,",
     "static const double d3q7_w[7] = {1.0 / 8.0, 1.0 / 8.0, 1.0 / 4.0, 1.0 / 8.0,"),
    ("D2Q5 table: weights of D2Q9",
     "static const double d2q5_w[5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};",
     "static const double d2q5_w[5] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0};"),
    ("streaming: pull from x + e_k",
     "int c3[3] = {x - e[k][0], y - e[k][1], z - e[k][2]};",
     "int c3[3] = {x + e[k][0], y + e[k][1], z + e[k][2]};"),
    ("wall ghost: periodic copy instead of mirror",
     "return v < 0 ? 0 : n - 1;",
     "return (v + n) % n;"),
    ("init: g without the variable-change shift",
     "s->g[k * N + i] = s->w[k] * phi - 0.5 * G[k];",
     "s->g[k * N + i] = s->w[k] * phi;"),
    ("init: h without the variable-change shift",
     "s->h[k * N + i] = h_equilibrium(s, k, c, lam) - 0.5 * h_source(s, k, F);",
     "s->h[k * N + i] = h_equilibrium(s, k, c, lam);"),
    ("D2Q9 table: vector 5 mistyped",
     "{1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};\nstatic const double d2q9_w",
     "{1, -1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};\nstatic const double d2q9_w"),
    # the alternative equilibrium h^eq,alt
    ("h^eq,alt: flux term dropped",
     "return s->wh[k] * (lam + r / s->cs2h);",
     "return s->wh[k] * lam;"),
    ("h^eq,alt: 1/xi_s^2 dropped",
     "return s->wh[k] * (lam + r / s->cs2h);",
     "return s->wh[k] * (lam + r);"),
    ("h^eq,alt: flux with the wrong sign",
     "return s->wh[k] * (lam + r / s->cs2h);",
     "return s->wh[k] * (lam - r / s->cs2h);"),
    ("h^eq,alt: rest population c - Lambda",
     "if (k == s->resth) return c - (1.0 - s->wh[k]) * lam;\n  double r = 0.0;",
     "if (k == s->resth) return c - lam;\n  double r = 0.0;"),
    ("alt collision: source added as well",
     "s->hs[k * N + i] = hk - omega_h * t;",
     "s->hs[k * N + i] = (hk - omega_h * t) + h_source(s, k, F);"),
    ("alt init: shifted by -H/2",
     "s->h[k * N + i] = h_equilibrium_alt(s, k, c, lam, F);",
     "s->h[k * N + i] = h_equilibrium_alt(s, k, c, lam, F) - 0.5 * h_source(s, k, F);"),
    # general quadratic free energies
    ("closure (general): eps_s and eps_l swapped in the denominator",
     "/ ((p->eps_s * phi) + (p->eps_l * (1.0 - phi)));",
     "/ ((p->eps_l * phi) + (p->eps_s * (1.0 - phi)));"),
    ("closure (general): m_s and m_l swapped",
     "return fac * ((c - (phi * p->m_l)) - ((1.0 - phi) * p->m_s));",
     "return fac * ((c - (phi * p->m_s)) - ((1.0 - phi) * p->m_l));"),
    ("closure (general): prefactor dropped",
     "return fac * ((c - (phi * p->m_l)) - ((1.0 - phi) * p->m_s));",
     "return ((c - (phi * p->m_l)) - ((1.0 - phi) * p->m_s));"),
    ("source (general): sign of the mu^2 term",
     "return (((k2 * (mu * mu)) * 0.5) - ((p->m_l - p->m_s) * mu)) - p->df_min;",
     "return (((-k2 * (mu * mu)) * 0.5) - ((p->m_l - p->m_s) * mu)) - p->df_min;"),
    ("source (general): 1/2 of the mu^2 term dropped",
     "return (((k2 * (mu * mu)) * 0.5) - ((p->m_l - p->m_s) * mu)) - p->df_min;",
     "return (((k2 * (mu * mu)) * 1.0) - ((p->m_l - p->m_s) * mu)) - p->df_min;"),
    ("source (general): m_l - m_s reversed",
     "return (((k2 * (mu * mu)) * 0.5) - ((p->m_l - p->m_s) * mu)) - p->df_min;",
     "return (((k2 * (mu * mu)) * 0.5) - ((p->m_s - p->m_l) * mu)) - p->df_min;"),
    ("source (general): sign of df_min",
     "return (((k2 * (mu * mu)) * 0.5) - ((p->m_l - p->m_s) * mu)) - p->df_min;",
     "return (((k2 * (mu * mu)) * 0.5) - ((p->m_l - p->m_s) * mu)) + p->df_min;"),
    ("anti-trapping (general): sign of the mu term",
     "double ks = -((p->eps_s - p->eps_l) / sqrt(p->eps_s * p->eps_l));",
     "double ks = ((p->eps_s - p->eps_l) / sqrt(p->eps_s * p->eps_l));"),
    ("anti-trapping (general): m_s - m_l reversed",
     "return ((ks * mu) + p->m_s) - p->m_l;",
     "return ((ks * mu) + p->m_l) - p->m_s;"),
    ("D3Q19 table: axis and diagonal weights swapped",
     "    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,\n    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,\n    1.0 / 18.0,",
     "    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,\n    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,\n    1.0 / 18.0,"),
    ("p'(phi): not limited to [0, 1]",
     "  double pl = limit01(phi);\n  double pprime",
     "  double pl = phi;\n  double pprime"),
    ("D(phi): q not limited to [0, 1]",
     "  double q = limit01(phi);",
     "  double q = phi;"),
    ("limit: lower bound dropped",
     "  if (phi < 0.0) return 0.0;",
     "  if (phi < -1.0) return 0.0;"),
    ("diagnostics: phi <= 1/2 counted as solid",
     "if (phi < 0.5) count = count + 1.0;",
     "if (phi <= 0.5) count = count + 1.0;"),
    ("diagnostics: min and max swapped",
     "if (phi < mn) mn = phi;",
     "if (phi > mn) mn = phi;"),
    ("diagnostics: solid fraction from phi",
     "solid = solid + (1.0 - phi);",
     "solid = solid + phi;"),
]


def _run_mutant(tmp, idx, name, old, new):
    import oracle
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutant '{name}': original text not found exactly once"
    mdir = os.path.join(tmp, f"m{idx:02d}")
    os.makedirs(mdir, exist_ok=True)
    msrc = os.path.join(mdir, "oracle.c")
    with open(msrc, "w") as f:
        f.write(src.replace(old, new))
    lib = os.path.join(mdir, "liboracle.so")
    oracle.compile_library(msrc, lib, quiet=True)
    env = dict(os.environ, GPLBM_ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    # exit 1: a pin failed; anything else but 0 (a crash) also exposes the slip
    caught = r.returncode not in (0, 4, 5)
    first_fail = ""
    for line in r.stdout.splitlines():
        if line.startswith("FAILED"):
            first_fail = line
            break
    return name, caught, first_fail, r.returncode


@pytest.mark.slow
def test_every_mutant_is_caught_by_a_pin(tmp_path):
    workers = min(8, os.cpu_count() or 1)
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        futs = [ex.submit(_run_mutant, str(tmp_path), i, *m) for i, m in enumerate(MUTANTS)]
        results = [f.result() for f in futs]
    for name, caught, first_fail, rc in results:
        print(f"{'caught' if caught else 'SURVIVED'} (rc {rc}) {name}: {first_fail}")
    survivors = [name for name, caught, _, _ in results if not caught]
    assert not survivors, f"mutants not caught by any pin: {survivors}"
