"""FP64 restatement of the coupled step in PyTorch (CPU), differentiated by
autograd: the oracle of the adjoint.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  It restates S1-S9 of
oracle.c (same readings of the paper, same lattices) with tensor operations so
that torch.autograd provides exact derivatives of the discrete map; its forward
is pinned against the C oracle by the tests.  Shares no code with the GPU
library.

State: natural populations g, h of shape (Q, nz, ny, nx) and phi (nz, ny, nx).
"""
from __future__ import annotations

import math

import numpy as np
import torch

D2Q9_E = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0),
          (1, 1, 0), (-1, 1, 0), (-1, -1, 0), (1, -1, 0)]
D2Q9_W = [4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36]
D3Q19_E = [(0, 0, 1), (1, 0, 1), (-1, 0, 1), (0, 1, 1), (0, -1, 1), (0, 0, 0),
           (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (1, 1, 0), (-1, 1, 0),
           (-1, -1, 0), (1, -1, 0), (0, 0, -1), (-1, 0, -1), (1, 0, -1), (0, -1, -1),
           (0, 1, -1)]
D3Q19_W = [1 / 18, 1 / 36, 1 / 36, 1 / 36, 1 / 36, 1 / 3, 1 / 18, 1 / 18, 1 / 18, 1 / 18,
           1 / 36, 1 / 36, 1 / 36, 1 / 36, 1 / 18, 1 / 36, 1 / 36, 1 / 36, 1 / 36]
# the light sets: D2Q5 = rest and axes of D2Q9; D3Q7 grouped by e_z
D2Q5_E = D2Q9_E[:5]
D2Q5_W = [1 / 3, 1 / 6, 1 / 6, 1 / 6, 1 / 6]
D3Q7_E = [(0, 0, 1), (0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, -1)]
D3Q7_W = [1 / 8, 1 / 4, 1 / 8, 1 / 8, 1 / 8, 1 / 8, 1 / 8]


class Lattice:
    """Velocity set, weights and the index maps of streaming and of the
    gradient stencil for one grid (periodic wrap / zero-flux walls).  role
    "g" or "h": the lattice of that distribution (lattice 0 D2Q9, 1 D3Q19,
    2 D2Q5, 3 D3Q7 for g; h on D2Q5 / D3Q7 under g on a light lattice or with
    h_lattice = 1).  cs2 = xi_s^2 of the set, inv_cs2 its inverse (3 or 4)."""

    def __init__(self, cfg, role="g"):
        lat = int(cfg["lattice"])
        self.d3 = lat in (1, 3)
        light = lat in (2, 3) or (role == "h" and int(cfg.get("h_lattice", 0)) == 1)
        if self.d3:
            e, w = (D3Q7_E, D3Q7_W) if light else (D3Q19_E, D3Q19_W)
        else:
            e, w = (D2Q5_E, D2Q5_W) if light else (D2Q9_E, D2Q9_W)
        self.e = e
        self.w = torch.tensor(w, dtype=torch.float64)
        self.cs2 = 0.25 if (self.d3 and light) else 1.0 / 3.0
        self.inv_cs2 = 4.0 if (self.d3 and light) else 3.0
        self.Q = len(self.e)
        self.D = 3 if self.d3 else 2
        self.rest = self.e.index((0, 0, 0))
        self.opp = [self.e.index((-a, -b, -c)) for (a, b, c) in self.e]
        nz, ny, nx = cfg["shape"]
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz
        bc = list(cfg["bc"])
        if not self.d3:
            bc[2] = 0
        z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        coords = (x.ravel(), y.ravel(), z.ravel())
        n3 = (nx, ny, nz)

        def flat(cx, cy, cz):
            return cx + nx * (cy + ny * cz)

        # pull streaming: destination (k, i) reads source flat index into (Q*N)
        src = np.empty((self.Q, self.N), dtype=np.int64)
        for k, ek in enumerate(self.e):
            c = [coords[a] - ek[a] for a in range(3)]
            wall = np.zeros(self.N, dtype=bool)
            for a in range(3):
                out = (c[a] < 0) | (c[a] >= n3[a])
                if bc[a]:
                    wall |= out
                c[a] = np.mod(c[a], n3[a])
            s = k * self.N + flat(*c)
            s[wall] = self.opp[k] * self.N + np.arange(self.N)[wall]
            src[k] = s
        self.stream_src = torch.from_numpy(src.ravel())

        # gradient stencil: flat index of x + e_k (wrap or mirror ghost)
        def nbr(d):
            c = []
            for a in range(3):
                v = coords[a] + d[a]
                if bc[a]:
                    v = np.clip(v, 0, n3[a] - 1)
                else:
                    v = np.mod(v, n3[a])
                c.append(v)
            return torch.from_numpy(flat(*c))

        self.plus = [nbr(ek) for ek in self.e]
        self.minus = [nbr(tuple(-v for v in ek)) for ek in self.e]
        self.ev = torch.tensor(self.e, dtype=torch.float64)  # (Q, 3)


def _edot(L, k, v):
    """e_k . v for a field of vectors v (3, N)."""
    r = torch.zeros_like(v[0])
    for a in range(L.D):
        if L.e[k][a] != 0:
            r = r + float(L.e[k][a]) * v[a]
    return r


def gradient_normal(L, phi, eps_n):
    acc = [torch.zeros_like(phi) for _ in range(3)]
    for k in range(L.Q):
        if k == L.rest:
            continue
        d = 0.5 * (phi[L.plus[k]] - phi[L.minus[k]])
        for a in range(L.D):
            if L.e[k][a] != 0:
                acc[a] = acc[a] + (float(L.w[k]) * float(L.e[k][a])) * d
    g = torch.stack([L.inv_cs2 * acc[a] for a in range(3)])
    den = torch.sqrt((g[:L.D] ** 2).sum(0) + eps_n * eps_n)
    return g, g / den


def _quadratic(P):
    return int(P.get("free_energy", 0)) == 1


def coupling(P, mu):
    """S_phi / p'(phi): dc (mu - mu_eq), or for general quadratic free
    energies ((eps_l - eps_s)/sqrt(eps_l eps_s)) mu^2/2 - (m_l - m_s) mu - df_min."""
    if _quadratic(P):
        k2 = (P["eps_l"] - P["eps_s"]) / math.sqrt(P["eps_l"] * P["eps_s"])
        return (k2 * mu * mu) * 0.5 - (P["m_l"] - P["m_s"]) * mu - P["df_min"]
    return (P["c_s_co"] - P["c_l_co"]) * (mu - P["mu_eq"])


def at_jump(P, mu):
    """Composition jump of the anti-trapping current."""
    if _quadratic(P):
        ks = -((P["eps_s"] - P["eps_l"]) / math.sqrt(P["eps_s"] * P["eps_l"]))
        return ks * mu + P["m_s"] - P["m_l"]
    return P["c_s_co"] - P["c_l_co"]


def limit01(phi):
    """phi limited to [0, 1]: the argument of the interpolation functions p'
    (of S_phi) and q (of D), defined on the range of the phase field."""
    return torch.clamp(phi, 0.0, 1.0)


def sources(L, P, phi, mu, n):
    pp = phi * (1.0 - phi)
    pl = limit01(phi)
    Gst = -((P["lam"] * P["M_phi"]) / (P["W"] * P["W"])) * ((6.0 * (pl * (1.0 - pl)))
                                                           * coupling(P, mu))
    if P["counter_term"]:
        kphi = (4.0 / P["W"]) * pp
        G = torch.stack([float(L.w[k]) * (Gst + kphi * _edot(L, k, n)) for k in range(L.Q)])
        return G, Gst
    Gdw = -((8.0 * P["M_phi"]) / (P["W"] * P["W"])) * (2.0 * (pp * (1.0 - 2.0 * phi)))
    G = torch.stack([float(L.w[k]) * (Gst + Gdw) for k in range(L.Q)])
    return G, Gst + Gdw


def closure(P, c, phi):
    if _quadratic(P):
        fac = math.sqrt(P["eps_s"] * P["eps_l"]) / (P["eps_s"] * phi + P["eps_l"] * (1.0 - phi))
        return fac * (c - phi * P["m_l"] - (1.0 - phi) * P["m_s"])
    return P["mu_eq"] + (c - (P["c_l_co"] * phi + P["c_s_co"] * (1.0 - phi)))


def h_parts(L, P, c, phi, mu, F):
    """Equilibrium and source of h.  With h^eq,alt (h_scheme = 1) the flux is
    folded into the moving populations, w_k (Lambda + e_k . F / xi_s^2), and
    the source is zero."""
    q = limit01(phi)
    D = P["D_l"] * q + P["D_s"] * (1.0 - q)
    lam_ = (P["gamma"] * D) * mu
    alt = int(P.get("h_scheme", 0)) == 1
    heq = []
    for k in range(L.Q):
        if k == L.rest:
            heq.append(c - (1.0 - float(L.w[k])) * lam_)
        elif alt:
            heq.append(float(L.w[k]) * (lam_ + _edot(L, k, F) / L.cs2))
        else:
            heq.append(float(L.w[k]) * lam_)
    heq = torch.stack(heq)
    if alt:
        return heq, torch.zeros_like(heq)
    H = torch.stack([(P["gamma"] * float(L.w[k])) * _edot(L, k, F) for k in range(L.Q)])
    return heq, H


def init(L, Lh, P, phi0, c0):
    """Initial natural state (g, h, phi) from flat phi0, c0 (N,); L, Lh the
    lattices of g and h."""
    mu = closure(P, c0, phi0)
    gr, n = gradient_normal(L, phi0, P["eps_n"])
    G, _ = sources(L, P, phi0, mu, n)
    g = L.w[:, None] * phi0[None, :] - 0.5 * G
    F = (mu * (P["D_l"] - P["D_s"]))[None, :] * gr
    heq, H = h_parts(Lh, P, c0, phi0, mu, F)
    h = heq - 0.5 * H
    return g, h, phi0


def step(L, Lh, P, g, h, phi):
    """One step S1-S9 on flat (Q, N) / (N,) tensors; L, Lh the lattices of g
    and h."""
    Q, N = L.Q, L.N
    omega_g = 1.0 / (L.inv_cs2 * P["M_phi"] + 0.5)
    omega_h = 1.0 / (1.0 / (P["gamma"] * Lh.cs2) + 0.5)
    c = h.sum(0)
    mu = closure(P, c, phi)
    gr, n = gradient_normal(L, phi, P["eps_n"])
    G, sbar = sources(L, P, phi, mu, n)
    gs = g - omega_g * ((g - L.w[:, None] * phi[None, :]) + 0.5 * G) + G
    g1 = gs.reshape(-1)[L.stream_src].reshape(Q, N)
    phi1 = g1.sum(0) + 0.5 * sbar
    F = (mu * (P["D_l"] - P["D_s"]))[None, :] * gr
    if P["anti_trapping"]:
        jat = ((P["a_at"] * P["W"]) * at_jump(P, mu)) * (phi1 - phi)
        F = F + jat[None, :] * n
    heq, H = h_parts(Lh, P, c, phi, mu, F)
    hs = h - omega_h * ((h - heq) + 0.5 * H) + H
    h1 = hs.reshape(-1)[Lh.stream_src].reshape(Lh.Q, N)
    return g1, h1, phi1


def run(cfg, phi0, c0, nsteps, lam=None, D_l=None):
    """phi^K and c^K (flat) after nsteps from (phi0, c0); lam and D_l may be
    tensors (with requires_grad) that replace the mapping's values."""
    L, Lh = Lattice(cfg, "g"), Lattice(cfg, "h")
    P = dict(cfg)
    if lam is not None:
        P["lam"] = lam
    if D_l is not None:
        P["D_l"] = D_l
    g, h, phi = init(L, Lh, P, phi0, c0)
    for _ in range(nsteps):
        g, h, phi = step(L, Lh, P, g, h, phi)
    return phi, h.sum(0)


def objectives(cfg, phi0, phiK):
    """J1 = final solid fraction mean(1 - phi^K); J2 = mean recession
    distance (sum phi^K - sum phi0) / sum (4/W) phi^K (1 - phi^K)."""
    W = cfg["W"]
    J1 = (1.0 - phiK).mean()
    area = ((4.0 / W) * phiK * (1.0 - phiK)).sum()
    J2 = (phiK.sum() - phi0.sum()) / area
    return J1, J2
