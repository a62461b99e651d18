"""Error measures of a reduced-precision run against the FP64 oracle (test
infrastructure; no arithmetic of the scheme).

Interface-position error.  The local normal displacement of the diffuse
interface between two phase fields is, to first order, |phi_a - phi_b| /
|grad phi_b| at a node inside the interface.  Inside a well-formed interface
of width W the equilibrium profile phi = (1 + tanh(2 d / W)) / 2 has
|grad phi| = (1 - tanh^2) / W, at least 0.36 / W over 0.1 < phi < 0.9; the
gradient is small there only where the interface is degenerate: at the
centre of a thin ligament or a vanishing grain, or at a saddle where two
interfaces meet, where phi stays inside (0.1, 0.9) with a vanishing gradient
and the position of the interface is not defined (such places are where the
topology is about to change, and any perturbation is amplified there).  So
the measure is taken over the nodes with 0.1 < phi_b < 0.9 and
|grad phi_b| >= 1 / (4 W), a floor below every slope of a well-formed profile
in that band:

    d_int = max |phi_a - phi_b| / |grad phi_b|  over those nodes.

The nodes left out are counted and reported.  Beside it, the mean normal
displacement of the whole interface (a volume difference over the interface
area, the area being sum |grad phi_b| by the co-area formula):

    d_mean = |sum (phi_a - phi_b)| / sum |grad phi_b|.
"""
from __future__ import annotations

import numpy as np

BAND = (0.1, 0.9)


def gradient_floor(W: float) -> float:
    """Smallest |grad phi| taken into the interface measure: 1 / (4 W)."""
    return 0.25 / W


def interface_error(phi_a, phi_b, grad_b, W: float):
    """(d_int, nodes used, nodes of the band left out) of phi_a against the
    reference phi_b with gradient grad_b (shape phi_b.shape + (3,))."""
    g = np.sqrt((np.asarray(grad_b) ** 2).sum(axis=-1))
    band = (phi_b > BAND[0]) & (phi_b < BAND[1])
    used = band & (g >= gradient_floor(W))
    if not np.any(used):
        return 0.0, 0, int(np.count_nonzero(band))
    d = np.abs(np.asarray(phi_a) - np.asarray(phi_b))[used] / g[used]
    return float(np.max(d)), int(np.count_nonzero(used)), int(np.count_nonzero(band & ~used))


def mean_interface_shift(phi_a, phi_b, grad_b) -> float:
    """Mean normal displacement of the interface: volume difference over
    interface area."""
    area = float(np.sqrt((np.asarray(grad_b) ** 2).sum(axis=-1)).sum())
    return abs(float((np.asarray(phi_a) - np.asarray(phi_b)).sum())) / max(area, 1e-300)
