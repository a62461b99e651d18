"""The interface-position measures of tests/metrics.py on fields whose
displacement is known."""
import numpy as np

from tests import metrics


def _front(shift, W=2.5, n=64):
    x = np.arange(n, dtype=np.float64) - 30.0 - shift
    phi = 0.5 * (1.0 + np.tanh(2.0 * x / W))
    dphi = (1.0 - np.tanh(2.0 * x / W) ** 2) / W
    phi3 = np.broadcast_to(phi, (4, 5, n)).copy()
    grad = np.zeros((4, 5, n, 3))
    grad[..., 0] = dphi
    return phi3, grad


def test_shifted_front_displacement_is_recovered():
    """A planar equilibrium front moved by delta along its normal: both
    measures return delta to first order (the band's second-order term is
    delta^2 |phi''| / |phi'|, below 1% of delta here)."""
    W = 2.5
    for delta in (1e-4, 1e-3, 3e-3):
        phi_b, grad_b = _front(0.0, W)
        phi_a, _ = _front(delta, W)
        d, used, left = metrics.interface_error(phi_a, phi_b, grad_b, W)
        assert used > 0 and left == 0
        assert abs(d / delta - 1.0) < 0.01, (delta, d)
        dm = metrics.mean_interface_shift(phi_a, phi_b, grad_b)
        assert abs(dm / delta - 1.0) < 1e-3, (delta, dm)


def test_degenerate_interface_nodes_are_left_out():
    """A thin solid ligament whose phi never goes below 0.3: its centre has
    phi in the band and a vanishing gradient.  It is left out of d_int and
    counted; a perturbation there does not enter d_int."""
    W = 2.5
    x = np.arange(40, dtype=np.float64) - 20.0
    phi_b = 1.0 - 0.7 * np.exp(-(x / 3.0) ** 2)
    grad = np.zeros(x.shape + (3,))
    grad[:, 0] = 0.7 * 2.0 * x / 9.0 * np.exp(-(x / 3.0) ** 2)
    phi_a = phi_b.copy()
    phi_a[20] += 1e-3  # at the centre, where |grad| = 0
    d, used, left = metrics.interface_error(phi_a, phi_b, grad, W)
    assert left >= 1 and used > 0
    assert d == 0.0
    phi_a[17] += 1e-3  # on the flank, where the gradient is large
    d, _, _ = metrics.interface_error(phi_a, phi_b, grad, W)
    assert d > 0.0 and np.isfinite(d)
