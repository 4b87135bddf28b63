"""Pins for the phase-only conversion oracle: a phase-only hologram is its own
optimum (zero loss and zero gradient at its phase), and the phase gradient
matches central differences of the loss."""
import numpy as np

from oracle import phase_only

LAMS = (639e-9, 473e-9)
Z = (0.6e-3, 1.4e-3)
PITCH = 8e-6


def test_phase_only_hologram_is_a_fixed_point():
    rng = np.random.default_rng(0)
    phi0 = rng.uniform(0, 2 * np.pi, size=(1, 2, 10, 12))
    U = phase_only.layer_fields(np.exp(1j * phi0), LAMS, Z, PITCH)
    loss, g = phase_only.phase_only_loss(U, phi0, LAMS, Z, PITCH)
    assert abs(loss) < 1e-12
    assert np.max(np.abs(g)) < 1e-12


def test_phase_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    P = rng.uniform(0.2, 1.0, size=(1, 2, 10, 12)) * np.exp(2j * np.pi * rng.uniform(size=(1, 2, 10, 12)))
    U = phase_only.layer_fields(P, LAMS, Z, PITCH)
    phi = rng.uniform(0, 2 * np.pi, size=(1, 2, 10, 12))
    loss, g = phase_only.phase_only_loss(U, phi, LAMS, Z, PITCH)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (0, 1, 5, 6), (0, 0, 9, 11), (0, 1, 2, 9)]:
        pp, pm = phi.copy(), phi.copy()
        pp[idx] += h
        pm[idx] -= h
        fd = (phase_only.phase_only_loss(U, pp, LAMS, Z, PITCH)[0]
              - phase_only.phase_only_loss(U, pm, LAMS, Z, PITCH)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-7 * max(1.0, abs(fd)), (idx, fd, g[idx])
    # the SSIM term contributes
    loss0, _ = phase_only.phase_only_loss(U, phi, LAMS, Z, PITCH, weight=0.0)
    assert loss0 < loss
