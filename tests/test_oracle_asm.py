"""Pins for the oracle's band-limited angular-spectrum propagation (Eqs. 7, 14, 16).

Each test checks the oracle against something other than itself: a brute-force
DFT written from the definition, closed-form propagation of plane waves and of
a Gaussian beam, energy conservation, inverse and semigroup identities, and the
adjoint identity.
"""
import math

import numpy as np
import pytest

from oracle import asm

LAM = 515e-9
PITCH = 8e-6


def _signed(k, n):
    return k if k < n - k else k - n  # the Nyquist bin's sign does not change f^2 or |f|


def _brute_asm(U, lam, z, pitch, pad, mode):
    """Direct O(N^4) evaluation of crop(IDFT2(H . DFT2(pad U))) from the definitions."""
    H, W = U.shape
    pH, pW = pad * H, pad * W
    P = np.zeros((pH, pW), complex)
    P[:H, :W] = U
    n = np.arange(pH)
    m = np.arange(pW)
    out = np.zeros((H, W), complex)
    dfx, dfy = 1.0 / (pW * pitch), 1.0 / (pH * pitch)
    for ky in range(pH):
        for kx in range(pW):
            fy = _signed(ky, pH) * dfy
            fx = _signed(kx, pW) * dfx
            ok = True
            if mode >= 1:
                ok &= fx * fx + fy * fy <= 1 / lam ** 2
            if mode >= 2:
                ok &= abs(fx) <= 1 / (lam * math.sqrt((2 * dfx * z) ** 2 + 1))
                ok &= abs(fy) <= 1 / (lam * math.sqrt((2 * dfy * z) ** 2 + 1))
            if not ok:
                continue
            arg = 1 / lam ** 2 - fx * fx - fy * fy
            if arg >= 0:
                h = np.exp(2j * np.pi * z * np.sqrt(arg))
            else:   # mode 0 only: the decaying evanescent continuation
                h = np.exp(-2 * np.pi * abs(z) * np.sqrt(-arg))
            X = np.sum(P * np.exp(-2j * np.pi * (ky * n[:, None] / pH + kx * m[None, :] / pW)))
            r = np.arange(H)[:, None]
            c = np.arange(W)[None, :]
            out += h * X * np.exp(2j * np.pi * (ky * r / pH + kx * c / pW))
    return out / (pH * pW)


@pytest.mark.parametrize("shape,pad,mode,pitch,z", [
    ((4, 4), 2, 2, PITCH, 1e-3),
    ((3, 5), 2, 1, PITCH, 2e-3),       # radix 3 and 5 on the padded 6 x 10 grid
    ((9, 15), 1, 2, PITCH, -1.5e-3),   # odd sizes, negative distance
    ((6, 5), 2, 2, 0.3e-6, 4e-6),      # evanescent and sampling masks both active
    ((6, 5), 2, 0, 0.3e-6, 4e-6),      # no band limit: evanescent bins decay
    ((5, 6), 1, 0, 0.3e-6, -3e-6),     # ... for either sign of z
])
def test_matches_brute_force_dft(shape, pad, mode, pitch, z):
    rng = np.random.default_rng(7)
    U = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    got = asm.propagate(U, LAM, z, pitch, pad, mode)
    ref = _brute_asm(U, LAM, z, pitch, pad, mode)
    assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_plane_wave_gets_phase_2pi_z_over_lambda():
    U = np.full((16, 24), 0.7 + 0.2j)
    for z in (0.5e-3, 1e-3, -2e-3):
        u = asm.propagate(U, LAM, z, PITCH, pad=1, mode=2)
        expected = U * np.exp(2j * np.pi * z / LAM)
        assert np.max(np.abs(u - expected)) < 1e-11


def test_tilted_plane_wave_on_a_bin():
    H, W = 16, 32
    kx, ky = 3, -2
    r = np.arange(H)[:, None]
    c = np.arange(W)[None, :]
    U = np.exp(2j * np.pi * (kx * c / W + ky * r / H))
    z = 1.3e-3
    fx, fy = kx / (W * PITCH), ky / (H * PITCH)
    expected = U * np.exp(2j * np.pi * z * math.sqrt(1 / LAM ** 2 - fx * fx - fy * fy))
    u = asm.propagate(U, LAM, z, PITCH, pad=1, mode=2)
    assert np.max(np.abs(u - expected)) < 1e-11


def test_parseval_on_padded_grid():
    rng = np.random.default_rng(1)
    U = rng.normal(size=(20, 30)) + 1j * rng.normal(size=(20, 30))
    u = asm.propagate(U, LAM, 1e-3, PITCH, pad=2, mode=2, crop=False)
    assert abs(np.sum(np.abs(u) ** 2) / np.sum(np.abs(U) ** 2) - 1) < 1e-12


def test_round_trip_and_semigroup():
    rng = np.random.default_rng(2)
    P = rng.normal(size=(24, 40)) + 1j * rng.normal(size=(24, 40))
    z = 1.7e-3
    fwd = asm.propagate(P, LAM, z, PITCH, mode=1, crop=False, padded_input=True)
    back = asm.propagate(fwd, LAM, -z, PITCH, mode=1, crop=False, padded_input=True)
    assert np.max(np.abs(back - P)) < 1e-12
    a, b = 0.4e-3, 1.1e-3
    two = asm.propagate(asm.propagate(P, LAM, a, PITCH, mode=1, crop=False, padded_input=True),
                        LAM, b, PITCH, mode=1, crop=False, padded_input=True)
    one = asm.propagate(P, LAM, a + b, PITCH, mode=1, crop=False, padded_input=True)
    # phases reach 2 pi z / lambda ~ 2e4 rad, so FP64 rounding alone gives ~4e-12
    assert np.max(np.abs(two - one)) < 1e-10


@pytest.mark.parametrize("z", [1e-3, 50e-3])
def test_gaussian_beam_closed_form(z):
    """Paraxial Gaussian beam: u = e^{ikz} (w0^2/q) exp(-r^2/q), q = w0^2 + i lambda z / pi.

    The non-paraxial correction is about 2 pi z lambda^3 f^4 / 8 ~ 1e-8 rad here.
    At 50 mm the beam widens by 1.29x and the sampling band limit is active but
    lies an order of magnitude outside the beam's spectrum.
    """
    H = W = 128
    w0 = 100e-6
    x = (np.arange(W) + 0.5 - W / 2) * PITCH
    y = (np.arange(H) + 0.5 - H / 2) * PITCH
    r2 = x[None, :] ** 2 + y[:, None] ** 2
    U = np.exp(-r2 / w0 ** 2)
    u = asm.propagate(U, LAM, z, PITCH, pad=2, mode=2)
    q = w0 ** 2 + 1j * LAM * z / np.pi
    expected = np.exp(2j * np.pi * z / LAM) * (w0 ** 2 / q) * np.exp(-r2 / q)
    err = np.linalg.norm(u - expected) / np.linalg.norm(expected)
    assert err < 1e-6, err
    if z > 10e-3:
        assert np.abs(expected).max() < 0.8   # the test is sensitive: the peak has dropped


def test_evanescent_and_sampling_masks_remove_plane_waves():
    H = W = 32
    pitch = 0.2e-6                    # Nyquist 2.5e6 /m exceeds 1/lambda = 1.94e6 /m
    r = np.arange(H)[:, None]
    c = np.arange(W)[None, :]
    fcut = 1 / LAM
    k_evan = int(math.ceil(fcut * W * pitch * 1.02))   # a bin above the cut
    k_prop = int(math.floor(fcut * W * pitch * 0.9))   # a bin below it
    assert k_evan < W // 2 and k_prop > 0
    for k, alive in ((k_evan, False), (k_prop, True)):
        U = np.exp(2j * np.pi * k * c / W) * np.ones((H, 1))
        u = asm.propagate(U, LAM, 1e-7, pitch, pad=1, mode=1)
        assert (np.max(np.abs(u)) > 0.99) == alive
        if not alive:
            assert np.max(np.abs(u)) < 1e-12
    # sampling limit (mode 2) at a large distance: f_lim = 1/(lambda sqrt((2 df z)^2 + 1))
    pitch, z = 8e-6, 0.5
    dfx = 1 / (W * pitch)
    flim = 1 / (LAM * math.sqrt((2 * dfx * z) ** 2 + 1))
    k_lim = flim / dfx
    for k, alive in ((int(math.floor(k_lim)), True), (int(math.floor(k_lim)) + 1, False)):
        U = np.exp(2j * np.pi * k * c / W) * np.ones((H, 1))
        u1 = asm.propagate(U, LAM, z, pitch, pad=1, mode=1)
        u2 = asm.propagate(U, LAM, z, pitch, pad=1, mode=2)
        assert np.max(np.abs(u1)) > 0.99                      # mode 1 keeps it
        assert (np.max(np.abs(u2)) > 0.99) == alive


def test_evanescent_plane_wave_decays_without_band_limit():
    """Band mode 0: a plane wave on a bin beyond 1/lambda is kept and scaled by
    exp(-2 pi |z| sqrt(f^2 - 1/lambda^2)); one inside the band gets the phase
    of Eq. 7 exactly as with the band limit."""
    H = W = 32
    pitch = 0.2e-6
    c = np.arange(W)[None, :]
    k_evan = int(math.ceil(W * pitch / LAM * 1.02))
    f = k_evan / (W * pitch)
    for z in (3e-7, -3e-7):
        U = np.exp(2j * np.pi * k_evan * c / W) * np.ones((H, 1))
        u = asm.propagate(U, LAM, z, pitch, pad=1, mode=0)
        expect = math.exp(-2 * math.pi * abs(z) * math.sqrt(f * f - 1 / LAM ** 2))
        assert 1e-3 < expect < 0.9
        assert np.allclose(u, expect * U, rtol=0, atol=1e-12)
    k_prop = int(math.floor(W * pitch / LAM * 0.9))
    U = np.exp(2j * np.pi * k_prop * c / W) * np.ones((H, 1))
    assert np.allclose(asm.propagate(U, LAM, 3e-7, pitch, 1, 0), asm.propagate(U, LAM, 3e-7, pitch, 1, 1),
                       rtol=0, atol=1e-13)


def test_adjoint_identity():
    rng = np.random.default_rng(3)
    for mode, pad in ((2, 2), (1, 1), (0, 2)):
        u = rng.normal(size=(12, 20)) + 1j * rng.normal(size=(12, 20))
        v = rng.normal(size=(12, 20)) + 1j * rng.normal(size=(12, 20))
        Au = asm.propagate(u, LAM, 0.8e-3, PITCH, pad, mode)
        AHv = asm.propagate_adjoint(v, LAM, 0.8e-3, PITCH, pad, mode)
        lhs = np.vdot(v, Au)
        rhs = np.vdot(AHv, u)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)
