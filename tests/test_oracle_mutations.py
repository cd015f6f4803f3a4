"""Plant plausible mistakes in the oracle (on the CPU) and check a pin catches each.

Each test swaps one oracle function for a subtly wrong version -- a flipped
sign, a dropped factor, a transposed operand, a wrong index offset -- and
asserts that one of the pins in test_oracle_pins.py then fails.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import nufds_oracle as mod
from tests import test_oracle_pins as pins


def _patch(monkeypatch, name, fn):
    monkeypatch.setattr(mod, name, fn)
    monkeypatch.setattr(O, name, fn)


def test_flipped_chirp_sign_is_caught(monkeypatch):
    def bad_frt(h, band, wavelength, pitch, z):
        k = 2.0 * math.pi / wavelength
        xi_x = (np.arange(band.mx) - band.mx // 2) * (band.nx * pitch / band.mx)
        xi_y = (np.arange(band.my) - band.my // 2) * (band.ny * pitch / band.my)
        chirp = np.exp(-1j * k * (xi_y[:, None] ** 2 + xi_x[None, :] ** 2) / (2.0 * z))
        return mod.centred_dft2(h * chirp)
    _patch(monkeypatch, "fresnel_frt", bad_frt)
    with pytest.raises(AssertionError):
        pins.test_frt_of_paraxial_wave_is_a_kronecker_delta()


def test_dropped_magnification_factor_is_caught(monkeypatch):
    from scipy import special

    def bad_mx(fx, fy, wavelength):
        fx = np.asarray(fx, dtype=np.float64)
        fy = np.asarray(fy, dtype=np.float64)
        a2 = 1.0 - (wavelength * fy) ** 2
        return special.hyp2f1(0.5, 0.75, 1.5, (wavelength * fx) ** 2 / a2)   # (1 - v^2)^(-1/4) dropped
    _patch(monkeypatch, "magnification_x", bad_mx)
    with pytest.raises(AssertionError):
        pins.test_eq15_is_the_derivative_of_eq16()


def test_missing_axis_centring_is_caught(monkeypatch):
    def bad_dft(a):
        # centring applied along y only: the x coordinates are off by N_x/2 samples
        return np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(a, axes=0)), axes=0)
    _patch(monkeypatch, "centred_dft2", bad_dft)
    with pytest.raises(AssertionError):
        pins.test_centred_dft_matches_explicit_matrices()


def test_wrong_centre_index_is_caught(monkeypatch):
    good = mod.plan_band

    def bad_plan(*a, **k):
        b = good(*a, **k)
        b.kcx = -b.kcx            # sub-band centred on the mirror image of the window
        return b
    _patch(monkeypatch, "plan_band", bad_plan)
    with pytest.raises(AssertionError):
        pins.test_point_focuses_at_its_true_position(90.0, 0.5)


def test_unconjugated_input_is_caught(monkeypatch):
    good = mod.reconstruct

    def bad_reconstruct(H, *a, flags=0, **k):
        return good(H, *a, flags=flags | O.CONVERGING, **k)   # diverging input read as converging
    _patch(monkeypatch, "reconstruct", bad_reconstruct)
    with pytest.raises(AssertionError):
        pins.test_point_focuses_at_its_true_position(60.0, 0.5)


def test_stack_sharing_the_smallest_size_is_caught(monkeypatch):
    def bad_stack(H, wavelength, pitch, zs, flags=0):
        H = np.asarray(H, dtype=np.complex128)
        ny, nx = H.shape
        bands = [mod.plan_band(nx, ny, wavelength, pitch, z, None, flags) for z in zs]
        size = (min(b.mx for b in bands), min(b.my for b in bands))   # smallest instead of largest
        return [mod.reconstruct(H, wavelength, pitch, z, flags=flags, frt_size=size) for z in zs]
    _patch(monkeypatch, "focal_stack", bad_stack)
    with pytest.raises(AssertionError):
        pins.test_focal_stack_focuses_a_point_at_its_depth()


def test_stack_in_sorted_depth_order_is_caught(monkeypatch):
    good = mod.focal_stack

    def bad_stack(H, wavelength, pitch, zs, flags=0):
        return good(H, wavelength, pitch, sorted(zs), flags)
    _patch(monkeypatch, "focal_stack", bad_stack)
    with pytest.raises(AssertionError):
        pins.test_focal_stack_focuses_a_point_at_its_depth()


def test_off_centre_padding_is_caught(monkeypatch):
    good = mod.centred_dft2

    def bad_dft(a):
        # a padded array whose hologram sits one sample right of the centre: the spectrum picks up
        # a phase ramp (the mistake an off-by-one pad offset makes)
        if a.shape == (96, 128):
            a = np.roll(a, 1, axis=1)
        return good(a)
    _patch(monkeypatch, "centred_dft2", bad_dft)
    with pytest.raises(AssertionError):
        pins.test_oversampled_spectrum_interleaves_the_plain_one()


def test_lower_degree_paper_polynomial_is_caught(monkeypatch):
    from scipy import special

    def bad_poly(s, degree=8, samples=51):
        u = np.linspace(-s, s, samples)
        return np.polyfit(u, special.hyp2f1(0.5, 0.75, 1.5, u * u), 4)   # degree 4 instead of 8
    _patch(monkeypatch, "paper_polynomial", bad_poly)
    with pytest.raises(AssertionError):
        pins.test_paper_polynomial_matches_eq16_where_fitted(120.0, 1e-3)
