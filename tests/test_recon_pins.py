"""Pins of the oracle's focal-stack reconstruction (simulated viewing: focal
planes, pupil filtering and time multiplexing, Sec. 5.3) against what the
mathematics fixes: plane waves inside and outside the pupil, the frame mean,
the paraxial Gaussian beam, and the power a circular pupil passes from a
Gaussian spectrum."""
import numpy as np

from oracle import asm, recon

D, LAM = 8e-6, 520e-9


def _plane(ny, nx, kx, ky):
    y, x = np.meshgrid(np.arange(ny) * D, np.arange(nx) * D, indexing="ij")
    return np.exp(2j * np.pi * (kx / (nx * D) * x + ky / (ny * D) * y))


def test_pupil_passes_plane_waves_by_angle():
    """On one period: a plane wave with lambda |f| below NA keeps unit
    intensity, one above is removed, and in a sum of the two only the first
    survives (the pupil acts on the frequency radius, per wavelength)."""
    ny, nx = 32, 64
    inside, outside = (3, 2), (12, -5)
    f_in = np.hypot(3 / (nx * D), 2 / (ny * D))
    f_out = np.hypot(12 / (nx * D), 5 / (ny * D))
    na = LAM * 0.5 * (f_in + f_out)
    assert LAM * f_in < na < LAM * f_out
    for k, expect in ((inside, 1.0), (outside, 0.0)):
        u = _plane(ny, nx, *k)[None, None]
        I = recon.focal_stack(u, D, [LAM], [2e-3], na=na, band_limit=False, pad=False)
        assert np.allclose(I, expect, atol=1e-12), k
    both = (_plane(ny, nx, *inside) + 0.7 * _plane(ny, nx, *outside))[None, None]
    I = recon.focal_stack(both, D, [LAM], [2e-3, -1e-3], na=na, band_limit=False, pad=False)
    assert np.allclose(I, 1.0, atol=1e-12)
    # at a wavelength long enough that lambda f_in exceeds NA the same aperture removes it
    I = recon.focal_stack(_plane(ny, nx, *inside)[None, None], D, [2.2 * LAM * f_out / f_in], [0.0],
                          na=na, band_limit=False, pad=False)
    assert np.allclose(I, 0.0, atol=1e-12)


def test_frames_average_and_global_phase():
    rng = np.random.default_rng(3)
    u = rng.normal(size=(2, 20, 24)) + 1j * rng.normal(size=(2, 20, 24))
    d = [1e-3, 4e-3]
    both = recon.focal_stack(u[None], D, [LAM], d, na=0.03)
    one = recon.focal_stack(u[None, :1], D, [LAM], d, na=0.03)
    two = recon.focal_stack(u[None, 1:], D, [LAM], d, na=0.03)
    assert np.allclose(both, 0.5 * (one + two), rtol=1e-12)
    shifted = recon.focal_stack(u[None, :1] * np.exp(0.9j), D, [LAM], d, na=0.03)
    assert np.allclose(shifted, one, rtol=1e-12)


def test_without_pupil_is_the_asm_intensity():
    rng = np.random.default_rng(4)
    u = rng.normal(size=(3, 17, 13)) + 1j * rng.normal(size=(3, 17, 13))
    I = recon.focal_stack(u[None], D, [LAM], [5e-3], na=0.0)[0, 0]
    ref = np.mean(np.abs(asm.propagate(u, D, LAM, 5e-3)) ** 2, axis=0)
    assert np.allclose(I, ref, rtol=1e-12)


def test_gaussian_beam_on_axis_intensity():
    """u0 = exp(-r^2 / w0^2): paraxially the on-axis intensity at z is
    1 / (1 + (z / zR)^2), zR = pi w0^2 / lambda; with w0 = 6 pitches the
    beam's divergence is 3e-3 rad, so the exact propagation departs from the
    paraxial law by ~1e-5. Power is conserved without a pupil, up to the
    beam's tail outside the 64-pitch window (exp(-2 (32 / 11.8)^2) ~ 4e-7 of
    it at the farthest plane)."""
    n, w0 = 64, 6 * D
    xc = (np.arange(n) - 32) * D
    X, Y = np.meshgrid(xc, xc)
    u0 = np.exp(-(X ** 2 + Y ** 2) / w0 ** 2)
    zR = np.pi * w0 ** 2 / LAM
    zs = [0.3 * zR, zR, 1.7 * zR]
    I = recon.focal_stack(u0[None, None], D, [LAM], zs, band_limit=False)[0]
    for p, z in enumerate(zs):
        assert abs(I[p, 32, 32] - 1.0 / (1.0 + (z / zR) ** 2)) < 1e-4, z
        assert abs(I[p].sum() / (np.abs(u0) ** 2).sum() - 1.0) < 1e-6


def test_pupil_power_of_a_gaussian_spectrum():
    """The power spectrum of the Gaussian spot is proportional to
    exp(-2 pi^2 w0^2 f^2), so a pupil of cutoff f_c = NA / lambda passes the
    fraction 1 - exp(-2 pi^2 w0^2 f_c^2) of its power (the discrete disc on
    a 512 x 512 frequency grid is within 2 % of the continuous one)."""
    n, w0 = 256, 4 * D
    xc = (np.arange(n) - 128) * D
    X, Y = np.meshgrid(xc, xc)
    u0 = np.exp(-(X ** 2 + Y ** 2) / w0 ** 2)
    for frac_target in (0.3, 0.7):
        fc = np.sqrt(-np.log(1 - frac_target) / (2 * np.pi ** 2 * w0 ** 2))
        I = recon.focal_stack(u0[None, None], D, [LAM], [1e-3], na=fc * LAM, band_limit=False)[0, 0]
        frac = I.sum() / (np.abs(u0) ** 2).sum()
        assert abs(frac - frac_target) < 0.02 * frac_target, (frac, frac_target)
