"""Pins of the oracle's angular-spectrum propagation (second stage of the
two-stage scheme, Sec. 4.4; angular spectrum, Sec. 3) against what the
mathematics fixes: the Rayleigh-Sommerfeld integral it must reproduce, plane
waves, unitarity, reversibility, evanescent waves, and the Nyquist criterion
behind the band limit."""
import numpy as np
import pytest

from oracle import asm

D, LAM = 8e-6, 520e-9


def test_padded_size():
    assert [asm.padded_size(n) for n in (1, 2, 3, 64, 100, 1080, 1920)] == [2, 4, 8, 128, 256, 4096, 4096]


def test_identity_at_zero_distance():
    rng = np.random.default_rng(0)
    u = rng.normal(size=(2, 30, 41)) + 1j * rng.normal(size=(2, 30, 41))
    out = asm.propagate(u, D, LAM, 0.0)
    assert np.abs(out - u).max() < 1e-12 * np.abs(u).max()


@pytest.mark.parametrize("z,sig_px", [(2e-3, 2.0), (0.5e-3, 2.0), (6e-3, 2.5)])
def test_matches_rayleigh_sommerfeld_integral(z, sig_px):
    """A Gaussian spot sampled well above Nyquist (its spectrum at the grid's
    Nyquist frequency is below 1e-8): the padded ASM equals the
    first-kind RS integral of the continuous spot (fine midpoint quadrature)."""
    n = 64
    sig = sig_px * D
    xc = (np.arange(n) + 0.5) * D - n * D / 2
    X, Y = np.meshgrid(xc, xc)
    g = lambda x, y: np.exp(-(x ** 2 + y ** 2) / (2 * sig ** 2))  # noqa: E731
    out = asm.propagate(g(X, Y), D, LAM, z)
    idx = [(32, 32), (32, 35), (30, 36), (28, 28), (33, 40), (20, 44)]
    ref = asm.rs_direct(g, (-9 * sig, 9 * sig, -9 * sig, 9 * sig), 900, LAM, z,
                        [xc[j] for i, j in idx], [xc[i] for i, j in idx])
    got = np.array([out[i, j] for i, j in idx])
    assert np.abs(got - ref).max() < 1e-7 * np.abs(ref).max()


def test_plane_waves_pick_up_k_z_cos_theta():
    """On one period of the grid (no padding) a plane wave of spatial
    frequency f tilted by sin(theta) = lambda |f| is multiplied by
    exp(i k z cos(theta))."""
    ny, nx, z = 16, 32, 3.7e-3
    y, x = np.meshgrid(np.arange(ny) * D, np.arange(nx) * D, indexing="ij")
    for kx, ky in [(0, 0), (3, 0), (-5, 2), (15, -7), (-16, -8), (1, 7)]:
        fx, fy = kx / (nx * D), ky / (ny * D)
        u = np.exp(2j * np.pi * (fx * x + fy * y))
        out = asm.propagate(u, D, LAM, z, pad=False, band_limit=False)
        sin_t = LAM * np.hypot(fx, fy)
        expect = u * np.exp(1j * (2 * np.pi / LAM) * z * np.sqrt(1 - sin_t ** 2))
        assert np.abs(out - expect).max() < 1e-9, (kx, ky)


def test_unitary_and_reversible_on_one_period():
    rng = np.random.default_rng(1)
    u = rng.normal(size=(24, 40)) + 1j * rng.normal(size=(24, 40))
    z = 11e-3
    out = asm.propagate(u, D, LAM, z, pad=False, band_limit=False)
    assert abs(np.sum(np.abs(out) ** 2) / np.sum(np.abs(u) ** 2) - 1) < 1e-12
    back = asm.propagate(out, D, LAM, -z, pad=False, band_limit=False)
    assert np.abs(back - u).max() < 1e-10 * np.abs(u).max()


def test_evanescent_components_are_dropped():
    """With a pitch finer than lambda/2 the grid holds frequencies beyond
    1/lambda; those do not propagate."""
    d, n = 0.2e-6, 32
    x = np.arange(n) * d
    X = np.tile(x, (4, 1))
    f_ev = 12 / (n * d)              # lambda f = 0.975: still propagating
    f_far = 15 / (n * d)             # lambda f = 1.22: evanescent
    assert LAM * f_ev < 1 < LAM * f_far
    keep = asm.propagate(np.exp(2j * np.pi * f_ev * X), d, LAM, 1e-6, pad=False, band_limit=False)
    gone = asm.propagate(np.exp(2j * np.pi * f_far * X), d, LAM, 1e-6, pad=False, band_limit=False)
    assert np.allclose(np.abs(keep), 1.0, atol=1e-12)
    assert np.abs(gone).max() < 1e-12


def test_band_limit_is_the_nyquist_limit_of_the_sampled_transfer_function():
    """The band limit keeps exactly the frequency samples at which the
    sampled transfer function's phase advances by at most pi per sample
    (beyond that the chirp aliases on the padded grid)."""
    p, z = 128, 40e-3
    Hfull = asm.transfer(p, p, D, LAM, z, band_limit=False)[0]     # f_y = 0 row
    Hlim = asm.transfer(p, p, D, LAM, z, band_limit=True)[0]
    f = asm.freqs(p, D)
    order = np.argsort(f)
    f, Hfull, Hlim = f[order], Hfull[order], Hlim[order]
    kept = np.abs(Hlim) > 0
    assert 2 < kept.sum() < p            # the limit is active at this distance
    # exact phase of the transfer function (unwrapped), advance per sample
    phase = 2 * np.pi * z * np.sqrt(1 / LAM ** 2 - f ** 2)
    step = np.abs(np.diff(phase))        # between f[k] and f[k+1]
    mid = np.searchsorted(f, 0.0)
    for k in range(len(f)):
        inner = k + 1 if k < mid else k - 1      # neighbour toward f = 0
        if inner < 0 or inner >= len(f) or k == mid:
            continue
        s = step[min(k, inner)]
        if kept[k]:
            assert s <= np.pi * (1 + 1e-9), (k, s)
        elif kept[inner]:                # first sample past the limit
            assert s > np.pi * 0.95, (k, s)
    # Hlim equals Hfull where kept
    assert np.allclose(Hlim[kept], Hfull[kept])
