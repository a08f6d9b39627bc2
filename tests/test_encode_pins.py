"""Pins of the oracle's phase-only encoding (complex-amplitude supervision on
one plane with a phase-shift-invariant scale factor, optimised by Adam;
Sec. 2 and Sec. 5.3) against what the mathematics fixes: the adjoint of the
propagation, the gradient by finite differences, the optimal scale, the
invariances of the loss, Adam's published update, and convergence on a
target that a phase-only SLM can produce exactly."""
import numpy as np
import pytest

from oracle import asm, encode

D, LAM = 8e-6, 520e-9


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


@pytest.mark.parametrize("band_limit", [True, False])
def test_adjoint_is_propagation_by_minus_z(band_limit):
    """<P_z x, y> = <x, P_{-z} y> for the padded, cropped ASM."""
    x, y = _rand((21, 34), 1), _rand((21, 34), 2)
    z = 30e-3
    lhs = np.vdot(asm.propagate(x, D, LAM, z, band_limit=band_limit), y)
    rhs = np.vdot(x, asm.propagate(y, D, LAM, -z, band_limit=band_limit))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    h, w, z = 12, 15, 4e-3
    V = asm.propagate(_rand((h, w), 4), D, LAM, z)
    phi = rng.uniform(-np.pi, np.pi, size=(h, w))
    g, L = encode.gradient(phi, V, D, LAM, z)
    eps = 1e-6
    for (i, j) in [(0, 0), (5, 7), (11, 14), (3, 12)]:
        p1, p0 = phi.copy(), phi.copy()
        p1[i, j] += eps
        p0[i, j] -= eps
        _, L1 = encode.scale_and_loss(encode.forward(p1, D, LAM, z), V)
        _, L0 = encode.scale_and_loss(encode.forward(p0, D, LAM, z), V)
        fd = (L1 - L0) / (2 * eps)
        assert abs(fd - g[i, j]) < 1e-6 * max(1.0, abs(fd)), (i, j, fd, g[i, j])


def test_optimal_scale_and_invariances():
    """s minimises ||A - s V|| (no complex factor does better); the loss does
    not change when the target is multiplied by any complex constant or the
    phase pattern is shifted by a constant."""
    A, V = _rand((9, 11), 5), _rand((9, 11), 6)
    s, L = encode.scale_and_loss(A, V)
    rng = np.random.default_rng(7)
    for d in rng.normal(size=(20, 2)) * 0.1:
        s2 = s + d[0] + 1j * d[1]
        assert np.sum(np.abs(A - s2 * V) ** 2) > L
    _, L2 = encode.scale_and_loss(A, (0.3 - 2.1j) * V)
    assert abs(L2 - L) < 1e-12 * L
    U = _rand((10, 13), 8)
    Vt = asm.propagate(U, D, LAM, 2e-3)
    phi = rng.uniform(-np.pi, np.pi, size=(10, 13))
    r0 = encode.relative_loss(phi, Vt, D, LAM, 2e-3)
    r1 = encode.relative_loss(phi + 1.234, Vt, D, LAM, 2e-3)
    assert abs(r0 - r1) < 1e-12 and 0 <= r0 <= 1


def test_adam_update_on_a_scalar_quadratic():
    """Adam's first step moves every coordinate by lr against its gradient's
    sign (bias-corrected m / sqrt(v) = sign g); later steps follow the
    recursions of the published algorithm, written out here for f = x^2 / 2."""
    x = np.array([3.0, -0.5, 1e-3])
    m = np.zeros(3)
    v = np.zeros(3)
    x1, m, v = encode.adam(x, x, m, v, 1, 0.1)
    assert np.allclose(x1, x - 0.1 * np.sign(x) * np.abs(x) / (np.abs(x) + 1e-8), rtol=1e-12)
    # second step by hand
    g = x1
    m2 = 0.9 * (0.1 * x) + 0.1 * g
    v2 = 0.999 * (0.001 * x * x) + 0.001 * g * g
    expect = x1 - 0.1 * (m2 / (1 - 0.81)) / (np.sqrt(v2 / (1 - 0.999 ** 2)) + 1e-8)
    x2, _, _ = encode.adam(x1, g, m, v, 2, 0.1)
    assert np.allclose(x2, expect, rtol=1e-12)


def test_reaches_a_phase_only_target():
    """The target is the field of a phase-only pattern phi*: starting from a
    perturbed phase, the relative loss falls by orders of magnitude (a
    wrong-sign gradient or adjoint makes it rise)."""
    rng = np.random.default_rng(9)
    h, w, z = 24, 24, 3e-3
    phi_star = rng.uniform(-np.pi, np.pi, size=(h, w))
    U = np.exp(1j * phi_star)
    start = phi_star + rng.normal(size=(h, w)) * 0.5
    V = asm.propagate(U, D, LAM, z)
    l0 = encode.relative_loss(start, V, D, LAM, z)
    phi, l1 = encode.encode(U, D, LAM, z, 150, 0.05, phi0=start)
    assert l0 > 0.05 and l1 < 1e-2 * l0, (l0, l1)
