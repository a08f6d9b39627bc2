"""FP64 phase-only hologram encoding -- TEST INFRASTRUCTURE ONLY (tests,
smoke check and the benchmark's CPU leg).

The rendered complex field is turned into a phase-only SLM pattern by
stochastic-gradient optimisation under complex-amplitude supervision on one
reconstruction plane, with a phase-shift-invariant scale factor (abstract;
Sec. 2, hologram encoding; Sec. 5.3, phase-only hologram encoding). The
supplement with the details is not available; the reading implemented here:

  a   = exp(i phi)                the SLM's phase-only field, [h][w]
  A   = P_z a                     its field at the supervision plane (the
                                  padded, optionally band-limited ASM of
                                  oracle.asm, distance z)
  V   = P_z U                     the target: the rendered field U carried to
                                  the same plane
  s   = <V, A> / <V, V>           the complex factor that best matches s V to
                                  A (<x, y> = sum conj(x) y): the target's
                                  global amplitude and phase are free
  L   = || A - s V ||^2           summed over the window
  dL/dphi = 2 Im( G conj(a) ),    G = P_z^H (A - s V) = P_{-z} (A - s V)
                                  (s is optimal, so its own variation drops
                                  out; the ASM's adjoint conjugates the
                                  transfer function, which is H at -z)
  phi_0 = arg U                   (0 where U = 0)
  Adam (Kingma and Ba, ICLR 2015), beta1 = 0.9, beta2 = 0.999, eps = 1e-8,
  step size lr; K steps.

Reported loss: L / ||A||^2 = 1 - |<V, A>|^2 / (||V||^2 ||A||^2) of the final
phase (scale-free, in [0, 1]).
"""
import numpy as np

from . import asm

BETA1, BETA2, EPS = 0.9, 0.999, 1e-8


def forward(phi, pitch, lam, z, band_limit=True):
    return asm.propagate(np.exp(1j * phi), pitch, lam, z, band_limit=band_limit)


def scale_and_loss(A, V):
    """Optimal complex s per field and L = ||A - s V||^2 (arrays [..., h, w])."""
    dot = np.sum(np.conj(V) * A, axis=(-2, -1))
    vv = np.sum(np.abs(V) ** 2, axis=(-2, -1))
    s = dot / vv
    L = np.sum(np.abs(A - s[..., None, None] * V) ** 2, axis=(-2, -1))
    return s, L


def gradient(phi, V, pitch, lam, z, band_limit=True):
    """dL/dphi at phi (and L), from the adjoint propagation."""
    a = np.exp(1j * phi)
    A = asm.propagate(a, pitch, lam, z, band_limit=band_limit)
    s, L = scale_and_loss(A, V)
    G = asm.propagate(A - s[..., None, None] * V, pitch, lam, -z, band_limit=band_limit)
    return 2.0 * np.imag(G * np.conj(a)), L


def relative_loss(phi, V, pitch, lam, z, band_limit=True):
    A = forward(phi, pitch, lam, z, band_limit)
    _, L = scale_and_loss(A, V)
    return L / np.sum(np.abs(A) ** 2, axis=(-2, -1))


def adam(phi, g, m, v, k, lr):
    """One Adam step (k = 1, 2, ...); returns the new phi, m, v."""
    m = BETA1 * m + (1 - BETA1) * g
    v = BETA2 * v + (1 - BETA2) * g * g
    mh = m / (1 - BETA1 ** k)
    vh = v / (1 - BETA2 ** k)
    return phi - lr * mh / (np.sqrt(vh) + EPS), m, v


def encode(U, pitch, lam, z, iterations, lr, band_limit=True, phi0=None):
    """U [..., h, w] complex (rendered SLM-plane fields) -> (phi [..., h, w],
    relative loss per field of the final phi)."""
    U = np.asarray(U, dtype=np.complex128)
    V = asm.propagate(U, pitch, lam, z, band_limit=band_limit)
    phi = np.angle(U) if phi0 is None else np.array(phi0, dtype=np.float64)
    m = np.zeros_like(phi)
    v = np.zeros_like(phi)
    for k in range(1, iterations + 1):
        g, _ = gradient(phi, V, pitch, lam, z, band_limit)
        phi, m, v = adam(phi, g, m, v, k, lr)
    return phi, relative_loss(phi, V, pitch, lam, z, band_limit)
