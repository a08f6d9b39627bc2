"""Band-limited random phase tables of Eq. 4 (Sec. 4.3) for the oracle.

r_t(x, y) = sum over passband bins of exp(i xi_t) exp(2 pi i (f_x x + f_y y)),
sampled on the periodic grid of pitch d; phi_t = arg r_t. The spectral phases
xi_t come from the oracle's counter-based generator; the inverse transform is
numpy's FFT (a library step). Values are scaled by 1/sqrt(#passband bins) so
that E|r|^2 = 1; the scale does not change the phase.

The tables are stored as complex64: the FP64 inverse transform, each value
rounded once to complex64 (the precision a table is held in). Sec. 4.3
takes phi_t as the argument of r_t at the image point, which is
ill-conditioned near the zeros of r_t (an error e in r moves the phase by
about e / |r|), so the lookup must interpolate the same stored values on
both sides; it then works in FP64 on them.
"""
import numpy as np

from . import _lib


def grf_phases(gw, gh, t0, nt, seed):
    """Spectral phases xi [nt, gh, gw] of frames t0..t0+nt-1 and the passband mask."""
    xi = np.zeros((nt, gh, gw), dtype=np.float64)
    mask = np.zeros((nt, gh, gw), dtype=np.uint8)
    _lib.lib().oracle_grf_phases(int(gw), int(gh), int(t0), int(nt), int(seed),
                                 xi.ctypes.data, mask.ctypes.data)
    return xi, mask.astype(bool)


def grf_table(gw, gh, T, seed, stored=True):
    """Complex table [gh, gw, T] (complex128 array): frame t at texel (i, j);
    stored=True: the values as stored (rounded to complex64), False: the
    FP64 transform itself."""
    out = np.empty((gh, gw, T), dtype=np.complex128)
    for t in range(T):
        xi, mask = grf_phases(gw, gh, t, 1, seed)
        scale = (gw * gh) / np.sqrt(int(mask[0].sum()))
        spec = np.where(mask[0], np.exp(1j * xi[0]), 0.0)
        out[:, :, t] = np.fft.ifft2(spec) * scale
    if stored:
        out = out.astype(np.complex64).astype(np.complex128)
    return out
