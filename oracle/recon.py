"""FP64 focal-stack reconstruction of recorded fields -- TEST INFRASTRUCTURE
ONLY (tests, smoke check and the benchmark's CPU leg).

Simulated viewing of a hologram, as in the paper's display set-up (Sec. 5.3,
physical configuration): the field is carried to several observation planes
(the paper uses five planes 1.25 mm apart within 80-85 mm of the SLM), an
iris between eyepiece and camera filters the angular spectrum (pupil
filtering), and the T random-phase frames are shown in turn and averaged by
the eye or sensor (time multiplexing), i.e. their intensities add:

  I_c,p(x) = (1/T) sum_t | IFFT2( FFT2(pad U_c,t) H_{lambda_c, d_p} P_{lambda_c} ) (x) |^2

H: the angular-spectrum transfer function of oracle.asm (evanescent cut,
optional band limit); P: the pupil, 1 where lambda |f| <= NA and 0 elsewhere
(a circular aperture that passes plane waves up to the angle asin(NA)); NA
<= 0 means no pupil. The paper gives no aperture size in the main text, so NA
is an argument. numpy's FFT is the library step.
"""
import numpy as np

from . import asm


def pupil(py, px, pitch, lam, na):
    """P [py, px] on the FFT's frequency grid (all ones when na <= 0)."""
    fy = asm.freqs(py, pitch)[:, None]
    fx = asm.freqs(px, pitch)[None, :]
    if na <= 0:
        return np.ones((py, px))
    return ((fx ** 2 + fy ** 2) * lam ** 2 <= na ** 2).astype(np.float64)


def focal_stack(U, pitch, lambdas, distances, na=0.0, band_limit=True, pad=True):
    """U [n_ch][T][h][w] complex -> I [n_ch][n_planes][h][w] float64, the
    frame-averaged intensity at each distance. pad=False propagates the grid
    as one period (no padding, no crop)."""
    U = np.asarray(U, dtype=np.complex128)
    n_ch, T, h, w = U.shape
    py, px = (asm.padded_size(h), asm.padded_size(w)) if pad else (h, w)
    out = np.zeros((n_ch, len(distances), h, w))
    for c in range(n_ch):
        buf = np.zeros((T, py, px), dtype=np.complex128)
        buf[:, :h, :w] = U[c]
        spec = np.fft.fft2(buf)
        for p, z in enumerate(distances):
            H = asm.transfer(py, px, pitch, lambdas[c], z, band_limit) * pupil(py, px, pitch, lambdas[c], na)
            u = np.fft.ifft2(spec * H)[:, :h, :w]
            out[c, p] = np.mean(np.abs(u) ** 2, axis=0)
    return out
