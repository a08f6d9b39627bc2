"""FP64 angular-spectrum propagation (ASM) of recorded fields -- TEST
INFRASTRUCTURE ONLY (tests, smoke check and the benchmark's CPU leg).

Second stage of the two-stage scheme (Sec. 4.4): the field traced onto a wave
recording plane is carried to the hologram plane by the angular spectrum
method (Sec. 3, "Angular Spectrum of Wave Field": the field's Fourier
transform is its plane-wave decomposition). Written from the definition:

  U(f)   = FFT2 of the field, zero-padded on each axis to the next power of
           two >= 2 N (the paper's double zero-padding against wrap-around);
  H(f)   = exp(+i 2 pi z sqrt(1/lambda^2 - |f|^2)) for |f| < 1/lambda, 0 for
           evanescent components (+i: the recorded fields carry exp(+i k r),
           so moving a distance z further from the scene adds k_z z);
  band limit (Matsushima and Shimobaba, Opt. Express 17(22), 2009): H = 0
           where |f_x| > 1 / (lambda sqrt((2 du_x z)^2 + 1)), du_x = 1/(P_x d)
           the padded grid's frequency step (likewise for y), which keeps the
           sampled transfer function free of aliasing;
  u(z)   = IFFT2(U H), cropped to the input's window (top-left corner of
           the padded grid).

Frequencies follow the FFT's order (k / (P d) for k < P/2, (k - P) / (P d)
otherwise). numpy's FFT is the library step.
"""
import numpy as np


def padded_size(n):
    """Padded length of one axis: the next power of two >= 2 n."""
    p = 1
    while p < 2 * n:
        p *= 2
    return p


def freqs(p, pitch):
    return np.fft.fftfreq(p, d=pitch)


def transfer(py, px, pitch, lam, z, band_limit=True):
    """H [py, px] (complex128) on the FFT's frequency grid."""
    fy = freqs(py, pitch)[:, None]
    fx = freqs(px, pitch)[None, :]
    arg = 1.0 / lam ** 2 - fx ** 2 - fy ** 2
    prop = arg > 0
    kz = np.sqrt(np.where(prop, arg, 0.0))
    H = np.where(prop, np.exp(2j * np.pi * z * kz), 0.0)
    if band_limit:
        lim_x = 1.0 / (lam * np.sqrt((2.0 * z / (px * pitch)) ** 2 + 1.0))
        lim_y = 1.0 / (lam * np.sqrt((2.0 * z / (py * pitch)) ** 2 + 1.0))
        H = np.where((np.abs(fx) <= lim_x) & (np.abs(fy) <= lim_y), H, 0.0)
    return H


def propagate(u, pitch, lam, z, pad=True, band_limit=True):
    """Field(s) u [..., h, w] (complex) carried a distance z by the ASM.
    pad=False propagates the given grid as one period (no padding, no crop)."""
    u = np.asarray(u, dtype=np.complex128)
    h, w = u.shape[-2:]
    py, px = (padded_size(h), padded_size(w)) if pad else (h, w)
    buf = np.zeros(u.shape[:-2] + (py, px), dtype=np.complex128)
    buf[..., :h, :w] = u
    H = transfer(py, px, pitch, lam, z, band_limit)
    out = np.fft.ifft2(np.fft.fft2(buf) * H)
    return out[..., :h, :w]


def rs_direct(u0, window, n_quad, lam, z, x, y):
    """Rayleigh-Sommerfeld integral of the first kind of the field u0(x', y')
    (a callable on metre coordinates) at the points (x, y, z): with
    G = exp(i k r) / r, u(P) = (1/2 pi) integral u0 (z / r) (1/r - i k) G dA,
    by the midpoint rule on an n_quad x n_quad grid over the window
    (x_lo, x_hi, y_lo, y_hi). Used only as an independent check of the ASM
    (ASM and RS-I coincide for a field band-limited inside the window)."""
    k = 2 * np.pi / lam
    x_lo, x_hi, y_lo, y_hi = window
    dx, dy = (x_hi - x_lo) / n_quad, (y_hi - y_lo) / n_quad
    X, Y = np.meshgrid(x_lo + (np.arange(n_quad) + 0.5) * dx, y_lo + (np.arange(n_quad) + 0.5) * dy)
    f = u0(X, Y)
    out = []
    for px_, py_ in zip(np.atleast_1d(x), np.atleast_1d(y)):
        r = np.sqrt((px_ - X) ** 2 + (py_ - Y) ** 2 + z ** 2)
        K = (z / r) * (1.0 / r - 1j * k) * np.exp(1j * k * r) / r / (2 * np.pi)
        out.append(np.sum(f * K) * dx * dy)
    return np.array(out)
