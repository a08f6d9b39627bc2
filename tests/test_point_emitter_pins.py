"""Pins of the oracle's point emitter (Eq. 2 for a source concentrated at one
point: the spherical wave exp(ikr)/r) and of its weight readings, against
closed forms computed here from the geometry alone: pixel centres, the
recordable cone sin(theta) <= lambda/2d (Sec. 4.1), the shadow of an
analytic sphere by point-to-segment distance, and the hologram-from-world
transform of Eq. 3."""
import math

import numpy as np
import pytest

import oracle
import scenes
from scenes import jobs

LAM = 520e-9
PITCH = 8e-6
S = LAM / (2 * PITCH)


def _job(**kw):
    j = dict(jobs.JOB_DEFAULTS)
    j.update(width=40, height=36, lambdas=[LAM], comps=[1], spp=1, max_bounces=2, T=1,
             random_phase=0, grf_w=64, grf_h=64)
    j.update(kw)
    return j


def _pixels(job):
    W, H = job["width"], job["height"]
    x = ((np.arange(W) + 0.5) - W / 2) * PITCH
    y = ((np.arange(H) + 0.5) - H / 2) * PITCH
    return np.meshgrid(x, y)


def _closed_form(job, pts, comp, shift, sphere=None, margin=1e-9):
    """sum_e a_e exp(i k r_e) / r_e over the emitters in the cone and not
    shadowed; also the mask of pixels whose cone or shadow decision is
    within `margin` (relative) of its boundary for some emitter."""
    X, Y = _pixels(job)
    k = 2 * np.pi / job["lambdas"][0]
    U = np.zeros(X.shape, complex)
    unsure = np.zeros(X.shape, bool)
    for p in pts:
        y = np.array(p[:3], float)
        a = float(np.float32(p[3 + comp]))
        q = y + shift                                       # hologram space (a translation T)
        dx, dy, dz = q[0] - X, q[1] - Y, q[2]
        r = np.sqrt(dx * dx + dy * dy + dz * dz)
        sin_t = np.sqrt(dx * dx + dy * dy) / r
        inside = (sin_t <= S) & (dz > 0)
        unsure |= np.abs(sin_t - S) < margin
        if sphere is not None:
            c, R = np.array(sphere[:3], float), float(sphere[3])
            # world-space segment from the pixel (T^-1 x_p) to the emitter
            ox, oy, oz = X - shift[0], Y - shift[1], -shift[2]
            sx, sy, sz = y[0] - ox, y[1] - oy, y[2] - oz
            L2 = sx * sx + sy * sy + sz * sz
            tt = np.clip(((c[0] - ox) * sx + (c[1] - oy) * sy + (c[2] - oz) * sz) / L2, 0, 1)
            dist = np.sqrt((ox + tt * sx - c[0]) ** 2 + (oy + tt * sy - c[1]) ** 2 + (oz + tt * sz - c[2]) ** 2)
            shadow = dist < R
            unsure |= np.abs(dist - R) < margin * R
            inside &= ~shadow
        U += np.where(inside, a * np.exp(1j * k * r) / r, 0)
    return U, unsure


PTS = [(30e-6, -20e-6, 2.0e-3, 0.7, 1.3, 0.4),
       (-90e-6, 60e-6, 3.1e-3, 0.2, 0.9, 1.1),
       (150e-6, 40e-6, 1.2e-3, 0.5, 0.0, 0.3)]


def _f32(pts):
    return [tuple(float(v) for v in np.float32(p)) for p in pts]


@pytest.mark.parametrize("comp", [0, 1])
def test_point_emitters_spherical_waves(oracle_lib, comp):
    """Three point emitters, no occluder, translated hologram frame: the
    field is the sum of exp(ikr)/r over the emitters whose direction from the
    pixel lies in the recordable cone, exactly (FP64 rounding), and 0 for
    the others (both sides of the cone edge are present)."""
    shift = np.array([12e-6, -7e-6, 0.35e-3])
    sc = scenes.scene_point_emitters(PTS)
    job = _job(comps=[comp], holo_from_world=(1, 0, 0, shift[0], 0, 1, 0, shift[1], 0, 0, 1, shift[2]))
    U, _, _ = oracle.trace(oracle.OracleScene(sc), job, grf=np.ones((64, 64, 1), complex))
    ref, unsure = _closed_form(job, _f32(PTS), comp, shift)
    assert not unsure.any()
    n_lit = (np.abs(ref) > 0).sum()
    assert 100 < n_lit < ref.size             # the cone edges cross the window
    assert np.abs(U[0, 0] - ref).max() <= 1e-12 * np.abs(ref).max()


def test_point_emitter_sphere_shadow(oracle_lib):
    """A sphere between an emitter and the SLM removes exactly the pixels
    whose segment to the emitter passes within the sphere's radius (analytic
    point-to-segment distance); the others keep the spherical wave."""
    pts = [(10e-6, 5e-6, 3.0e-3, 1.0, 1.0, 1.0)]
    sph = (40e-6, 0.0, 1.5e-3, 60e-6)
    sc = scenes.scene_point_emitters(pts, occluder=sph)
    job = _job()
    U, _, _ = oracle.trace(oracle.OracleScene(sc), job, grf=np.ones((64, 64, 1), complex))
    sph32 = tuple(float(v) for v in np.float32(sph))
    ref, unsure = _closed_form(job, _f32(pts), 1, np.zeros(3), sphere=sph32, margin=1e-7)
    free, _ = _closed_form(job, _f32(pts), 1, np.zeros(3))
    shadowed = (np.abs(free) > 0) & (np.abs(ref) == 0)
    assert shadowed.sum() > 50 and (np.abs(ref) > 0).sum() > 50
    ok = ~unsure
    assert np.abs(U[0, 0] - ref)[ok].max() <= 1e-12 * np.abs(ref).max()


def test_point_emitter_frames_and_chunks(oracle_lib):
    """Path Reuse on the exact term: every frame has the same magnitude and
    frame t carries the random-field phasor at Q; a job adds the term once,
    in the sample range that starts at 0 (chunks still sum to the whole)."""
    pts = [(20e-6, 10e-6, 2.5e-3, 1.0, 1.0, 1.0)]
    sc = scenes.scene_point_emitters(pts)
    o = oracle.OracleScene(sc)
    job = _job(T=4, random_phase=1, grf_w=48, grf_h=44, spp=6)
    grf = oracle.grf_table(48, 44, 4, 3)
    U, _, _ = oracle.trace(o, job, grf=grf)
    mag = np.abs(U[0])
    assert np.allclose(mag, mag[0], rtol=1e-12, atol=0)
    q = np.float32(pts[0][:3]).astype(float)
    for t in range(4):
        ph = oracle.grf_lookup(job, grf, t, q[0], q[1])
        ref, _ = _closed_form(dict(job), _f32(pts), 1, np.zeros(3))
        assert np.abs(U[0, t] - ref * ph).max() <= 1e-12 * np.abs(ref).max()
    parts = [oracle.trace(o, dict(job, spp_begin=a, spp_end=b), grf=grf)[0] for a, b in ((0, 2), (2, 6))]
    assert np.abs(parts[1]).max() == 0
    assert np.allclose(parts[0] + parts[1], U, rtol=0, atol=1e-15 * np.abs(U).max())


def test_weight_reading_P_is_eq5_as_printed(oracle_lib):
    """Reading P (Eq. 5 as printed, no weight) takes the same paths and
    phases as reading R and drops only the weight W = r / p(v), with
    p(v) = v_z / (pi s^2) the disc density per unit solid angle: per path
    amp_R = amp_P * r pi s^2 / v_z, where v_z follows from the image point."""
    sc = scenes.scene_lambert_plane(2e-3, (0.5,) * 3, env=1.0, half=3e-3)
    o = oracle.OracleScene(sc)
    job = _job(width=12, height=10, spp=8, random_phase=0)
    _, rR, _ = oracle.trace(o, job, grf=np.ones((64, 64, 1), complex), records=True)
    _, rP, _ = oracle.trace(o, dict(job, weight_mode=1), grf=np.ones((64, 64, 1), complex), records=True)
    assert np.array_equal(rR["sig"], rP["sig"]) and np.array_equal(rR["rev"], rP["rev"])
    img = rR["amp"] != 0
    assert img.sum() > 100
    X, Y = _pixels(job)
    xp = np.broadcast_to(X[None, :, :, None], rR.shape)[img]
    yp = np.broadcast_to(Y[None, :, :, None], rR.shape)[img]
    r = rR["r"][img]
    al, be = (rR["qx"][img] - xp) / r, (rR["qy"][img] - yp) / r
    vz = np.sqrt(1 - al * al - be * be)
    assert np.allclose(rP["W"][img], 1.0, rtol=0, atol=0)
    assert np.allclose(rR["amp"][img], rP["amp"][img] * r * math.pi * S * S / vz, rtol=1e-9)
