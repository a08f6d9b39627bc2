"""Pins of the oracle's next-event estimation with multiple importance
sampling in the incoherent tail (the variance-reduction step the paper's
Mitsuba-based tracer uses; Eq. 1 estimated by light sampling and BSDF
sampling combined with the power heuristic). Fixed by the mathematics:

* a Lambert plane lit by a rectangular emitter: the reflected radiance is
  albedo x Le x the point-to-parallel-rectangle form factor (closed form),
  per image point, with and without next-event estimation;
* a GGX plane: light sampling and BSDF sampling are both unbiased, so their
  means agree (a wrong f cos or pdf in either breaks it);
* a black sheet between plane and light leaves nothing;
* light sampling cuts the variance for a small light.
"""
import numpy as np
import pytest

import oracle
import scenes
from scenes import jobs

LAM = 520e-9
MM = 1e-3
Z0, H = 5 * MM, 2 * MM
LIGHT = (1 * MM, 3 * MM, -1 * MM, 1 * MM)


@pytest.fixture(scope="module")
def oracle_lib():
    return oracle


def _job(**kw):
    j = dict(jobs.JOB_DEFAULTS)
    j.update(width=8, height=8, lambdas=[LAM], comps=[1], spp=1024, max_bounces=2, T=1,
             random_phase=0, grf_w=64, grf_h=64)
    j.update(kw)
    return j


def _grf_dummy(job):
    return np.ones((job["grf_h"], job["grf_w"], job["T"]), dtype=np.complex128)


def _corner(X, Y, h):
    """Form factor from a point to a parallel rectangle [0, X] x [0, Y] at
    height h above it, one corner over the point (signed sides)."""
    x, y = np.abs(X) / h, np.abs(Y) / h
    ax, ay = np.sqrt(1 + x * x), np.sqrt(1 + y * y)
    f = (x / ax * np.arctan(y / ax) + y / ay * np.arctan(x / ay)) / (2 * np.pi)
    return np.sign(X) * np.sign(Y) * f


def _form_factor(px, py):
    x1, x2, y1, y2 = LIGHT
    return (_corner(x2 - px, y2 - py, H) - _corner(x1 - px, y2 - py, H)
            - _corner(x2 - px, y1 - py, H) + _corner(x1 - px, y1 - py, H))


def _lhat(sc, **kw):
    o = oracle.OracleScene(sc)
    job = _job(**kw)
    _, recs, _ = oracle.trace(o, job, grf=_grf_dummy(job), records=True)
    r = recs.reshape(-1)
    return r, r["A"] ** 2   # image point directly on the plane: beta_pre = 1


@pytest.mark.parametrize("nee", [1, 0])
def test_lambert_plane_form_factor(oracle_lib, nee):
    rho, le = 0.7, 3.0
    sc = scenes.scene_lit_plane(Z0, (scenes.LAMBERT, (rho,) * 3), light=LIGHT, h=H, emit=le)
    r, L = _lhat(sc, nee=nee, spp=2048 if nee else 8192)
    assert (r["bP"] == 1).all()
    expect = rho * le * _form_factor(r["qx"], r["qy"])
    d = L - expect
    se = d.std() / np.sqrt(d.size)
    assert abs(d.mean()) < 4 * se, (d.mean(), se)
    assert se < 0.02 * expect.mean()


def test_ggx_plane_light_and_bsdf_sampling_agree(oracle_lib):
    """The light at 56-68 degrees from the normal, where the masking of the
    light direction (G1(L) = 0.7-0.85) matters: dropping it from f cos
    biases the light-sampled mean by several standard errors."""
    grazing = (3 * MM, 5 * MM, -1 * MM, 1 * MM)
    sc = scenes.scene_lit_plane(Z0, (scenes.GGX, (0.8,) * 3, 0.6), light=grazing, h=H, emit=2.0)
    _, Ln = _lhat(sc, nee=1, spp=4096)
    _, Lb = _lhat(sc, nee=0, spp=32768)
    se = np.sqrt(Ln.var() / Ln.size + Lb.var() / Lb.size)
    assert Ln.mean() > 40 * se
    assert abs(Ln.mean() - Lb.mean()) < 4 * se, (Ln.mean(), Lb.mean(), se)


def test_blocked_light_gives_nothing(oracle_lib):
    sc = scenes.scene_lit_plane(Z0, (scenes.LAMBERT, (0.7,) * 3), light=LIGHT, h=H, emit=3.0,
                                blocker=True)
    r, L = _lhat(sc, nee=1, spp=256)
    assert np.all(L == 0)


def test_light_sampling_reduces_variance(oracle_lib):
    small = (1.8 * MM, 2.0 * MM, -0.1 * MM, 0.1 * MM)
    rho, le = 0.7, 50.0
    sc = scenes.scene_lit_plane(Z0, (scenes.LAMBERT, (rho,) * 3), light=small, h=H, emit=le)
    _, Ln = _lhat(sc, nee=1, spp=512)
    _, Lb = _lhat(sc, nee=0, spp=512)
    assert Ln.var() < 0.05 * Lb.var()


def test_nee_off_leaves_paths_unchanged(oracle_lib):
    """With nee = 0 the estimator and signatures are the plain BSDF-sampling
    ones: emission is only collected by lobe samples, at full weight."""
    sc = scenes.scene_lit_plane(Z0, (scenes.LAMBERT, (0.7,) * 3), light=LIGHT, h=H, emit=3.0)
    r, L = _lhat(sc, nee=0, spp=256)
    hit_light = r["kind"] == 3
    assert hit_light.any() and np.all(L[~hit_light] == 0)
    assert np.allclose(L[hit_light], float(np.float32(0.7)) * 3.0, rtol=1e-12)
