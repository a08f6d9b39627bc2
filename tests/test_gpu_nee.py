"""Next-event estimation with MIS on the GPU against the FP64 oracle through
the C ABI (Eq. 1 by light sampling and BSDF sampling combined with the power
heuristic): closed-form lit planes (Lambert, GGX, blocked light), the tiny
scene with its quad light, the mixed-material scene with random phases, the
reflected radiance against the form factor, and batches that mix jobs with
and without it. Bar as for the rest of the tracer: >= 99.9 % identical path
signatures (now including each next-event light choice and visibility) and
field error <= 1e-4 x RMS on matched paths."""
import sys

import numpy as np
import pytest

import scenes
from scenes import jobs
from parity_util import compare, gpu_run, oracle_run

pytestmark = pytest.mark.gpu
MM = 1e-3
Z0, H = 5 * MM, 2 * MM
LIGHT = (1 * MM, 3 * MM, -1 * MM, 1 * MM)


@pytest.fixture(scope="module")
def ctx():
    import paper_2606_14173_amd as hpt
    c = hpt.Context(0)
    yield c
    c.close()


def _say(name, r):
    print("%s: paths %d match %.5f err/rms %.2e self %.1e" % (name, r["n_paths"], r["match"], r["err"],
                                                            r["self_err"]))
    sys.stdout.flush()


def _job(**kw):
    j = dict(jobs.JOB_DEFAULTS)
    j.update(width=16, height=16, lambdas=[520e-9], comps=[1], spp=64, max_bounces=2, T=4,
             grf_w=96, grf_h=96, grf_seed=3, phase_mode=jobs.PHASE_SPLIT, nee=1)
    j.update(kw)
    return j


def _parity(ctx, sc, job, name):
    sid = ctx.upload_scene(sc)
    r = compare(*gpu_run(ctx, sid, job), *oracle_run(sc, job))
    ctx.release_scene(sid)
    _say(name, r)
    assert r["ok"] and r["self_err"] < 1e-5, name
    return r


@pytest.mark.parametrize("material,name", [((scenes.LAMBERT, (0.7,) * 3), "lambert"),
                                           ((scenes.GGX, (0.8,) * 3, 0.4), "ggx")])
@pytest.mark.parametrize("bounces", [2, 4])
def test_lit_plane_parity(ctx, material, name, bounces):
    sc = scenes.scene_lit_plane(Z0, material, light=LIGHT, h=H, emit=3.0)
    _parity(ctx, sc, _job(max_bounces=bounces), "%s b=%d" % (name, bounces))


def test_blocked_light_parity(ctx):
    sc = scenes.scene_lit_plane(Z0, (scenes.LAMBERT, (0.7,) * 3), light=LIGHT, h=H, emit=3.0, blocker=True)
    sid = ctx.upload_scene(sc)
    U, rec, _ = gpu_run(ctx, sid, _job())
    ctx.release_scene(sid)
    assert np.all(U == 0)


def test_tiny_scene_parity(ctx):
    sc = scenes.scene_tiny(0)
    job = jobs.job_for_config(0, T=4, nee=1, max_bounces=4, width=48, height=40, spp=16, grf_w=160,
                              grf_h=160, grf_seed=5, phase_mode=jobs.PHASE_SPLIT)
    _parity(ctx, sc, job, "tiny nee")


def test_mid_scene_parity(ctx):
    """The ~58k-triangle mixed-material scene (Lambert, GGX, mirror,
    dielectric, quad light), RGB, T = 8, on a crop."""
    sc = scenes.scene_mid(1)
    job = jobs.job_for_config(1, T=8, nee=1, crop=(236, 236, 40, 36), spp=16)
    _parity(ctx, sc, job, "mid nee")


def test_lambert_plane_form_factor(ctx):
    """Reflected radiance of the lit Lambert plane, per image point, against
    albedo x Le x the point-to-rectangle form factor (mean within 4 SE)."""
    from test_nee_pins import _form_factor
    rho, le = 0.7, 3.0
    sc = scenes.scene_lit_plane(Z0, (scenes.LAMBERT, (rho,) * 3), light=LIGHT, h=H, emit=le)
    job = _job(width=8, height=8, spp=2048, T=1, random_phase=0)
    sid = ctx.upload_scene(sc)
    rec = ctx.trace(sid, job, records=True)[1]
    ctx.release_scene(sid)
    r = rec.reshape(-1)
    L = r["A"].astype(np.float64) ** 2
    d = L - rho * le * _form_factor(r["qx"], r["qy"])
    se = d.std() / np.sqrt(d.size)
    print("form factor: mean diff %.3e, SE %.3e" % (d.mean(), se))
    assert abs(d.mean()) < 4 * se


def test_mixed_modes_match_alone(ctx):
    """Jobs with and without next-event estimation submitted together run in
    separate batches; each result equals the job traced alone, bit for bit."""
    sc = scenes.scene_tiny(0)
    sid = ctx.upload_scene(sc)
    reqs = [jobs.job_for_config(0, T=4, nee=n, seed=7 + n, max_bounces=4, spp=16) for n in (1, 0, 1, 0)]
    alone = [ctx.trace(sid, j) for j in reqs]
    jids = [ctx.submit(sid, j) for j in reqs]
    for jid, j, a in zip(jids, reqs, alone):
        ctx.wait(jid)
        got = ctx.read_field(jid, j)
        ctx.release_job(jid)
        assert np.array_equal(got.view(np.uint32), a.view(np.uint32))
    ctx.release_scene(sid)
