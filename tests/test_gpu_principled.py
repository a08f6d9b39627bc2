"""Principled reflectance on the GPU (Burley diffuse, GGX specular, GTR1
clearcoat, one-sample MIS over the lobes) against the FP64 oracle through the
C ABI: a principled sphere in a uniform environment and a principled plane
under a rectangular light with and without next-event estimation, over the
parameter corners. Bar: >= 99.9 % identical path signatures (the sampled lobe
is part of them) and field error <= 1e-4 x RMS on matched paths."""
import sys

import numpy as np
import pytest

import scenes
from scenes import jobs
from parity_util import compare, gpu_run, oracle_run

pytestmark = pytest.mark.gpu
MM = 1e-3

# (base, roughness, metallic, specular, clearcoat, clearcoat gloss)
PARAMS = [(0.7, 0.5, 0.0, 0.5, 0.0, 1.0),
          (0.4, 0.8, 0.3, 0.8, 0.6, 0.0),
          (0.9, 0.3, 1.0, 0.5, 0.0, 1.0),
          (0.2, 0.7, 0.0, 0.2, 1.0, 0.7)]


@pytest.fixture(scope="module")
def ctx():
    import paper_2606_14173_amd as hpt
    c = hpt.Context(0)
    yield c
    c.close()


def _principled(sc, k, params):
    """Scene sc with material k made principled with params."""
    base, r, m, s, c, g = params
    sc = {key: np.array(v, copy=True) for key, v in sc.items()}
    sc["mat_type"][k] = scenes.PRINCIPLED
    sc["mat_rgb"][k] = base
    sc["mat_rough"][k] = r
    sc["mat_pbr"][k] = (m, s, c, g)
    return sc


def _job(**kw):
    j = dict(jobs.JOB_DEFAULTS)
    j.update(width=16, height=16, lambdas=[520e-9], comps=[1], spp=64, max_bounces=4, T=4,
             grf_w=96, grf_h=96, grf_seed=3, phase_mode=jobs.PHASE_SPLIT)
    j.update(kw)
    return j


def _parity(ctx, sc, job, name):
    sid = ctx.upload_scene(sc)
    r = compare(*gpu_run(ctx, sid, job), *oracle_run(sc, job))
    ctx.release_scene(sid)
    print("%s: paths %d match %.5f err/rms %.2e self %.1e" % (name, r["n_paths"], r["match"], r["err"],
                                                            r["self_err"]))
    sys.stdout.flush()
    assert r["ok"] and r["self_err"] < 1e-5, name


@pytest.mark.parametrize("params", PARAMS)
def test_sphere_in_environment(ctx, params):
    sc = _principled(scenes.scene_furnace_sphere(3e-3, 1e-3, env=1.0), 0, params)
    _parity(ctx, sc, _job(), "sphere %s" % (params,))


@pytest.mark.parametrize("params", PARAMS)
@pytest.mark.parametrize("nee", [0, 1])
def test_lit_plane(ctx, params, nee):
    sc = _principled(scenes.scene_lit_plane(5 * MM, (scenes.LAMBERT, (0.5,) * 3),
                                            light=(1 * MM, 3 * MM, -1 * MM, 1 * MM), h=2 * MM, emit=3.0),
                     0, params)
    _parity(ctx, sc, _job(nee=nee, max_bounces=3), "plane %s nee=%d" % (params, nee))


def test_rejects_out_of_range_parameters(ctx):
    import paper_2606_14173_amd as hpt
    sc = _principled(scenes.scene_furnace_sphere(3e-3, 1e-3), 0, PARAMS[0])
    for bad in ((0, 1.5), (2, -0.1)):
        s2 = {k: np.array(v, copy=True) for k, v in sc.items()}
        s2["mat_pbr"][0, bad[0]] = bad[1]
        with pytest.raises(hpt.HptError):
            ctx.upload_scene(s2)
    s3 = {k: np.array(v, copy=True) for k, v in sc.items()}
    s3["mat_rough"][0] = 0.0
    with pytest.raises(hpt.HptError):
        ctx.upload_scene(s3)
