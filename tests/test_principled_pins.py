"""Pins of the oracle's principled reflectance (Burley 2012, metallic-roughness
core: Burley diffuse, GGX specular, GTR1 clearcoat; one-sample MIS over the
lobes) against what the mathematics fixes: the directional albedo from the
sampled weights equals the quadrature of f cos over the hemisphere, the
combined pdf integrates to the mass above the horizon, sampled directions
follow that pdf, and a
fully metallic surface without clearcoat is the pinned GGX lobe."""
import numpy as np
import pytest

import oracle
import scenes
from scenes import jobs

# (base, roughness, metallic, specular, clearcoat, clearcoat gloss)
PARAMS = [(0.7, 0.5, 0.0, 0.5, 0.0, 1.0),
          (0.4, 0.8, 0.3, 0.8, 0.6, 0.0),
          (0.9, 0.6, 1.0, 0.5, 0.0, 1.0),
          (0.2, 0.7, 0.0, 0.2, 1.0, 0.2)]


def _view(theta):
    return np.array([np.sin(theta), 0.0, np.cos(theta)])


def _quad(f, n_t=600, n_p=300):
    """Integral of f(L) over the upper hemisphere, midpoint rule in
    (cos theta, phi) (uniform in solid angle)."""
    mu = (np.arange(n_t) + 0.5) / n_t
    ph = (np.arange(n_p) + 0.5) / n_p * 2 * np.pi
    s = 0.0
    for m in mu:
        st = np.sqrt(1 - m * m)
        for p in ph:
            s += f(np.array([st * np.cos(p), st * np.sin(p), m]))
    return s * (1.0 / n_t) * (2 * np.pi / n_p)


@pytest.mark.parametrize("params", PARAMS)
def test_albedo_from_samples_equals_quadrature(params):
    V = _view(0.6)
    rng = np.random.default_rng(1)
    w = np.array([oracle.principled_sample(params, V, rng.random(3))[1] for _ in range(60000)])
    q = _quad(lambda L: oracle.principled_eval(params, V, L)[0], 300, 150)
    se = w.std() / np.sqrt(w.size)
    assert abs(w.mean() - q) < 4 * se + 2e-3 * q, (w.mean(), q, se)


@pytest.mark.parametrize("params", PARAMS)
def test_pdf_integrates_to_the_mass_above_the_horizon(params):
    """Seen along the normal, a lobe sample is lost below the horizon when its
    half vector is more than 45 degrees off: for GGX with probability
    a^2 / (1 + a^2), for GTR1 ln((1 + a^2) / 2) / (2 ln a) (from the
    half-vector CDFs); the combined pdf integrates to one minus the lost
    mass."""
    base, r, m, spec, cc, gloss = params
    a = r * r
    ac = 0.1 * (1 - gloss) + 0.001 * gloss
    w = np.array([1 - m, 1.0, 0.25 * cc])
    p = w / w.sum()
    lost = p[1] * a * a / (1 + a * a) + p[2] * np.log((1 + ac * ac) / 2) / (2 * np.log(ac))
    V = _view(0.0)
    total = _quad(lambda L: oracle.principled_eval(params, V, L)[1], 400, 200)
    assert abs(total - (1.0 - lost)) < 3e-3, (total, 1 - lost)


def test_sampled_directions_follow_the_pdf():
    """Histogram of sampled cos(theta) against the pdf integrated over each
    bin (chi-square over 12 bins; every lobe contributes)."""
    params = PARAMS[1]
    V = _view(0.4)
    rng = np.random.default_rng(2)
    n = 40000
    mus = []
    for _ in range(n):
        L, w, lobe = oracle.principled_sample(params, V, rng.random(3))
        if L[2] > 0:
            mus.append(L[2])
    edges = np.linspace(0, 1, 13)
    hist, _ = np.histogram(mus, edges)
    exp = []
    for a, b in zip(edges[:-1], edges[1:]):
        k_t, k_p = 40, 120
        mu = a + (np.arange(k_t) + 0.5) / k_t * (b - a)
        ph = (np.arange(k_p) + 0.5) / k_p * 2 * np.pi
        s = 0.0
        for m in mu:
            st = np.sqrt(1 - m * m)
            for p in ph:
                s += oracle.principled_eval(params, V, np.array([st * np.cos(p), st * np.sin(p), m]))[1]
        exp.append(s * (b - a) / k_t * 2 * np.pi / k_p * n)
    exp = np.array(exp)
    chi2 = np.sum((hist - exp) ** 2 / exp)
    assert chi2 < 35, (chi2, hist, exp.round())   # 11 dof: p ~ 2e-4


def test_metallic_without_clearcoat_is_ggx():
    """A fully metallic principled plane without clearcoat, roughness r,
    reflects exactly like the GGX material with alpha = r^2 and F0 = base:
    same directions (the specular lobe is always chosen and consumes the
    same uniforms) and the same weights, path by path."""
    r, f0 = 0.75, 0.8   # r and r^2 exact in FP32, as both materials store them
    g = scenes.scene_ggx_plane(3e-3, f0, r * r, env=1.0)
    p = dict(g, mat_type=np.array([scenes.PRINCIPLED], np.uint32),
             mat_rough=np.array([r], np.float32),
             mat_pbr=np.array([[1.0, 0.5, 0.0, 1.0]], np.float32))
    j = dict(jobs.JOB_DEFAULTS)
    j.update(width=8, height=8, lambdas=[520e-9], comps=[1], spp=64, max_bounces=3, T=1, random_phase=0,
             grf_w=64, grf_h=64)
    grf = np.ones((64, 64, 1), dtype=np.complex128)
    _, rg, _ = oracle.trace(oracle.OracleScene(g), j, grf=grf, records=True)
    _, rp, _ = oracle.trace(oracle.OracleScene(p), j, grf=grf, records=True)
    hit = rg["bP"] > 0
    assert hit.sum() > 1000
    assert np.allclose(rp["A"][hit], rg["A"][hit], rtol=1e-10, atol=1e-14)


def test_burley_diffuse_is_lambert_where_fd90_is_one():
    """Burley's diffuse term is Lambertian (base / pi) wherever its grazing
    factor F_D90 = 0.5 + 2 r cos^2(theta_d) equals one: for r = 1/2 that is
    cos(theta_d) = 1/sqrt(2), i.e. V and L 90 degrees apart. The diffuse part
    is the change of f with the base colour (the dielectric F0 does not
    depend on it)."""
    for tv in (0.2, 0.5, 0.8):
        V = np.array([np.sin(tv), 0.0, np.cos(tv)])
        for phi in (0.0, 1.0, 2.5):
            # a unit L perpendicular to V, in the upper hemisphere
            u = np.array([np.cos(tv) * np.cos(phi), np.sin(phi), -np.sin(tv) * np.cos(phi)])
            L = u if u[2] > 0 else -u
            if L[2] < 0.05:
                continue
            f1 = oracle.principled_eval((0.8, 0.5, 0.0, 0.5, 0.0, 1.0), V, L)[0]
            f0 = oracle.principled_eval((0.0, 0.5, 0.0, 0.5, 0.0, 1.0), V, L)[0]
            assert abs((f1 - f0) / L[2] - 0.8 / np.pi) < 1e-12, (tv, phi)
