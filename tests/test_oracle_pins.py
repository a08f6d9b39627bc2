"""Pins of the FP64 oracle against closed forms, brute force, textbook values
and invariants -- never against the oracle itself.

Each test names the passage of the paper (HoloPathTracer) whose computation
it pins, and the independent fact it checks.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import scenes
from scenes import jobs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LAM = 520e-9
PITCH = 8e-6
S_CONE = LAM / (2 * PITCH)


def _job(**kw):
    j = dict(jobs.JOB_DEFAULTS)
    j.update(width=16, height=16, lambdas=[LAM], comps=[1], spp=64, max_bounces=4, T=1,
             random_phase=0, grf_w=64, grf_h=64)
    j.update(kw)
    return j


def _grf_dummy(job):
    return np.ones((job["grf_h"], job["grf_w"], job["T"]), dtype=np.complex128)


# --------------------------------------------------------------- generator

def test_philox_known_answers(oracle_lib):
    """Counter-based generator: Philox4x32-10 known-answer vectors (SC'11)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = oracle.philox(v[0:4], v[4:6])
        assert out.tolist() == v[6:10]


# --------------------------------------------------------------- geometry

def test_sphere_hit_closed_form(oracle_lib):
    sc = scenes.scene_furnace_sphere(3e-3, 1e-3)
    o = oracle.OracleScene(sc)
    zc, R = float(np.float32(3e-3)), float(np.float32(1e-3))   # stored in float32
    t, g = o.closest_hit([0, 0, 0], [0, 0, 1])
    assert g == 0 and t == pytest.approx(zc - R, rel=1e-14)
    # from inside the sphere: the far root
    t, g = o.closest_hit([0, 0, zc], [0, 0, 1])
    assert g == 0 and t == pytest.approx(R, rel=1e-12)
    # tangent-free miss
    t, g = o.closest_hit([2e-3, 0, 0], [0, 0, 1])
    assert g == -1


def test_triangle_hit_closed_form(oracle_lib):
    sc = scenes.scene_lambert_plane(2e-3, (0.5, 0.5, 0.5), half=1e-3)
    o = oracle.OracleScene(sc)
    # oblique ray: plane z=2mm reached at t = 2mm / cos
    d = np.array([0.3, -0.2, 1.0])
    d /= np.linalg.norm(d)
    t, g = o.closest_hit([1e-4, 2e-4, 0], d)
    assert g in (0, 1) and t == pytest.approx(float(np.float32(2e-3)) / d[2], rel=1e-13)
    t, g = o.closest_hit([0, 0, 0], [1, 0, 0])
    assert g == -1


def test_tie_break_lower_id(oracle_lib):
    """Equal t: the lower primitive id wins (brute force and BVH)."""
    sc = scenes.scene_lambert_plane(2e-3, (0.5,) * 3, half=1e-3)
    tri = np.concatenate([sc["tri"], sc["tri"]])
    sc["tri"] = tri
    sc["tri_mat"] = np.zeros(len(tri), np.uint32)
    o = oracle.OracleScene(sc)
    for brute in (True, False):
        t, g = o.closest_hit([3e-4, 1e-4, 0], [0, 0, 1], brute=brute)
        t2, g2 = o.closest_hit([3e-4, 1e-4, 0], [0, 0, 1], exclude=g, brute=brute)
        assert g < 2 and t2 == t and g2 == g + 2


def test_bvh_matches_brute_force(oracle_lib):
    """The oracle's BVH returns exactly the brute-force closest hit."""
    sc = scenes.scene_mid()
    sub = np.random.default_rng(5).choice(len(sc["tri"]), 6000, replace=False)
    sc["tri"] = sc["tri"][sub]
    sc["tri_mat"] = sc["tri_mat"][sub]
    o = oracle.OracleScene(sc)
    rng = np.random.default_rng(0)
    n_hit = 0
    for i in range(600):
        org = np.array([rng.uniform(-3, 3), rng.uniform(-3, 3), rng.uniform(0, 20)]) * 1e-3
        d = rng.normal(size=3)
        if i % 2 == 0:   # aim at a random triangle's centroid
            d = sc["tri"][rng.integers(len(sc["tri"]))].mean(0) - org
        d /= np.linalg.norm(d)
        a = o.closest_hit(org, d, brute=True)
        b = o.closest_hit(org, d, brute=False)
        assert a == b
        n_hit += a[1] >= 0
    assert n_hit > 250


# --------------------------------------------------------------- BSDFs

def test_fresnel_textbook(oracle_lib):
    rows = [list(map(float, l.split())) for l in open(os.path.join(GOLDEN, "fresnel_textbook.txt"))
            if l.strip() and not l.startswith("#")]
    for ci, ei, et, F in rows:
        assert oracle.fresnel(ci, ei, et) == pytest.approx(F, rel=1e-12, abs=1e-15)
    # critical angle from inside: asin(1/1.5) = 41.81 deg
    crit = math.cos(math.asin(1 / 1.5))
    assert oracle.fresnel(crit - 1e-9, 1.5, 1.0) == 1.0
    assert oracle.fresnel(crit + 1e-6, 1.5, 1.0) < 1.0


def test_lambert_cosine_distribution(oracle_lib):
    """Cosine-weighted hemisphere: cos^2(theta) is uniform, azimuth uniform."""
    from scipy import stats
    rng = np.random.default_rng(1)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    u = rng.random((4000, 2))
    d = np.array([oracle.sample_lambert(n, a, b) for a, b in u])
    assert np.allclose(np.linalg.norm(d, axis=1), 1, atol=1e-14)
    c = d @ n
    assert (c >= 0).all()
    assert stats.kstest(c * c, "uniform").pvalue > 1e-3
    # cos^2 = 1 - u1 exactly (the radius sqrt(u1) maps to sin^2 = u1)
    assert np.allclose(c * c, 1 - u[:, 0], atol=1e-12)


def _ggx_D(m, a):
    c2 = m[..., 2] ** 2
    t2 = (m[..., 0] ** 2 + m[..., 1] ** 2) / c2
    return 1.0 / (np.pi * a * a * c2 * c2 * (1 + t2 / (a * a)) ** 2)


def _ggx_lambda(w, a):
    t2 = (w[..., 0] ** 2 + w[..., 1] ** 2) / w[..., 2] ** 2
    return (-1 + np.sqrt(1 + a * a * t2)) / 2


def test_vndf_density_and_masking(oracle_lib):
    """GGX visible normals: the sampled normals follow
    D_V(m) = G1(V) max(0, V.m) D(m) / V_z (Heitz 2018, textbook GGX D and Smith
    Lambda), and E[G1(L)] matches quadrature."""
    from scipy import stats
    a = 0.35
    th_v = 0.9
    V = np.array([math.sin(th_v), 0.0, math.cos(th_v)])
    rng = np.random.default_rng(2)
    N = 60000
    u = rng.random((N, 2))
    M = np.array([oracle.sample_vndf(V, a, x, y) for x, y in u])
    assert np.allclose(np.linalg.norm(M, axis=1), 1, atol=1e-13)
    # analytic density on a (cos theta, phi) grid
    nb_t, nb_p = 12, 16
    ct_edges = np.linspace(0, 1, nb_t + 1)
    ph_edges = np.linspace(-np.pi, np.pi, nb_p + 1)
    G1V = 1.0 / (1.0 + _ggx_lambda(V, a))
    qn = 40
    expected = np.zeros((nb_t, nb_p))
    for i in range(nb_t):
        ct = ct_edges[i] + (np.arange(qn) + 0.5) / qn * (ct_edges[i + 1] - ct_edges[i])
        for j in range(nb_p):
            ph = ph_edges[j] + (np.arange(qn) + 0.5) / qn * (ph_edges[j + 1] - ph_edges[j])
            CT, PH = np.meshgrid(ct, ph)
            st = np.sqrt(1 - CT ** 2)
            m = np.stack([st * np.cos(PH), st * np.sin(PH), CT], -1)
            dens = G1V * np.maximum(0, m @ V) * _ggx_D(m, a) / V[2]
            expected[i, j] = dens.mean() * (ct_edges[i + 1] - ct_edges[i]) * (2 * np.pi / nb_p)
    assert expected.sum() == pytest.approx(1.0, abs=2e-3)
    ct = M[:, 2]
    ph = np.arctan2(M[:, 1], M[:, 0])
    H, _, _ = np.histogram2d(ct, ph, [ct_edges, ph_edges])
    E = expected * N
    keep = E > 20
    chi2 = ((H[keep] - E[keep]) ** 2 / E[keep]).sum()
    dof = keep.sum() - 1
    assert stats.chi2.sf(chi2, dof) > 1e-4
    # masking of the reflected direction: E[G1(L)] by MC and by quadrature
    L = 2 * (M @ V)[:, None] * M - V
    g1 = np.array([oracle.smith_g1(l, a) if l[2] > 0 else 0.0 for l in L])
    mc = g1.mean()
    Lq = []
    wq = []
    for i in range(nb_t * 4):
        c = (i + 0.5) / (nb_t * 4)
        for j in range(64):
            p = -np.pi + (j + 0.5) / 64 * 2 * np.pi
            s = math.sqrt(1 - c * c)
            m = np.array([s * math.cos(p), s * math.sin(p), c])
            d = G1V * max(0, m @ V) * _ggx_D(m, a) / V[2]
            l = 2 * (m @ V) * m - V
            gl = 1.0 / (1.0 + _ggx_lambda(l, a)) if l[2] > 0 else 0.0
            Lq.append(gl)
            wq.append(d)
    quad = np.sum(np.array(Lq) * np.array(wq)) / np.sum(wq)
    assert abs(mc - quad) < 4 * g1.std() / math.sqrt(N) + 2e-3


# --------------------------------------------------------------- cache maps

def test_octahedral_map_round_trip(oracle_lib):
    rng = np.random.default_rng(3)
    for _ in range(500):
        w = rng.normal(size=3)
        w /= np.linalg.norm(w)
        uv, b = oracle.oct_map(w, 8)
        assert np.abs(uv).max() <= 1 + 1e-15
        assert np.allclose(oracle.oct_decode(uv[0], uv[1]), w, atol=1e-13)
        assert 0 <= b < 64
    # every bin centre decodes to a direction that maps back into its bin
    for bv in range(8):
        for bu in range(8):
            u = -1 + 2 * (bu + 0.5) / 8
            v = -1 + 2 * (bv + 0.5) / 8
            assert oracle.oct_map(oracle.oct_decode(u, v), 8)[1] == bv * 8 + bu


def test_round_fp16_matches_ieee(oracle_lib):
    """binary16 round-to-nearest-even against numpy's IEEE conversion."""
    rng = np.random.default_rng(4)
    xs = np.concatenate([rng.uniform(0, 5, 3000), rng.uniform(0, 1e-4, 1000),
                         10.0 ** rng.uniform(-8, 4.5, 2000)])
    # exact ties between binary16 neighbours
    h = np.arange(1, 2000, dtype=np.float64)
    xs = np.concatenate([xs, 1.0 + (2 * h + 1) * 2.0 ** -11])
    for x in xs:
        assert oracle.round_fp16(x) == float(np.float64(x).astype(np.float16))


# --------------------------------------------------------------- cone sampling

def test_cone_directions_uniform_disc(oracle_lib):
    """Sec. 4.1/4.2: directions fill the recordable cone sin(theta) <= lambda/2d,
    uniform over direction cosines (the passband of Eq. 4)."""
    from scipy import stats
    sc = scenes.scene_lambert_plane(2e-3, (0.5,) * 3, env=1.0, half=3e-3)
    o = oracle.OracleScene(sc)
    job = _job(width=4, height=4, spp=2048, max_bounces=2)
    U, recs, _ = oracle.trace(o, job, grf=_grf_dummy(job), records=True)
    r = recs.reshape(-1)
    assert (r["kind"] == 4).all()
    px = np.arange(4)
    xp = ((px + 0.5) - 2) * PITCH
    XP = np.broadcast_to(xp[None, :, None], (4, 4, 2048)).reshape(-1)
    YP = np.broadcast_to(xp[:, None, None], (4, 4, 2048)).reshape(-1)
    al = (r["qx"] - XP) / r["r"]
    be = (r["qy"] - YP) / r["r"]
    rad2 = (al ** 2 + be ** 2) / S_CONE ** 2
    assert rad2.max() <= 1 + 1e-12
    assert stats.kstest(rad2, "uniform").pvalue > 1e-3
    ang = np.arctan2(be, al)
    assert stats.kstest((ang + np.pi) / (2 * np.pi), "uniform").pvalue > 1e-3
    # the plane lies at depth z0: r = z0 / v_z along the primary direction
    vz = np.sqrt(1 - al ** 2 - be ** 2)
    assert np.allclose(r["r"], 2e-3 / vz, rtol=1e-12)
    # Lambert albedo 0.5 under env 1 with one tail bounce: A = sqrt(0.5)
    assert np.allclose(r["A"], math.sqrt(0.5), rtol=1e-14)


# --------------------------------------------------------------- RS integral

def _rs_quadrature(xp, yp, z_img, half, center, k, s, h_q, block=None):
    """Band-limited RS integral of Eq. 2 over a square source of unit
    amplitude facing the SLM at depth z_img: sum of exp(ikr) cos/r dS over
    source points whose direction from the pixel lies inside the cone.
    block(x, y) -> bool removes directions that are shadowed."""
    n = int(round(2 * half / h_q))
    g = (np.arange(n) + 0.5) / n * 2 * half - half
    X, Y = np.meshgrid(g + center[0], g + center[1])
    dx, dy = X - xp, Y - yp
    r = np.sqrt(dx * dx + dy * dy + z_img * z_img)
    inside = (dx * dx + dy * dy) <= (s * r) ** 2
    if block is not None:
        inside &= ~block(dx / r, dy / r, r)
    cos = z_img / r
    dS = (2 * half / n) ** 2
    return np.sum(np.where(inside, np.exp(1j * k * r) * cos / r, 0)) * dS


def _batch_means(o, job, K):
    """K independent chunks of the sample range -> mean and standard error."""
    N = job["spp"]
    parts = []
    for i in range(K):
        j = dict(job, spp_begin=i * N // K, spp_end=(i + 1) * N // K)
        U, _, _ = oracle.trace(o, j, grf=_grf_dummy(job))
        parts.append(U[0, 0] * K)
    parts = np.array(parts)
    mean = parts.mean(0)
    se = np.sqrt((np.abs(parts - mean) ** 2).sum(0) / (K - 1) / K)
    return mean, se


def test_rs_integral_patch_quadrature(oracle_lib):
    """Eq. 2 by brute force: a small emitter patch (L_e = 1, phases off) must
    reproduce the RS integral restricted to the recordable cone, including
    pixels where the cone edge cuts the patch. Pins the sample weight
    r / p(v), the cone radius lambda/2d and the sign of the phase."""
    z0, half = 1e-3, 16e-6
    sc = scenes.scene_patch(z0, half)
    o = oracle.OracleScene(sc)
    job = _job(width=12, height=12, spp=8192, max_bounces=2)
    mean, se = _batch_means(o, job, 32)
    k = 2 * np.pi / LAM
    idx = (np.arange(12) + 0.5 - 6) * PITCH
    quad = np.array([[_rs_quadrature(x, y, z0, half, (0, 0), k, S_CONE, 0.1e-6) for x in idx]
                     for y in idx])
    err = np.abs(mean - quad)
    lit = np.abs(quad) > 0
    assert lit.sum() > 40 and (~lit).sum() > 10
    ok = err <= 4 * se + 1e-3 * np.abs(quad).max()
    assert ok.mean() >= 0.99, (err / np.maximum(se, 1e-30))[~ok]
    # unlit pixels are exactly zero in both
    assert np.all(mean[~lit] == 0)
    # phase sign: conj(quad) would be far off
    bad = np.abs(mean - np.conj(quad))
    assert np.median(bad[lit] / se[lit]) > 10


def test_mirror_image_method(oracle_lib):
    """Coherent delta prefix (Sec. 4.2): a patch seen through a flat mirror
    equals the RS integral of its mirror image at depth 2 z_m - z_1 (OPL
    summed over the reflection), with the patch's back shadowing the direct
    directions."""
    z1, zm, half = 1.0e-3, 1.5e-3, 12e-6
    sc = scenes.scene_mirror_patch(z1, zm, half)
    o = oracle.OracleScene(sc)
    job = _job(width=12, height=12, spp=8192, max_bounces=4)
    mean, se = _batch_means(o, job, 32)
    k = 2 * np.pi / LAM
    z_img = 2 * zm - z1
    idx = (np.arange(12) + 0.5 - 6) * PITCH
    quad = np.zeros((12, 12), complex)
    for iy, y in enumerate(idx):
        for ix, x in enumerate(idx):
            def block(a, b, r, x=x, y=y):
                # crossing of the plane z1 on the way up: hits the patch's back
                vz = np.sqrt(1 - a * a - b * b)
                tz = z1 / vz
                cx, cy = x + a * tz, y + b * tz
                return (np.abs(cx) <= half) & (np.abs(cy) <= half)
            quad[iy, ix] = _rs_quadrature(x, y, z_img, half, (0, 0), k, S_CONE, 0.1e-6, block)
    lit = np.abs(quad) > 0
    assert lit.sum() > 20
    err = np.abs(mean - quad)
    ok = err <= 4 * se + 2e-3 * np.abs(quad).max()
    assert ok.mean() >= 0.99


def test_dielectric_slab_opl_closed_form(oracle_lib):
    """OPL = sum n_i L_i through ideal refraction (Sec. 4.2) against Snell's
    law for a slab: z_a/cos0 + n (z_b - z_a)(1 + 2m)/cos1 + (z_c - z_b)/cos0,
    m = number of internal round trips."""
    za, zb, zc, n = 1e-3, 1.5e-3, 2e-3, 1.5
    sc = scenes.scene_slab(za, zb, zc, ior=n)
    o = oracle.OracleScene(sc)
    job = _job(width=6, height=6, spp=512, max_bounces=8)
    U, recs, _ = oracle.trace(o, job, grf=_grf_dummy(job), records=True)
    r = recs.reshape(-1)
    px = ((np.arange(6) + 0.5) - 3) * PITCH
    XP = np.broadcast_to(px[None, :, None], (6, 6, 512)).reshape(-1)
    YP = np.broadcast_to(px[:, None, None], (6, 6, 512)).reshape(-1)
    sel = r["bP"] >= 3
    assert sel.sum() > 1000
    ell = r["ell"][sel]
    a = (r["qx"][sel] - XP[sel]) / ell
    b = (r["qy"][sel] - YP[sel]) / ell
    s0 = np.sqrt(a * a + b * b)
    c0 = np.sqrt(1 - s0 * s0)
    c1 = np.sqrt(1 - (s0 / n) ** 2)
    m = (r["bP"][sel] - 3) // 2
    assert set(np.unique(r["bP"][sel])) <= {3, 5, 7}
    za, zb, zc = (float(np.float32(z)) for z in (za, zb, zc))   # stored in float32
    closed = za / c0 + n * (zb - za) * (1 + 2 * m) / c1 + (zc - zb) / c0
    assert np.allclose(ell, closed, rtol=1e-13, atol=0)
    # radiance scaling (1/n^2)(n^2) = 1 for the in-out pair: A^2 = beta_pre * L
    assert (r["kind"][r["bP"] == 3] >= 0).all()


# --------------------------------------------------------------- amplitude

def test_white_furnace_sphere(oracle_lib):
    """Eq. 1 with albedo 1 under a uniform environment of radiance 1: every
    path that reaches the convex Lambert sphere gets L = 1 exactly (A = 1)."""
    sc = scenes.scene_furnace_sphere(3e-3, 1e-3, env=1.0)
    o = oracle.OracleScene(sc)
    job = _job(width=8, height=8, spp=256, max_bounces=3)
    U, recs, _ = oracle.trace(o, job, grf=_grf_dummy(job), records=True)
    r = recs.reshape(-1)
    assert (r["kind"] == 4).all()
    assert np.allclose(r["A"], 1.0, rtol=0, atol=1e-15)


def test_emitter_one_sided(oracle_lib):
    sc = scenes.scene_patch(1e-3, 20e-6, face=+1)
    o = oracle.OracleScene(sc)
    job = _job(width=8, height=8, spp=256)
    U, recs, _ = oracle.trace(o, job, grf=_grf_dummy(job), records=True)
    assert np.all(U == 0)
    assert (recs["kind"][recs["n_hits"] > 0] == 3).all()


def test_channel_albedo_component(oracle_lib):
    """Channels are traced independently, each with its own colour component."""
    sc = scenes.scene_lambert_plane(2e-3, (0.2, 0.5, 0.8), env=1.0)
    o = oracle.OracleScene(sc)
    job = _job(width=4, height=4, spp=64, max_bounces=2, lambdas=[638e-9, 520e-9, 450e-9],
               comps=[0, 1, 2])
    U, recs, _ = oracle.trace(o, job, grf=_grf_dummy(job), records=True)
    for c, a in enumerate((0.2, 0.5, 0.8)):
        assert np.allclose(recs[c]["A"], math.sqrt(a), rtol=1e-14)


# --------------------------------------------------------------- Eq. 3

def _rot90(sc):
    rot = dict(sc)
    tri = sc["tri"].copy()
    rot["tri"] = np.stack([-tri[..., 1], tri[..., 0], tri[..., 2]], -1).astype(np.float32)
    sph = sc["sph"].copy()
    rot["sph"] = np.stack([-sph[:, 1], sph[:, 0], sph[:, 2], sph[:, 3]], -1).astype(np.float32)
    return rot


def test_transform_rotation_invariance(oracle_lib):
    """Eq. 3: rotating the world by R (90 degrees about z, exact in float32)
    and setting T = R^-1 leaves the coherent prefix (hits, OPL, image point
    Q in hologram space, weight) unchanged; with an emitter as the image point
    (no incoherent tail, whose local frames are not rotation-equivariant) the
    hologram itself is unchanged."""
    T = (0.0, 1.0, 0.0, 0.0, -1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0)
    sc = scenes.scene_tiny()
    job = _job(width=16, height=16, spp=16, max_bounces=2, random_phase=1, T=2,
               grf_w=64, grf_h=64, grf_seed=3)
    grf = oracle.grf_table(64, 64, 2, 3)
    _, r0, _ = oracle.trace(oracle.OracleScene(sc), job, grf=grf, records=True)
    _, r1, _ = oracle.trace(oracle.OracleScene(_rot90(sc)), dict(job, holo_from_world=T),
                            grf=grf, records=True)
    assert np.mean(r0["first_gid"] == r1["first_gid"]) > 0.999
    same = r0["first_gid"] == r1["first_gid"]
    for f in ("r", "W", "qx", "qy", "ell"):
        assert np.allclose(r0[f][same], r1[f][same], rtol=1e-12, atol=1e-18)
    sc = scenes.scene_patch(1e-3, 16e-6, center=(5e-6, -3e-6))
    job = _job(width=12, height=12, spp=256, max_bounces=2, random_phase=1, T=2,
               grf_w=64, grf_h=64, grf_seed=3)
    U0, _, _ = oracle.trace(oracle.OracleScene(sc), job, grf=grf)
    U1, _, _ = oracle.trace(oracle.OracleScene(_rot90(sc)), dict(job, holo_from_world=T),
                            grf=grf)
    assert np.abs(U0).max() > 0
    assert np.allclose(U0, U1, rtol=0, atol=1e-9 * np.abs(U0).max())


# --------------------------------------------------------------- Eq. 4 GRF

def test_grf_brute_force_dft(oracle_lib):
    """Eq. 4 written as an explicit sum over passband frequencies on a small
    grid equals the table (which uses an FFT)."""
    gw, gh, T, seed = 12, 10, 2, 9
    tab = oracle.grf_table(gw, gh, T, seed, stored=False)
    # the stored table is that transform rounded once to complex64
    assert np.array_equal(oracle.grf_table(gw, gh, T, seed), tab.astype(np.complex64).astype(np.complex128))
    xi, mask = oracle.grf_phases(gw, gh, 0, T, seed)
    d = 1.0
    fx = np.fft.fftfreq(gw, d)
    fy = np.fft.fftfreq(gh, d)
    # passband: f_x^2 + f_y^2 <= (1/(2d))^2, checked in exact rationals
    for jy in range(gh):
        for jx in range(gw):
            Fx = Fraction(jx if jx < (gw + 1) // 2 else jx - gw, gw)
            Fy = Fraction(jy if jy < (gh + 1) // 2 else jy - gh, gh)
            assert mask[0, jy, jx] == (Fx * Fx + Fy * Fy <= Fraction(1, 4))
    nb = mask[0].sum()
    for t in range(T):
        for y in range(gh):
            for x in range(gw):
                acc = 0j
                for jy in range(gh):
                    for jx in range(gw):
                        if mask[t, jy, jx]:
                            acc += np.exp(1j * xi[t, jy, jx]) * np.exp(
                                2j * np.pi * (fx[jx] * x + fy[jy] * y))
                assert abs(acc / math.sqrt(nb) - tab[y, x, t]) < 1e-12


def test_grf_statistics(oracle_lib):
    """phi_t = arg r_t is uniform on (-pi, pi], the spectrum of r_t is
    confined to the passband, and frames are uncorrelated (Sec. 4.3)."""
    from scipy import stats
    gw, gh, T = 96, 64, 3
    tab = oracle.grf_table(gw, gh, T, 11)
    exact = oracle.grf_table(gw, gh, T, 11, stored=False)
    _, mask = oracle.grf_phases(gw, gh, 0, 1, 11)
    for t in range(T):
        spec = np.fft.fft2(exact[:, :, t])
        assert np.abs(spec[~mask[0]]).max() < 1e-9 * np.abs(spec).max()
        # the stored (complex64) table leaks only its rounding out of the band
        spec = np.fft.fft2(tab[:, :, t])
        assert np.abs(spec[~mask[0]]).max() < 1e-6 * np.abs(spec).max()
        ph = np.angle(tab[:, :, t]).ravel()
        assert stats.kstest((ph + np.pi) / (2 * np.pi), "uniform").pvalue > 1e-4
    n = gw * gh
    for t in range(T):
        for u in range(t + 1, T):
            c = np.mean(np.exp(1j * (np.angle(tab[:, :, t]) - np.angle(tab[:, :, u]))))
            assert abs(c) < 5 / math.sqrt(n)


# --------------------------------------------------------------- Path Reuse

def test_path_reuse_invariants(oracle_lib):
    """Sec. 4.3 Path Reuse: frames differ only by phi_t. With one sample per
    pixel |U_t| is the same for every t; with many samples the mean intensity
    of every frame agrees within the Monte Carlo error."""
    sc = scenes.scene_tiny()
    o = oracle.OracleScene(sc)
    T = 6
    job = _job(width=24, height=24, spp=1, max_bounces=2, T=T, random_phase=1,
               grf_w=96, grf_h=96, grf_seed=5)
    grf = oracle.grf_table(96, 96, T, 5)
    U, _, _ = oracle.trace(o, job, grf=grf)
    mag = np.abs(U[0])
    assert np.allclose(mag, mag[0][None], rtol=1e-12, atol=0)
    job = dict(job, spp=32, width=32, height=32, grf_w=128, grf_h=128)
    grf = oracle.grf_table(128, 128, T, 5)
    U, _, rt = oracle.trace(o, job, grf=grf)
    I = (np.abs(U[0]) ** 2).reshape(T, -1)
    m = I.mean(1)
    se = I.std(1).mean() / math.sqrt(I.shape[1])
    assert np.all(np.abs(m - m.mean()) < 4 * se * math.sqrt(2))
    # the T-batch is T independent frames of one path set: frame t equals the
    # single-frame job run with frame t's table
    for t in (0, 3):
        U1, _, _ = oracle.trace(o, dict(job, T=1), grf=np.ascontiguousarray(grf[:, :, t:t + 1]))
        assert np.array_equal(U1[0, 0], U[0, t])


def test_spp_chunks_sum_to_full(oracle_lib):
    """A job is resumable at any sample boundary: chunk fields sum to the
    one-shot field (the estimator is a sum over independently keyed samples)."""
    sc = scenes.scene_tiny()
    o = oracle.OracleScene(sc)
    job = _job(width=16, height=16, spp=24, max_bounces=2)
    U, _, _ = oracle.trace(o, job, grf=_grf_dummy(job))
    parts = sum(oracle.trace(o, dict(job, spp_begin=a, spp_end=b), grf=_grf_dummy(job))[0]
                for a, b in ((0, 5), (5, 17), (17, 24)))
    assert np.allclose(parts, U, rtol=1e-12, atol=1e-12 * np.abs(U).max())


# --------------------------------------------------------------- cache

def test_cache_furnace(oracle_lib):
    """Radiance cache: in a furnace (albedo 1, env 1, a single planar
    triangle) every entry is exactly 1, and a cached tail returns
    albedo * 1."""
    sc = scenes.scene_single_tri(2e-3, env=1.0)
    o = oracle.OracleScene(sc)
    c = oracle.OracleCache(o, res=8, bins=4, spb=4, max_bounces=4, seed=1)
    rng = np.random.default_rng(0)
    for _ in range(50):
        assert c.entry(1, int(rng.integers(512)), int(rng.integers(16))) == 1.0
    # a path whose image point is on the triangle ends in one cache lookup:
    # A^2 = albedo * entry = 1
    job = _job(width=4, height=4, spp=16, max_bounces=3, use_cache=1)
    sc = dict(sc, tri=(sc["tri"].astype(np.float64) * [[[40, 40, 1]]]).astype(np.float32))
    o = oracle.OracleScene(sc)
    c = oracle.OracleCache(o, res=8, bins=4, spb=4, max_bounces=4, seed=1)
    U, recs, _ = oracle.trace(o, job, grf=_grf_dummy(job), cache=c, records=True)
    r = recs.reshape(-1)
    hit = r["n_hits"] > 0
    assert hit.sum() > 40 and (r["kind"][hit] == 6).all()
    assert np.allclose(r["A"][hit], 1.0, rtol=0, atol=1e-15)


# --------------------------------------------------------------- more pins

def test_radiance_theorem_emitter_in_glass(oracle_lib):
    """Refraction scales radiance by (n_i/n_t)^2 (radiance theorem, L/n^2 is
    invariant): an emitter of radiance 1 embedded in glass n=1.5 is seen from
    air with A^2 = 1/1.5^2 through one refraction."""
    sc = scenes.scene_slab_emitter(1e-3, 2e-3, 1.5e-3, ior=1.5)
    o = oracle.OracleScene(sc)
    job = _job(width=6, height=6, spp=256, max_bounces=4)
    U, recs, _ = oracle.trace(o, job, grf=_grf_dummy(job), records=True)
    r = recs.reshape(-1)
    sel = (r["kind"] == 3) & (r["bP"] == 2)
    assert sel.sum() > 5000
    assert np.allclose(r["A"][sel] ** 2, 1 / 1.5 ** 2, rtol=1e-13)
    # Fresnel lobe choice: the fraction reflected at the first face is the
    # reflectance at near-normal incidence, ((n-1)/(n+1))^2 = 0.04
    refl = (r["kind"] == 1) & (r["n_hits"] == 1)
    f = refl.mean()
    assert abs(f - 0.04) < 4 * math.sqrt(0.04 * 0.96 / len(r))


def test_ggx_weight_furnace(oracle_lib):
    """GGX tail weight F_schlick * G1(L) (Sec. 4.2 non-delta lobe, Eq. 1): a
    rough plane under env 1 gives E[L] = E_m~D_V[F(V.m) G1(L)], computed
    here by quadrature of the textbook GGX D, Smith Lambda and Schlick F."""
    a, f0, tilt = 0.3, 0.1, 72.0
    sc = scenes.scene_ggx_plane(2e-3, f0, a, env=1.0, tilt_deg=tilt)
    o = oracle.OracleScene(sc)
    job = _job(width=8, height=8, spp=1024, max_bounces=2)
    U, recs, _ = oracle.trace(o, job, grf=_grf_dummy(job), records=True)
    L = recs["A"].reshape(-1) ** 2
    # view direction in the plane's frame: the ray travels +z onto a normal
    # tilted by `tilt`, so V makes that angle with the normal
    th = math.radians(tilt)
    V = np.array([0.0, math.sin(th), math.cos(th)])
    G1V = 1.0 / (1.0 + _ggx_lambda(V, a))
    n_t, n_p = 400, 64
    num = den = 0.0
    for i in range(n_t):
        c = (i + 0.5) / n_t
        s = math.sqrt(1 - c * c)
        ph = -np.pi + (np.arange(n_p) + 0.5) / n_p * 2 * np.pi
        m = np.stack([s * np.cos(ph), s * np.sin(ph), np.full(n_p, c)], -1)
        dv = G1V * np.maximum(0, m @ V) * _ggx_D(m, a) / V[2]
        vm = m @ V
        l = 2 * vm[:, None] * m - V
        gl = np.where(l[:, 2] > 0, 1.0 / (1.0 + _ggx_lambda(l, a)), 0.0)
        F = f0 + (1 - f0) * (1 - vm) ** 5
        num += (dv * F * gl).sum()
        den += dv.sum()
    expect = num / den
    assert abs(L.mean() - expect) < 4 * L.std() / math.sqrt(len(L)) + 1e-3


def test_rs_integral_high_na_plane(oracle_lib):
    """Eq. 2 at a wide recordable cone (lambda/2d = 0.4) for an emitter plane
    1.5 um in front of the SLM: with amplitude 1 and phases off, the field of
    every pixel is the RS integral over the cone, which for a plane parallel
    to the SLM reduces to the 1-D integral
        U = 2 pi int_0^theta_max exp(i k z0 / cos t) (z0 / cos t) sin t dt,
    sin(theta_max) = lambda/2d. Sensitive to the v_z factor of the sample
    density and of the weight."""
    from scipy import integrate
    lam, pitch = 520e-9, 0.65e-6
    s = lam / (2 * pitch)
    z0 = float(np.float32(1.5e-6))
    sc = scenes.scene_patch(1.5e-6, 2e-3)
    o = oracle.OracleScene(sc)
    job = _job(width=4, height=4, pitch=pitch, lambdas=[lam], spp=8192, max_bounces=2)
    mean, se = _batch_means(o, job, 16)
    k = 2 * np.pi / lam
    tmax = math.asin(s)
    re = integrate.quad(lambda t: math.cos(k * z0 / math.cos(t)) * z0 / math.cos(t) * math.sin(t),
                        0, tmax, epsabs=0, epsrel=1e-12)[0]
    im = integrate.quad(lambda t: math.sin(k * z0 / math.cos(t)) * z0 / math.cos(t) * math.sin(t),
                        0, tmax, epsabs=0, epsrel=1e-12)[0]
    U = 2 * math.pi * complex(re, im)
    assert np.all(se < 0.02 * abs(U))
    assert np.all(np.abs(mean - U) <= 4 * se + 1e-9 * abs(U))


def test_grf_lookup_texel_centres(oracle_lib):
    """Sec. 4.3 hologram-space phase: texel (i, j) of the random field sits on
    pixel centre (i, j); the lookup there returns r_t/|r_t| of that texel, and
    the table is periodic."""
    W, H, gw, gh, T = 8, 6, 20, 16, 2
    grf = oracle.grf_table(gw, gh, T, 4)
    job = _job(width=W, height=H, T=T, grf_w=gw, grf_h=gh)
    for t in range(T):
        for j in (0, 3, 5):
            for i in (0, 2, 7):
                qx = ((i + 0.5) - W / 2) * PITCH
                qy = ((j + 0.5) - H / 2) * PITCH
                want = grf[j, i, t] / abs(grf[j, i, t])
                assert abs(oracle.grf_lookup(job, grf, t, qx, qy) - want) < 1e-12
                got = oracle.grf_lookup(job, grf, t, qx + gw * PITCH, qy - gh * PITCH)
                assert abs(got - want) < 1e-9


def test_grf_lookup_bilinear_off_centres(oracle_lib):
    """Sec. 4.3 hologram-space phase between texel centres: bilinear
    interpolation reproduces an affine field exactly, so for a table
    r(i, j) = a + b i + c j the lookup at texel coordinates (i0 + fx,
    j0 + fy) is the unit phasor of a + b (i0 + fx) + c (j0 + fy). Offsets
    (1/4, 3/4), (3/4, 1/4) and random ones; a swap of the two weights, a
    half-texel offset or a wrong wrap fails it."""
    W, H, gw, gh, T = 10, 8, 24, 20, 2
    a = np.array([3.0 + 1.0j, -2.0 + 2.5j])
    b = np.array([0.40 - 0.15j, -0.10 + 0.35j])
    c = np.array([-0.25 + 0.30j, 0.45 + 0.05j])
    jj, ii = np.meshgrid(np.arange(gh), np.arange(gw), indexing="ij")
    grf = np.stack([a[t] + b[t] * ii + c[t] * jj for t in range(T)], axis=-1)
    job = _job(width=W, height=H, T=T, grf_w=gw, grf_h=gh)
    rng = np.random.default_rng(7)
    offs = [(0.25, 0.75), (0.75, 0.25), (0.5, 0.125)] + [tuple(rng.random(2)) for _ in range(12)]
    n = 0
    for fx, fy in offs:
        for i0, j0 in ((0, 0), (3, 5), (gw - 2, gh - 2), (11, 2)):
            u, v = i0 + fx, j0 + fy
            qx = (u + 0.5 - W / 2) * PITCH
            qy = (v + 0.5 - H / 2) * PITCH
            for t in range(T):
                z = a[t] + b[t] * u + c[t] * v
                assert abs(oracle.grf_lookup(job, grf, t, qx, qy) - z / abs(z)) < 1e-12
                n += 1
    assert n == len(offs) * 4 * T
    # across the periodic seam the neighbour of column gw-1 is column 0
    u, v = gw - 1 + 0.25, 3.5
    qx, qy = (u + 0.5 - W / 2) * PITCH, (v + 0.5 - H / 2) * PITCH
    z = 0.75 * 0.5 * (grf[3, gw - 1, 0] + grf[4, gw - 1, 0]) + 0.25 * 0.5 * (grf[3, 0, 0] + grf[4, 0, 0])
    assert abs(oracle.grf_lookup(job, grf, 0, qx, qy) - z / abs(z)) < 1e-12


def _box_classify(o, d, half):
    """Index of the first surface a ray meets inside the box [-half, half]^3
    of scene_emitter_box: wall k = 2 axis + (direction > 0), or 6 for the
    black half-plane z = 0, x < 0. Rays are started inside the box."""
    with np.errstate(divide="ignore", invalid="ignore"):
        tw = np.where(d != 0, (np.sign(d) * half - o) / d, np.inf)
    ax = int(np.argmin(tw))
    t_exit = tw[ax]
    if d[2] != 0:
        t0 = -o[2] / d[2]
        if 0 < t0 < t_exit and o[0] + t0 * d[0] < 0:
            return 6
    return 2 * ax + (1 if d[ax] > 0 else 0)


def test_cache_entries_by_cell_and_bin(oracle_lib):
    """Radiance cache ("texture baking", Sec. 4.2) beyond the furnace: inside
    a box whose six walls emit inward with six different radiances, with a
    black half-plane z = 0 over x < 0, an entry whose cell and direction bin
    see one surface from every point of the cell along every direction of
    the bin equals that surface's radiance (0 for the black plane). The
    surfaces are found here by ray casting the box geometry, for points of
    the cell box and directions of the bin's octahedral square (the pinned
    octahedral map); entries differ by cell (below / above the half-plane,
    x < 0 / x > 0) and by bin (the wall a direction faces), so a transposed
    cell order, a swapped bin decode or a misplaced sampling point fails."""
    half, res, bins = 1e-3, 6, 8
    rad = [(1.0, 2.0, 0.5), (2.0, 3.0, 1.5), (3.0, 0.25, 2.5), (4.0, 1.25, 3.5),
           (5.0, 4.5, 0.75), (6.0, 5.5, 1.75)]
    sc = scenes.scene_emitter_box(half, rad)
    o = oracle.OracleScene(sc)
    c = oracle.OracleCache(o, res=res, bins=bins, spb=4, max_bounces=3, seed=11)
    lo, hi = c.bounds()
    ext = (hi - lo) / res
    fr = np.array([0.0005, 0.5, 0.9995])
    cell_pts = np.stack(np.meshgrid(fr, fr, fr, indexing="ij"), -1).reshape(-1, 3)
    gu = np.array([0.002, 0.25, 0.5, 0.75, 0.998])
    want, keys = {}, []
    for iz in range(1, res - 1):
        for iy in range(1, res - 1):
            for ix in range(1, res - 1):
                cell = (iz * res + iy) * res + ix
                pts = lo + (np.array([ix, iy, iz]) + cell_pts) * ext
                for bv in range(bins):
                    for bu in range(bins):
                        seen = set()
                        for su in gu:
                            for sv in gu:
                                d = oracle.oct_decode(-1 + 2 * (bu + su) / bins, -1 + 2 * (bv + sv) / bins)
                                for p in pts:
                                    seen.add(_box_classify(p, d, half))
                            if len(seen) > 1:
                                break
                        if len(seen) == 1:
                            want[(cell, bv * bins + bu)] = seen.pop()
    assert len(want) > 600
    kinds = np.array(list(want.values()))
    assert set(kinds.tolist()) == set(range(7))
    cells = np.array([k[0] for k in want], np.int32)
    bns = np.array([k[1] for k in want], np.int32)
    for comp in range(3):
        expect = np.array([0.0 if k == 6 else rad[k][comp] for k in kinds])
        got = c.entries(np.full(len(cells), comp, np.int32), cells, bns)
        assert np.array_equal(got, expect), np.flatnonzero(got != expect)[:10]
    # the same bin differs between a cell above and below the half-plane at x < 0
    up = oracle.oct_map(np.array([0.0, 0.0, 1.0]), bins)[1]
    below = (2 * res + 2) * res + 1
    above = (3 * res + 2) * res + 1
    assert want.get((below, up)) == 6 and want.get((above, up)) == 5


def test_cache_lookup_cell_of_image_points(oracle_lib):
    """A path that ends in the radiance cache at its image point P reads the
    entry of the cell containing P (Sec. 4.2 texture baking, nearest cell):
    on a tilted Lambert plane around depth z0 every path's P lies on it, its
    position follows from the record (Q = P for the identity transform; the
    depth from r), and its cell index (iz res + iy) res + ix is computed
    here from the cache grid; points within 1e-9 of a cell face are skipped."""
    z0, half, res = 2e-3, 48e-6, 8
    sc = scenes.scene_lambert_plane(z0, (0.5,) * 3, env=1.0, half=half)
    a = math.radians(25.0)                        # tilt about x through (0, 0, z0): depth varies
    v = sc["tri"].astype(np.float64)
    y, z = v[..., 1], v[..., 2] - z0
    sc["tri"] = np.stack([v[..., 0], y * math.cos(a) - z * math.sin(a), z0 + y * math.sin(a) + z * math.cos(a)],
                         -1).astype(np.float32)
    o = oracle.OracleScene(sc)
    c = oracle.OracleCache(o, res=res, bins=4, spb=1, max_bounces=2, seed=3)
    lo, hi = c.bounds()
    job = _job(width=14, height=12, spp=24, max_bounces=3, use_cache=1)
    _, recs, _ = oracle.trace(o, job, grf=_grf_dummy(job), cache=c, records=True)
    r = recs.reshape(recs.shape[1], recs.shape[2], -1)
    X = ((np.arange(14) + 0.5) - 7) * PITCH
    Y = ((np.arange(12) + 0.5) - 6) * PITCH
    xp = np.broadcast_to(X[None, :, None], r.shape)
    yp = np.broadcast_to(Y[:, None, None], r.shape)
    used = r["cache_cell"] >= 0
    assert used.sum() > 1000
    P = np.stack([r["qx"], r["qy"], np.sqrt(np.maximum(r["r"] ** 2 - (r["qx"] - xp) ** 2 - (r["qy"] - yp) ** 2, 0))], -1)
    f = (P - lo) / (hi - lo) * res
    idx = np.clip(np.floor(f), 0, res - 1).astype(int)
    safe = np.all(np.abs(f - np.round(f)) > 1e-9, axis=-1) & used
    assert safe.sum() > 900
    cell = (idx[..., 2] * res + idx[..., 1]) * res + idx[..., 0]
    assert np.array_equal(cell[safe], r["cache_cell"][safe])
    assert len(np.unique(cell[safe])) >= 9        # the image points spread over several cells
