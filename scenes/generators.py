"""Seeded procedural scenes (NumPy PCG64), in metres.

The scene format is a dict of flat arrays:

  tri       float32 [N,3,3]  world-space triangle vertices (instances already baked)
  tri_mat   uint32  [N]      material index per triangle
  sph       float32 [S,4]    analytic spheres (cx, cy, cz, r)
  sph_mat   uint32  [S]
  mat_type  uint32  [M]      LAMBERT / GGX / MIRROR / DIELECTRIC / EMITTER
  mat_rgb   float32 [M,3]    Lambert albedo, or GGX Schlick F0
  mat_rough float32 [M]      GGX alpha
  mat_ior   float32 [M]      dielectric index
  mat_emit  float32 [M,3]    emitter radiance (one-sided, along the winding normal)
  mat_pbr   float32 [M,4]    PRINCIPLED: metallic, specular, clearcoat, clearcoat gloss
  env       float32 [3]      radiance of escaped rays

Primitive ids are global: spheres take ids [0, S), triangles [S, S+N).
The geometric normal of a triangle is (v1-v0) x (v2-v0). Light sources are
emitter quads stored as two triangles. Instancing is resolved here: instance
vertices are transformed in float64 and rounded once to float32, so both the
oracle and the GPU library see the same world-space triangles.

The workload shapes (resolution, counts, depth ranges, material mix) follow
the synthetic stand-ins for the paper's scenes (Section 5.1 uses edited
Mitsuba scenes that are not available; these generators replace them).
"""
import numpy as np

LAMBERT, GGX, MIRROR, DIELECTRIC, EMITTER, PRINCIPLED = 0, 1, 2, 3, 4, 5
MM = 1e-3


class _Builder:
    def __init__(self):
        self.tris, self.tri_mats = [], []
        self.sph, self.sph_mats = [], []
        self.mats = []  # (type, rgb, rough, ior, emit, pbr)

    def material(self, mtype, rgb=(0, 0, 0), rough=0.0, ior=1.0, emit=(0, 0, 0), pbr=(0.0, 0.5, 0.0, 1.0)):
        self.mats.append((mtype, tuple(map(float, rgb)), float(rough), float(ior),
                          tuple(map(float, emit)), tuple(map(float, pbr))))
        return len(self.mats) - 1

    def add_tris(self, verts, mat):
        verts = np.asarray(verts, dtype=np.float64).reshape(-1, 3, 3)
        self.tris.append(verts.astype(np.float32))
        self.tri_mats.append(np.full(len(verts), mat, dtype=np.uint32))

    def add_sphere(self, c, r, mat):
        self.sph.append((c[0], c[1], c[2], r))
        self.sph_mats.append(mat)

    def add_quad(self, p0, e1, e2, mat):
        """Parallelogram p0 + a*e1 + b*e2 as two triangles, normal e1 x e2."""
        p0, e1, e2 = (np.asarray(v, dtype=np.float64) for v in (p0, e1, e2))
        a, b, c, d = p0, p0 + e1, p0 + e1 + e2, p0 + e2
        self.add_tris([[a, b, c], [a, c, d]], mat)

    def finish(self, env=(0, 0, 0)):
        m = self.mats
        tri = (np.concatenate(self.tris) if self.tris else np.zeros((0, 3, 3), np.float32))
        tri_mat = (np.concatenate(self.tri_mats) if self.tri_mats else np.zeros(0, np.uint32))
        return dict(
            tri=np.ascontiguousarray(tri, dtype=np.float32),
            tri_mat=np.ascontiguousarray(tri_mat, dtype=np.uint32),
            sph=np.asarray(self.sph, dtype=np.float32).reshape(-1, 4),
            sph_mat=np.asarray(self.sph_mats, dtype=np.uint32),
            mat_type=np.asarray([x[0] for x in m], dtype=np.uint32),
            mat_rgb=np.asarray([x[1] for x in m], dtype=np.float32).reshape(-1, 3),
            mat_rough=np.asarray([x[2] for x in m], dtype=np.float32),
            mat_ior=np.asarray([x[3] for x in m], dtype=np.float32),
            mat_emit=np.asarray([x[4] for x in m], dtype=np.float32).reshape(-1, 3),
            mat_pbr=np.asarray([x[5] for x in m], dtype=np.float32).reshape(-1, 4),
            env=np.asarray(env, dtype=np.float32),
        )


def scene_arrays_ok(sc):
    """Structural validation of a scene dict (shapes, dtypes, index ranges)."""
    n_m = len(sc["mat_type"])
    ok = sc["tri"].ndim == 3 and sc["tri"].shape[1:] == (3, 3)
    ok &= sc["tri"].dtype == np.float32 and sc["sph"].dtype == np.float32
    ok &= len(sc["tri_mat"]) == len(sc["tri"]) and len(sc["sph_mat"]) == len(sc["sph"])
    ok &= bool(np.all(sc["tri_mat"] < n_m)) and bool(np.all(sc["sph_mat"] < n_m))
    ok &= bool(np.all(np.isfinite(sc["tri"]))) and bool(np.all(np.isfinite(sc["sph"])))
    return bool(ok)


# ----------------------------------------------------------------- meshes

_ICO_CACHE = {}


def _icosphere(level):
    """Unit icosphere: subdivided icosahedron, outward winding."""
    if level in _ICO_CACHE:
        return _ICO_CACHE[level]
    t = (1.0 + 5 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t),
         (0, -1, -t), (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9),
             (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2),
             (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10),
             (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        mid = {}

        def midpoint(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in mid:
                p = verts[a] + verts[b]
                verts.append(p / np.linalg.norm(p))
                mid[key] = len(verts) - 1
            return mid[key]
        nf = []
        for a, b, c in faces:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    V = np.asarray(verts)
    F = np.asarray(faces, dtype=np.int64)
    # orient every face outward
    tri = V[F]
    n = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    flip = np.einsum("ij,ij->i", n, tri.mean(axis=1)) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    _ICO_CACHE[level] = (V, F)
    return V, F


def _sinusoids(rng, n, amp, fmin, fmax):
    a = rng.uniform(0.2, 1.0, n)
    a *= amp / a.sum()
    ang = rng.uniform(0, 2 * np.pi, n)
    f = rng.uniform(fmin, fmax, n)
    ph = rng.uniform(0, 2 * np.pi, n)
    return a, f * np.cos(ang), f * np.sin(ang), ph


def _heightfield(rng, nv_x, nv_y, origin, ax_u, ax_v, normal, amp, fmin, fmax, face):
    """Grid of nv_x x nv_y vertices spanning origin + s*ax_u + t*ax_v, displaced
    along `normal` by a seeded sum of 8 sinusoids (|h| <= amp). Triangles are
    wound so their normals point along `face`."""
    a, fu, fv, ph = _sinusoids(rng, 8, amp, fmin, fmax)
    s = np.linspace(0.0, 1.0, nv_x)
    t = np.linspace(0.0, 1.0, nv_y)
    S, Tt = np.meshgrid(s, t)  # [nv_y, nv_x]
    lu, lv = np.linalg.norm(ax_u), np.linalg.norm(ax_v)
    h = np.zeros_like(S)
    for i in range(8):
        h += a[i] * np.sin(2 * np.pi * (fu[i] * S * lu + fv[i] * Tt * lv) + ph[i])
    P = (np.asarray(origin)[None, None, :] + S[..., None] * np.asarray(ax_u)
         + Tt[..., None] * np.asarray(ax_v) + h[..., None] * np.asarray(normal))
    v00, v10 = P[:-1, :-1], P[:-1, 1:]
    v01, v11 = P[1:, :-1], P[1:, 1:]
    t1 = np.stack([v00, v10, v11], axis=2).reshape(-1, 3, 3)
    t2 = np.stack([v00, v11, v01], axis=2).reshape(-1, 3, 3)
    tri = np.concatenate([t1, t2])
    n = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    flip = n @ np.asarray(face, dtype=np.float64) < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    return tri


def _random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def _material_mix(b, rng, kind):
    if kind == LAMBERT:
        return b.material(LAMBERT, rgb=rng.uniform(0.2, 0.8, 3))
    if kind == GGX:
        return b.material(GGX, rgb=rng.uniform(0.5, 1.0, 3), rough=rng.uniform(0.05, 0.5))
    if kind == MIRROR:
        return b.material(MIRROR)
    return b.material(DIELECTRIC, ior=1.5)


# ----------------------------------------------------------------- scenes

def scene_tiny(seed=0):
    """Three analytic Lambert spheres (r~U[0.5,2] mm, centre x,y~U[-2,2] mm,
    z~U[5,15] mm, albedo U[0.2,0.8]) and a one-sided 6 x 7.5 mm quad light of
    radiance 1 in the plane y=+4 mm facing -y. Resampled until one sphere
    covers the optical axis, no two spheres overlap and none reaches the
    light plane."""
    rng = np.random.default_rng(seed)
    while True:
        r = rng.uniform(0.5, 2.0, 3) * MM
        c = np.stack([rng.uniform(-2, 2, 3) * MM, rng.uniform(-2, 2, 3) * MM,
                      rng.uniform(5, 15, 3) * MM], axis=1)
        alb = rng.uniform(0.2, 0.8, 3)
        covers = np.hypot(c[:, 0], c[:, 1]) < r
        below_light = c[:, 1] + r < 4 * MM
        sep = all(np.linalg.norm(c[i] - c[j]) > r[i] + r[j]
                  for i in range(3) for j in range(i + 1, 3))
        if covers.any() and below_light.all() and sep:
            break
    b = _Builder()
    for i in range(3):
        m = b.material(LAMBERT, rgb=(alb[i],) * 3)
        b.add_sphere(c[i], r[i], m)
    light = b.material(EMITTER, emit=(1.0, 1.0, 1.0))
    b.add_quad((-3 * MM, 4 * MM, 0.5 * MM), (6 * MM, 0, 0), (0, 0, 7.5 * MM), light)
    return b.finish(env=(0, 0, 0))


def scene_mid(seed=1):
    """About 58k triangles: a 128x128-vertex heightfield over x,y in [-4,4] mm
    at z=30 mm (8-sinusoid displacement, |h|<=1.5 mm, Lambert) and 20
    icospheres of subdivision 3 (r~U[0.3,1.5] mm, x,y~U[-2.5,2.5] mm,
    z~U[3,28] mm) with a quarter each Lambert / GGX / mirror / dielectric 1.5.
    An 8 x 8 mm quad light of radiance 1 at y=+6 mm faces -y; env 0.05."""
    rng = np.random.default_rng(seed)
    b = _Builder()
    floor = b.material(LAMBERT, rgb=rng.uniform(0.2, 0.8, 3))
    hf = _heightfield(rng, 128, 128, (-4 * MM, -4 * MM, 30 * MM), (8 * MM, 0, 0),
                      (0, 8 * MM, 0), (0, 0, 1), 1.5 * MM, 0.1 / MM, 0.6 / MM, (0, 0, -1))
    b.add_tris(hf, floor)
    V, F = _icosphere(3)
    placed = []
    while len(placed) < 20:
        r = rng.uniform(0.3, 1.5) * MM
        c = np.array([rng.uniform(-2.5, 2.5) * MM, rng.uniform(-2.5, 2.5) * MM,
                      rng.uniform(3.0, 28.0) * MM])
        if c[2] + r > 28.0 * MM:
            continue
        if any(np.linalg.norm(c - c2) < r + r2 for c2, r2 in placed):
            continue
        placed.append((c, r))
    for i, (c, r) in enumerate(placed):
        m = _material_mix(b, rng, i % 4)
        R = _random_rotation(rng)
        w = (V @ R.T) * r + c
        b.add_tris(w[F], m)
    light = b.material(EMITTER, emit=(1.0, 1.0, 1.0))
    b.add_quad((-4 * MM, 6 * MM, 20 * MM), (8 * MM, 0, 0), (0, 0, 8 * MM), light)
    return b.finish(env=(0.05, 0.05, 0.05))


def scene_large(seed=2, grid=256, ico_level=5, n_inst=36):
    """About 1M triangles at depth 1-50 mm: a displaced floor grid
    (y~-5 mm, z in [1,50] mm) and a displaced ceiling grid (y~+5.5 mm), each
    grid x grid vertices; n_inst instances of a displaced icosphere (level
    ico_level) with mixed materials; a 20 x 12 mm mirror plane at z~48 mm
    tilted 10 degrees about x; a quad light under the ceiling; env 0.05.
    With the defaults: 2*130050 + 36*20480 + 2 + 2 = 997,384 triangles."""
    rng = np.random.default_rng(seed)
    b = _Builder()
    fl = b.material(LAMBERT, rgb=rng.uniform(0.3, 0.8, 3))
    ce = b.material(GGX, rgb=rng.uniform(0.6, 0.9, 3), rough=0.3)
    b.add_tris(_heightfield(rng, grid, grid, (-9 * MM, -5.5 * MM, 1 * MM), (18 * MM, 0, 0),
                            (0, 0, 49 * MM), (0, 1, 0), 0.6 * MM, 0.1 / MM, 0.8 / MM,
                            (0, 1, 0)), fl)
    b.add_tris(_heightfield(rng, grid, grid, (-9 * MM, 5.5 * MM, 1 * MM), (18 * MM, 0, 0),
                            (0, 0, 49 * MM), (0, 1, 0), 0.6 * MM, 0.1 / MM, 0.8 / MM,
                            (0, -1, 0)), ce)
    V, F = _icosphere(ico_level)
    a, fu, fv, ph = _sinusoids(rng, 8, 0.12, 0.5, 2.0)
    theta = np.arccos(np.clip(V[:, 2], -1, 1))
    phi = np.arctan2(V[:, 1], V[:, 0])
    disp = 1.0 + sum(a[i] * np.sin(fu[i] * 3 * theta + np.round(fv[i] * 3) * phi + ph[i])
                     for i in range(8))
    Vd = V * disp[:, None]
    placed = []
    while len(placed) < n_inst:
        r = rng.uniform(0.6, 2.0) * MM
        c = np.array([rng.uniform(-7.5, 7.5) * MM, rng.uniform(-3.5, 3.5) * MM,
                      rng.uniform(4.0, 44.0) * MM])
        if c[1] + 1.15 * r > 4.4 * MM or c[1] - 1.15 * r < -4.8 * MM:
            continue
        if any(np.linalg.norm(c - c2) < 1.15 * (r + r2) for c2, r2 in placed):
            continue
        placed.append((c, r))
    for i, (c, r) in enumerate(placed):
        m = _material_mix(b, rng, i % 4)
        R = _random_rotation(rng)
        b.add_tris(((Vd @ R.T) * r + c)[F], m)
    mirror = b.material(MIRROR)
    ang = np.deg2rad(10.0)
    e1 = np.array([20 * MM, 0, 0])
    e2 = np.array([0, 12 * MM * np.cos(ang), 12 * MM * np.sin(ang)])
    p0 = np.array([-10 * MM, -6 * MM * np.cos(ang), 48 * MM - 6 * MM * np.sin(ang)])
    b.add_quad(p0 + e2, e1, -e2, mirror)  # normal e1 x (-e2) faces the SLM
    light = b.material(EMITTER, emit=(4.0, 4.0, 4.0))
    b.add_quad((-6 * MM, 4.7 * MM, 10 * MM), (12 * MM, 0, 0), (0, 0, 25 * MM), light)
    return b.finish(env=(0.05, 0.05, 0.05))


def scene_translate(sc, t):
    """Copy of a scene moved by the vector t (metres)."""
    out = {k: np.array(v, copy=True) for k, v in sc.items()}
    t32 = np.asarray(t, dtype=np.float64)
    out["tri"] = (sc["tri"].astype(np.float64) + t32).astype(np.float32)
    if len(sc["sph"]):
        s = sc["sph"].astype(np.float64)
        s[:, :3] += t32
        out["sph"] = s.astype(np.float32)
    return out


def scene_depth_rescaled(sc, D):
    """Copy of a scene whose z range is mapped linearly onto [0.8 D, 1.2 D]
    (lateral coordinates unchanged): the depth sweep of the precision study."""
    out = {k: np.array(v, copy=True) for k, v in sc.items()}
    tri = sc["tri"].astype(np.float64)
    zs = [tri[..., 2].ravel()]
    if len(sc["sph"]):
        zs.append(sc["sph"][:, 2].astype(np.float64))
    z = np.concatenate(zs)
    z0, z1 = z.min(), z.max()
    f = lambda v: D * (0.8 + 0.4 * (v - z0) / (z1 - z0))
    tri[..., 2] = f(tri[..., 2])
    out["tri"] = tri.astype(np.float32)
    if len(sc["sph"]):
        s2 = sc["sph"].astype(np.float64)
        s2[:, 2] = f(s2[:, 2])
        out["sph"] = s2.astype(np.float32)
    return out


def make_scene(name, seed=None):
    if name in ("tiny", "config0"):
        return scene_tiny(0 if seed is None else seed)
    if name in ("mid", "config1"):
        return scene_mid(1 if seed is None else seed)
    if name in ("large", "config2"):
        return scene_large(2 if seed is None else seed)
    raise KeyError(name)


# ------------------------------------------------- closed-form test scenes

def empty_scene(env=(0, 0, 0)):
    return _Builder().finish(env=env)


def scene_patch(z0, half, center=(0.0, 0.0), emit=1.0, face=-1, material=None):
    """Square emitter patch of half-width `half` at depth z0, normal along
    face*z (face=-1: towards the SLM)."""
    b = _Builder()
    m = b.material(EMITTER, emit=(emit,) * 3) if material is None else b.material(*material)
    cx, cy = center
    p0 = (cx - half, cy - half, z0)
    if face < 0:
        b.add_quad(p0, (0, 2 * half, 0), (2 * half, 0, 0), m)
    else:
        b.add_quad(p0, (2 * half, 0, 0), (0, 2 * half, 0), m)
    return b.finish()


def scene_mirror_patch(z1, zm, half, center=(0.0, 0.0), mirror_half=5 * MM):
    """Emitter patch at depth z1 facing +z (away from the SLM) and a flat
    mirror at depth zm > z1 facing -z. Light reaches the SLM only through the
    mirror, so the field equals that of the mirror image of the patch."""
    b = _Builder()
    m = b.material(EMITTER, emit=(1.0, 1.0, 1.0))
    cx, cy = center
    b.add_quad((cx - half, cy - half, z1), (2 * half, 0, 0), (0, 2 * half, 0), m)
    mm = b.material(MIRROR)
    b.add_quad((-mirror_half, -mirror_half, zm), (0, 2 * mirror_half, 0),
               (2 * mirror_half, 0, 0), mm)
    return b.finish()


def scene_sheet_stack(n=4096, z0=3 * MM, dz=0.5e-6, half0=50e-6, dhalf=0.1e-6, albedo=0.5, env=1.0):
    """n parallel square Lambert sheets facing the SLM (-z), sheet k at depth
    z0 + k dz with half-width half0 + k dhalf: a ray at lateral distance r
    from the axis passes the nearer, smaller sheets and stops at the first one
    wider than r. The BVH splits the stack along z, so a ray's descent meets
    both children (both boxes span its path) at almost every level and keeps
    a pending far child per level."""
    b = _Builder()
    m = b.material(LAMBERT, rgb=(albedo,) * 3)
    for k in range(n):
        h = half0 + k * dhalf
        b.add_quad((-h, -h, z0 + k * dz), (0, 2 * h, 0), (2 * h, 0, 0), m)
    return b.finish(env=(env,) * 3)


def scene_slab(za, zb, zc, ior=1.5, half=5 * MM, albedo=0.5, env=0.0):
    """Dielectric slab between the planes z=za and z=zb (outward normals -z and
    +z) in front of a Lambert plane at z=zc."""
    b = _Builder()
    d = b.material(DIELECTRIC, ior=ior)
    b.add_quad((-half, -half, za), (0, 2 * half, 0), (2 * half, 0, 0), d)   # normal -z
    b.add_quad((-half, -half, zb), (2 * half, 0, 0), (0, 2 * half, 0), d)   # normal +z
    lam = b.material(LAMBERT, rgb=(albedo,) * 3)
    b.add_quad((-half, -half, zc), (0, 2 * half, 0), (2 * half, 0, 0), lam)
    return b.finish(env=(env,) * 3)


def scene_slab_emitter(za, zb, ze, ior=1.5, half=5 * MM, patch_half=2 * MM):
    """Dielectric slab between z=za and z=zb with an emitter patch of radiance 1
    embedded at za < ze < zb, facing -z."""
    b = _Builder()
    d = b.material(DIELECTRIC, ior=ior)
    b.add_quad((-half, -half, za), (0, 2 * half, 0), (2 * half, 0, 0), d)   # normal -z
    b.add_quad((-half, -half, zb), (2 * half, 0, 0), (0, 2 * half, 0), d)   # normal +z
    e = b.material(EMITTER, emit=(1.0, 1.0, 1.0))
    b.add_quad((-patch_half, -patch_half, ze), (0, 2 * patch_half, 0), (2 * patch_half, 0, 0), e)
    return b.finish()


def scene_ggx_plane(z0, f0, rough, env=1.0, half=5 * MM, tilt_deg=0.0):
    """GGX plane through (0, 0, z0), its normal turned from -z towards +y by
    tilt_deg about the x axis."""
    b = _Builder()
    m = b.material(GGX, rgb=(f0,) * 3, rough=rough)
    a = np.deg2rad(tilt_deg)
    ey = np.array([0.0, np.cos(a), np.sin(a)]) * 2 * half
    ex = np.array([2 * half, 0.0, 0.0])
    p0 = np.array([0.0, 0.0, z0]) - ex / 2 - ey / 2
    b.add_quad(p0, ey, ex, m)
    return b.finish(env=(env,) * 3)


def scene_furnace_sphere(z0, r, mtype=LAMBERT, env=1.0, rgb=(1.0, 1.0, 1.0), rough=0.2,
                         ior=1.5):
    """One analytic sphere in a uniform environment."""
    b = _Builder()
    m = b.material(mtype, rgb=rgb, rough=rough, ior=ior)
    b.add_sphere((0.0, 0.0, z0), r, m)
    return b.finish(env=(env,) * 3)


def scene_lambert_plane(z0, rgb, env=1.0, half=5 * MM):
    b = _Builder()
    m = b.material(LAMBERT, rgb=rgb)
    b.add_quad((-half, -half, z0), (0, 2 * half, 0), (2 * half, 0, 0), m)
    return b.finish(env=(env,) * 3)


def scene_lit_plane(z0, material, light=(1 * MM, 3 * MM, -1 * MM, 1 * MM), h=2 * MM, emit=1.0,
                    blocker=False, half=5 * MM):
    """A plane at depth z0 facing the SLM (material: (type, rgb, rough)) lit
    by a rectangular emitter [x1, x2] x [y1, y2] at depth z0 - h facing the
    plane (+z), beside the SLM's view of the plane; environment black.
    blocker: a black Lambert sheet halfway between them over the light's side."""
    b = _Builder()
    m = b.material(material[0], rgb=material[1], rough=material[2] if len(material) > 2 else 0.0)
    b.add_quad((-half, -half, z0), (0, 2 * half, 0), (2 * half, 0, 0), m)
    x1, x2, y1, y2 = light
    e = b.material(EMITTER, emit=(emit,) * 3)
    b.add_quad((x1, y1, z0 - h), (x2 - x1, 0, 0), (0, y2 - y1, 0), e)   # normal +z
    if blocker:
        k = b.material(LAMBERT, rgb=(0.0, 0.0, 0.0))
        b.add_quad((0.3 * MM, y1 - half, z0 - h / 2), (0, y2 - y1 + 2 * half, 0), (x2, 0, 0), k)
    return b.finish()


def scene_single_tri(z0, size=0.2 * MM, env=1.0, albedo=1.0):
    b = _Builder()
    m = b.material(LAMBERT, rgb=(albedo,) * 3)
    b.add_tris([[(0, 0, z0), (size, 0, z0), (0, size, z0 + size)]], m)
    return b.finish(env=(env,) * 3)


def scene_point_emitters(pts, occluder=None, env=0.0):
    """Point emitters (rows: x, y, z, amplitude per colour component) and,
    optionally, one black Lambert sphere (cx, cy, cz, r) between them and the
    recording plane. Paths that reach the sphere carry no radiance (albedo 0,
    environment `env`), so with env = 0 the field is the emitters' alone."""
    b = _Builder()
    m = b.material(LAMBERT, rgb=(0.0, 0.0, 0.0))
    if occluder is not None:
        b.add_sphere(occluder[:3], occluder[3], m)
    sc = b.finish(env=(env,) * 3)
    sc["pts"] = np.asarray(pts, dtype=np.float32).reshape(-1, 6)
    return sc


def scene_emitter_box(half, radiances, env=0.25):
    """Closed box [-half, half]^3 whose six walls are emitters facing inward,
    wall k (order -x, +x, -y, +y, -z, +z) with radiance radiances[k] (rgb),
    plus a black two-sided Lambert half-plane z = 0, x in [-half, 0]."""
    b = _Builder()
    axes = np.eye(3)
    k = 0
    for a in range(3):
        for sgn in (-1.0, 1.0):
            m = b.material(EMITTER, emit=radiances[k])
            u, v = axes[(a + 1) % 3] * 2 * half, axes[(a + 2) % 3] * 2 * half
            p0 = sgn * half * axes[a] - 0.5 * u - 0.5 * v
            if np.cross(u, v) @ axes[a] * (-sgn) < 0:   # normal must point into the box
                u, v = v, u
            b.add_quad(p0, u, v, m)
            k += 1
    m = b.material(LAMBERT, rgb=(0.0, 0.0, 0.0))
    b.add_quad((-half, -half, 0.0), (0, 2 * half, 0), (half, 0, 0), m)
    return b.finish(env=(env,) * 3)
