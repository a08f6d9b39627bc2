"""FP64 CPU oracle of the wave path tracer -- TEST INFRASTRUCTURE ONLY.

Plain, slow and double precision. Only the tests, the smoke check and the
benchmark's CPU-baseline leg use it; the GPU library never imports it and
shares no code with it. Each function cites the passage of the paper it
follows (HoloPathTracer: Eq. 1-5, Sec. 4.1-4.3).
"""
import ctypes as C

import numpy as np

from . import _lib
from .grf import grf_table, grf_phases  # noqa: F401

REC_DTYPE = np.dtype([("sig", np.uint64), ("kind", np.int32), ("bP", np.int32),
                      ("first_gid", np.int32), ("n_hits", np.int32),
                      ("ell", np.float64), ("r", np.float64), ("A", np.float64),
                      ("W", np.float64), ("amp", np.float64), ("qx", np.float64),
                      ("qy", np.float64), ("rev", np.float64), ("cache_cell", np.int32),
                      ("cache_bin", np.int32)])
assert REC_DTYPE.itemsize == C.sizeof(_lib.ORecord)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class OracleScene:
    """A scene dict (see scenes.generators) loaded into the oracle."""

    def __init__(self, sc):
        self._keep = [_c(sc["tri"], np.float32), _c(sc["tri_mat"], np.uint32),
                      _c(sc["sph"], np.float32), _c(sc["sph_mat"], np.uint32),
                      _c(sc["mat_type"], np.uint32), _c(sc["mat_rgb"], np.float32),
                      _c(sc["mat_rough"], np.float32), _c(sc["mat_ior"], np.float32),
                      _c(sc["mat_emit"], np.float32), _c(sc["env"], np.float32),
                      _c(sc.get("mat_pbr", np.tile(np.float32([0.0, 0.5, 0.0, 1.0]), (len(sc["mat_type"]), 1))),
                         np.float32),
                      _c(sc.get("pts", np.zeros((0, 6))), np.float32).reshape(-1, 6)]
        k = self._keep
        d = _lib.OScene(k[0].ctypes.data, len(k[1]), k[1].ctypes.data,
                        k[2].ctypes.data, len(k[3]), k[3].ctypes.data,
                        len(k[4]), k[4].ctypes.data, k[5].ctypes.data, k[6].ctypes.data,
                        k[7].ctypes.data, k[8].ctypes.data, k[9].ctypes.data, k[10].ctypes.data,
                        k[11].ctypes.data if len(k[11]) else None, len(k[11]))
        self.h = _lib.lib().oracle_scene_create(C.byref(d))
        self.n_sph = len(k[3])

    def __del__(self):
        try:
            if self.h:
                _lib.lib().oracle_scene_destroy(self.h)
        except Exception:
            pass

    def closest_hit(self, o, d, tmin=1e-7, exclude=-1, brute=False):
        o = _c(o, np.float64)
        d = _c(d, np.float64)
        t = C.c_double()
        g = C.c_int32()
        _lib.lib().oracle_closest_hit(self.h, o.ctypes.data, d.ctypes.data, float(tmin),
                                      int(exclude), int(brute), C.byref(t), C.byref(g))
        return t.value, g.value


class OracleCache:
    """Radiance cache of the oracle: entries computed on demand (each entry
    is a fixed function of its cell, bin and channel)."""

    def __init__(self, scene, res=64, bins=8, spb=4, max_bounces=6, seed=7):
        self.scene = scene
        self.h = _lib.lib().oracle_cache_create(scene.h, res, bins, spb, max_bounces, seed)
        self.res, self.bins = res, bins

    def __del__(self):
        try:
            if self.h:
                _lib.lib().oracle_cache_destroy(self.h)
        except Exception:
            pass

    def entry(self, comp, cell, b, rounded=True):
        return _lib.lib().oracle_cache_entry(self.h, comp, cell, b, int(rounded))

    def entries(self, comp, cell, b, threads=0):
        """binary16-rounded entries for arrays of (comp, cell, bin)."""
        comp = _c(comp, np.int32)
        cell = _c(cell, np.int32)
        b = _c(b, np.int32)
        out = np.zeros(len(comp))
        _lib.lib().oracle_cache_entries(self.h, len(comp), comp.ctypes.data, cell.ctypes.data,
                                        b.ctypes.data, out.ctypes.data, int(threads))
        return out

    def bounds(self):
        out = np.zeros(6)
        _lib.lib().oracle_cache_bounds(self.h, out.ctypes.data)
        return out[:3], out[3:]


def make_job(job, grf=None):
    """Fill the C job struct from a job dict; grf is the complex128 table
    [gh, gw, T] (kept alive by the caller)."""
    J = _lib.OJob()
    J.width, J.height, J.pitch = job["width"], job["height"], job["pitch"]
    lams = list(job["lambdas"])
    J.n_ch = len(lams)
    for i, l in enumerate(lams):
        J.lam[i] = l
        J.comp[i] = job["comps"][i]
    J.spp, J.max_bounces, J.T = job["spp"], job["max_bounces"], job["T"]
    J.seed = job["seed"]
    J.random_phase, J.use_cache, J.cache_depth = (job["random_phase"], job["use_cache"],
                                                  job["cache_depth"])
    J.nee = int(job.get("nee", 0))
    J.weight_mode = int(job.get("weight_mode", 0))
    for i in range(4):
        J.crop[i] = job["crop"][i]
    J.spp_begin, J.spp_end = job["spp_begin"], job["spp_end"]
    for i in range(12):
        J.holo_from_world[i] = job["holo_from_world"][i]
    J.grf_w, J.grf_h = job["grf_w"], job["grf_h"]
    J.grf = grf.ctypes.data if grf is not None else None
    return J


def crop_dims(job):
    x0, y0, w, h = job["crop"]
    if w == 0 or h == 0:
        return job["width"], job["height"]
    return w, h


def trace(scene, job, grf=None, cache=None, records=False, per_frame=False, threads=0):
    """Oracle field [n_ch, T, h, w] complex128 of a job (Eq. 5 summed over the
    samples, divided by spp). Optional per-path records [n_ch, h, w, n_s] and
    per-path per-frame contributions [n_ch, h, w, n_s, T]."""
    if grf is None:
        grf = grf_table(job["grf_w"], job["grf_h"], job["T"], job["grf_seed"])
    grf = np.ascontiguousarray(grf, dtype=np.complex128)
    assert grf.shape == (job["grf_h"], job["grf_w"], job["T"])
    w, h = crop_dims(job)
    nc = len(job["lambdas"])
    sb, se = job["spp_begin"], job["spp_end"]
    ns = (se - sb) if (sb or se) else job["spp"]
    field = np.zeros((nc, job["T"], h, w), dtype=np.complex128)
    recs = np.zeros((nc, h, w, ns), dtype=REC_DTYPE) if records else None
    rt = np.zeros((nc, h, w, ns, job["T"]), dtype=np.complex128) if per_frame else None
    J = make_job(job, grf)
    rc = _lib.lib().oracle_trace(scene.h, cache.h if cache is not None else None, C.byref(J),
                                 field.ctypes.data,
                                 recs.ctypes.data if recs is not None else None,
                                 rt.ctypes.data if rt is not None else None, int(threads))
    if rc != 0:
        raise ValueError("oracle_trace rejected the job")
    return field, recs, rt


def philox(ctr, key):
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _lib.lib().oracle_philox(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def fresnel(cos_i, eta_i, eta_t):
    return _lib.lib().oracle_fresnel(cos_i, eta_i, eta_t)


def sample_lambert(n, u1, u2):
    out = np.zeros(3)
    _lib.lib().oracle_sample_lambert(_c(n, np.float64).ctypes.data, u1, u2, out.ctypes.data)
    return out


def sample_vndf(V, alpha, u1, u2):
    out = np.zeros(3)
    _lib.lib().oracle_sample_vndf(_c(V, np.float64).ctypes.data, alpha, u1, u2, out.ctypes.data)
    return out


def smith_g1(w, alpha):
    return _lib.lib().oracle_smith_g1(_c(w, np.float64).ctypes.data, alpha)


def principled_eval(params, V, L):
    """(f cos, pdf) of the principled lobes for local directions V, L;
    params = (base, roughness, metallic, specular, clearcoat, gloss)."""
    out = np.zeros(2)
    _lib.lib().oracle_principled_eval(_c(params, np.float64).ctypes.data, _c(V, np.float64).ctypes.data,
                                      _c(L, np.float64).ctypes.data, out.ctypes.data)
    return out[0], out[1]


def principled_sample(params, V, u):
    """(local direction, weight f cos / pdf, lobe index) for uniforms u[0..2]."""
    L = np.zeros(3)
    w = np.zeros(1)
    lobe = np.zeros(1, dtype=np.int32)
    _lib.lib().oracle_principled_sample(_c(params, np.float64).ctypes.data, _c(V, np.float64).ctypes.data,
                                        _c(u, np.float64).ctypes.data, L.ctypes.data, w.ctypes.data,
                                        lobe.ctypes.data)
    return L, float(w[0]), int(lobe[0])


def oct_map(w, bins):
    uv = np.zeros(2)
    b = C.c_int32()
    _lib.lib().oracle_oct(_c(w, np.float64).ctypes.data, bins, uv.ctypes.data, C.byref(b))
    return uv, b.value


def oct_decode(u, v):
    out = np.zeros(3)
    _lib.lib().oracle_oct_decode(u, v, out.ctypes.data)
    return out


def round_fp16(x):
    return _lib.lib().oracle_round_fp16(float(x))


def grf_lookup(job, grf, t, qx, qy):
    """Unit phasor of frame t at hologram-space point (qx, qy)."""
    grf = np.ascontiguousarray(grf, dtype=np.complex128)
    J = make_job(job, grf)
    out = np.zeros(2)
    _lib.lib().oracle_grf_lookup(C.byref(J), int(t), float(qx), float(qy), out.ctypes.data)
    return complex(out[0], out[1])
