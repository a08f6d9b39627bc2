"""ctypes loader and structures for the oracle library (test infrastructure)."""
import ctypes as C
import os

from . import build as _build

_LIB = None

c_double_p = C.c_void_p


class OScene(C.Structure):
    _fields_ = [("tri", C.c_void_p), ("n_tri", C.c_int32), ("tri_mat", C.c_void_p),
                ("sph", C.c_void_p), ("n_sph", C.c_int32), ("sph_mat", C.c_void_p),
                ("n_mat", C.c_int32), ("mat_type", C.c_void_p), ("mat_rgb", C.c_void_p),
                ("mat_rough", C.c_void_p), ("mat_ior", C.c_void_p), ("mat_emit", C.c_void_p),
                ("env", C.c_void_p), ("mat_pbr", C.c_void_p), ("pts", C.c_void_p), ("n_pts", C.c_int32)]


class OJob(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("pitch", C.c_double),
                ("n_ch", C.c_int32), ("lam", C.c_double * 3), ("comp", C.c_int32 * 3),
                ("spp", C.c_int32), ("max_bounces", C.c_int32), ("T", C.c_int32),
                ("seed", C.c_uint64),
                ("random_phase", C.c_int32), ("use_cache", C.c_int32), ("cache_depth", C.c_int32),
                ("crop", C.c_int32 * 4), ("spp_begin", C.c_int32), ("spp_end", C.c_int32),
                ("holo_from_world", C.c_double * 12),
                ("grf_w", C.c_int32), ("grf_h", C.c_int32), ("grf", C.c_void_p), ("nee", C.c_int32),
                ("weight_mode", C.c_int32)]


class ORecord(C.Structure):
    _fields_ = [("sig", C.c_uint64), ("kind", C.c_int32), ("bP", C.c_int32),
                ("first_gid", C.c_int32), ("n_hits", C.c_int32),
                ("ell", C.c_double), ("r", C.c_double), ("A", C.c_double), ("W", C.c_double),
                ("amp", C.c_double), ("qx", C.c_double), ("qy", C.c_double),
                ("rev", C.c_double), ("cache_cell", C.c_int32), ("cache_bin", C.c_int32)]


def lib():
    global _LIB
    if _LIB is None:
        path = os.environ.get("HPT_ORACLE_LIB")   # a sanitizer build of the same source (tests only)
        if not path:
            path = _build.LIB
            if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
                _build.build()
        L = C.CDLL(path)
        vp, i32, u64, dbl = C.c_void_p, C.c_int32, C.c_uint64, C.c_double
        L.oracle_scene_create.restype = vp
        L.oracle_scene_create.argtypes = [C.POINTER(OScene)]
        L.oracle_scene_destroy.argtypes = [vp]
        L.oracle_cache_create.restype = vp
        L.oracle_cache_create.argtypes = [vp, i32, i32, i32, i32, u64]
        L.oracle_cache_destroy.argtypes = [vp]
        L.oracle_cache_entry.restype = dbl
        L.oracle_cache_entry.argtypes = [vp, i32, i32, i32, i32]
        L.oracle_cache_bounds.argtypes = [vp, vp]
        L.oracle_cache_entries.argtypes = [vp, C.c_int64, vp, vp, vp, vp, i32]
        L.oracle_grf_phases.argtypes = [i32, i32, i32, i32, u64, vp, vp]
        L.oracle_philox.argtypes = [vp, vp, vp]
        L.oracle_closest_hit.argtypes = [vp, vp, vp, dbl, i32, i32, vp, vp]
        L.oracle_fresnel.restype = dbl
        L.oracle_fresnel.argtypes = [dbl, dbl, dbl]
        L.oracle_sample_lambert.argtypes = [vp, dbl, dbl, vp]
        L.oracle_sample_vndf.argtypes = [vp, dbl, dbl, dbl, vp]
        L.oracle_smith_g1.restype = dbl
        L.oracle_smith_g1.argtypes = [vp, dbl]
        L.oracle_principled_eval.argtypes = [vp, vp, vp, vp]
        L.oracle_principled_sample.argtypes = [vp, vp, vp, vp, vp, vp]
        L.oracle_oct.argtypes = [vp, i32, vp, vp]
        L.oracle_oct_decode.argtypes = [dbl, dbl, vp]
        L.oracle_round_fp16.restype = dbl
        L.oracle_round_fp16.argtypes = [dbl]
        L.oracle_grf_lookup.argtypes = [C.POINTER(OJob), i32, dbl, dbl, vp]
        L.oracle_trace.restype = i32
        L.oracle_trace.argtypes = [vp, vp, C.POINTER(OJob), vp, vp, vp, i32]
        _LIB = L
    return _LIB
