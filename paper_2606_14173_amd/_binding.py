"""ctypes binding of libhpt.so (include/hpt.h): argument marshalling only.

Every step of the wave path tracer runs in the library's gfx950 kernels.
There is no CPU fallback: if the library or a gfx950 device is missing,
loading or creating a context raises.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhpt.so")

STATUS = {0: "HPT_OK", -1: "HPT_EINVAL", -2: "HPT_ENOMEM", -3: "HPT_EBUDGET", -4: "HPT_ENOTFOUND",
          -5: "HPT_EBUSY", -6: "HPT_EDEVICE", -7: "HPT_ETIMEOUT", -8: "HPT_ECANCELED",
          -9: "HPT_ENODEV"}
PHASE_FP64, PHASE_SPLIT, PHASE_FP32 = 0, 1, 2


class HptError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status
        self.name = STATUS.get(status, str(status))


class SceneDesc(C.Structure):
    _fields_ = [("tri", C.c_void_p), ("n_tri", C.c_uint32), ("tri_mat", C.c_void_p),
                ("sph", C.c_void_p), ("n_sph", C.c_uint32), ("sph_mat", C.c_void_p),
                ("n_mat", C.c_uint32), ("mat_type", C.c_void_p), ("mat_rgb", C.c_void_p),
                ("mat_rough", C.c_void_p), ("mat_ior", C.c_void_p), ("mat_emit", C.c_void_p),
                ("env", C.c_void_p), ("mat_pbr", C.c_void_p), ("pts", C.c_void_p), ("n_pts", C.c_uint32)]


class SceneInfo(C.Structure):
    _fields_ = [("n_nodes", C.c_uint32), ("n_prims", C.c_uint32), ("max_depth", C.c_uint32),
                ("reserved", C.c_uint32), ("device_bytes", C.c_uint64), ("build_ms", C.c_double),
                ("bounds", C.c_double * 6)]


class CacheDesc(C.Structure):
    _fields_ = [("res", C.c_uint32), ("bins", C.c_uint32), ("spb", C.c_uint32),
                ("max_bounces", C.c_uint32), ("seed", C.c_uint64)]


class JobDesc(C.Structure):
    _fields_ = [("width", C.c_uint32), ("height", C.c_uint32), ("pitch", C.c_double),
                ("n_ch", C.c_uint32), ("lam", C.c_double * 3), ("comp", C.c_uint32 * 3),
                ("spp", C.c_uint32), ("max_bounces", C.c_uint32), ("T", C.c_uint32),
                ("seed", C.c_uint64), ("grf_seed", C.c_uint64),
                ("grf_w", C.c_uint32), ("grf_h", C.c_uint32),
                ("phase_mode", C.c_uint32), ("random_phase", C.c_uint32),
                ("use_cache", C.c_uint32), ("cache_depth", C.c_uint32),
                ("crop", C.c_uint32 * 4), ("spp_begin", C.c_uint32), ("spp_end", C.c_uint32),
                ("holo_from_world", C.c_double * 12), ("debug", C.c_uint32), ("nee", C.c_uint32),
                ("weight_mode", C.c_uint32)]


class JobStats(C.Structure):
    _fields_ = [("paths", C.c_uint64), ("rays", C.c_uint64), ("batches", C.c_uint64),
                ("queued_ms", C.c_double), ("run_ms", C.c_double), ("trace_gpu_ms", C.c_double)]


class CtxStats(C.Structure):
    _fields_ = [("budget_bytes", C.c_uint64), ("used_bytes", C.c_uint64),
                ("batch_capacity_paths", C.c_uint64), ("batches", C.c_uint64),
                ("jobs_done", C.c_uint64), ("jobs_queued", C.c_uint64),
                ("jobs_running", C.c_uint64)]


class KernelTime(C.Structure):
    _fields_ = [("launches", C.c_uint64), ("items", C.c_uint64), ("total_ms", C.c_double)]


KERNEL_KINDS = ("raygen", "trace", "shade", "accumulate", "cache_reduce", "compact")

PATH_RECORD = np.dtype([("sig", np.uint64), ("kind", np.int32), ("bP", np.int32),
                        ("first_gid", np.int32), ("n_hits", np.int32),
                        ("ell", np.float64), ("r", np.float64), ("A", np.float64),
                        ("W", np.float64), ("amp", np.float64), ("qx", np.float64),
                        ("qy", np.float64), ("rev", np.float64), ("cache_cell", np.int32),
                        ("cache_bin", np.int32)])

# Every entry point declared in include/hpt.h, with its argument types.
_vp, _u32, _u64, _i64, _sz = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int64, C.c_size_t
SIGNATURES = {
    "hpt_create": (C.c_int, [C.c_int, _u64, _vp]),
    "hpt_destroy": (None, [_vp]),
    "hpt_last_error": (C.c_char_p, []),
    "hpt_version": (C.c_char_p, []),
    "hpt_scene_upload": (C.c_int, [_vp, C.POINTER(SceneDesc), C.POINTER(_u64)]),
    "hpt_scene_info_get": (C.c_int, [_vp, _u64, C.POINTER(SceneInfo)]),
    "hpt_scene_release": (C.c_int, [_vp, _u64]),
    "hpt_cache_build": (C.c_int, [_vp, _u64, C.POINTER(CacheDesc)]),
    "hpt_cache_export": (C.c_int, [_vp, _u64, _vp, _sz]),
    "hpt_cache_import": (C.c_int, [_vp, _u64, C.POINTER(CacheDesc), _vp, _sz]),
    "hpt_trace_submit": (C.c_int, [_vp, _u64, C.POINTER(JobDesc), _vp, _vp, C.POINTER(_u64)]),
    "hpt_job_wait": (C.c_int, [_vp, _u64, _i64]),
    "hpt_job_stats_get": (C.c_int, [_vp, _u64, C.POINTER(JobStats)]),
    "hpt_field_read": (C.c_int, [_vp, _u64, _vp, _sz]),
    "hpt_field_device_ptr": (C.c_int, [_vp, _u64, C.POINTER(_vp)]),
    "hpt_paths_read": (C.c_int, [_vp, _u64, _vp, _sz]),
    "hpt_contrib_read": (C.c_int, [_vp, _u64, _vp, _sz]),
    "hpt_sigsum_read": (C.c_int, [_vp, _u64, _vp, _sz]),
    "hpt_job_cancel": (C.c_int, [_vp, _u64]),
    "hpt_job_release": (C.c_int, [_vp, _u64]),
    "hpt_grf_read": (C.c_int, [_vp, _u32, _u32, _u32, _u64, _vp, _sz]),
    "hpt_ctx_stats_get": (C.c_int, [_vp, C.POINTER(CtxStats)]),
    "hpt_profile_set": (C.c_int, [_vp, _u32]),
    "hpt_profile_get": (C.c_int, [_vp, C.POINTER(KernelTime), C.POINTER(_u64), C.POINTER(_u64)]),
    "hpt_profile_reset": (C.c_int, [_vp]),
    "hpt_asm_propagate": (C.c_int, [_vp, _vp, _vp, _u32, _u32, _u32, C.c_double, C.c_double, C.c_double,
                                    _u32, _vp]),
    "hpt_reconstruct": (C.c_int, [_vp, _vp, _u32, _u32, _u32, _u32, C.c_double, C.POINTER(C.c_double), _u32,
                                  C.POINTER(C.c_double), C.c_double, _u32, _vp, _vp]),
    "hpt_encode_phase": (C.c_int, [_vp, _vp, _u32, _u32, _u32, C.c_double, C.c_double, C.c_double, _u32,
                                   C.c_double, _u32, _vp, C.POINTER(C.c_double), _vp]),
    "hpt_debug_fail_batches": (C.c_int, [_vp, _u32]),
    "hpt_asm_propagate_noalloc": (C.c_int, [_vp, _vp, _vp, _u32, _u32, _u32, C.c_double, C.c_double, C.c_double,
                                            _u32, _vp]),
}
ASM_BAND_LIMIT = 1
ENCODE_WARM_START = 2

_LIB = None


def load():
    """Load libhpt.so (built by paper_2606_14173_amd.build); raise if absent."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libhpt.so is not built (run __graft_entry__.build()); "
                              "the wave path tracer has no CPU fallback")
        # One HIP runtime per process: torch's libraries name the runtime
        # without its version suffix, so if libhpt.so loaded the system copy
        # first, torch would load a second copy that finds no device. Loading
        # torch first makes libhpt.so bind to the copy already in the process.
        import torch  # noqa: F401
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _LIB = lib
    return _LIB


def _check(status):
    if status != 0:
        msg = load().hpt_last_error()
        raise HptError(status, msg.decode() if msg else "")


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def job_desc(job):
    """hpt_job_desc from a job dict (see scenes.jobs for the keys)."""
    d = JobDesc()
    d.width, d.height, d.pitch = job["width"], job["height"], job["pitch"]
    lams = list(job["lambdas"])
    d.n_ch = len(lams)
    for i, l in enumerate(lams):
        d.lam[i] = l
        d.comp[i] = job["comps"][i]
    d.spp, d.max_bounces, d.T = job["spp"], job["max_bounces"], job["T"]
    d.seed, d.grf_seed = job["seed"], job["grf_seed"]
    d.grf_w, d.grf_h = job["grf_w"], job["grf_h"]
    d.phase_mode, d.random_phase = job["phase_mode"], job["random_phase"]
    d.use_cache, d.cache_depth = job["use_cache"], job["cache_depth"]
    for i in range(4):
        d.crop[i] = job["crop"][i]
    d.spp_begin, d.spp_end = job["spp_begin"], job["spp_end"]
    for i in range(12):
        d.holo_from_world[i] = job["holo_from_world"][i]
    d.debug = job.get("debug", 0)
    d.nee = job.get("nee", 0)
    d.weight_mode = job.get("weight_mode", 0)
    return d


def crop_dims(job):
    x0, y0, w, h = job["crop"]
    return (job["width"], job["height"]) if (w == 0 or h == 0) else (w, h)


def n_samples(job):
    sb, se = job["spp_begin"], job["spp_end"]
    return (se - sb) if (sb or se) else job["spp"]


class Context:
    """One hpt_ctx on a HIP device (one process per GPU)."""

    def __init__(self, device=0, budget_bytes=0):
        self.lib = load()
        h = C.c_void_p()
        _check(self.lib.hpt_create(device, budget_bytes, C.byref(h)))
        self.h = h
        self.device = device
        self._held = {}   # job id -> caller tensor the job writes, kept alive until wait/release

    def close(self):
        if getattr(self, "h", None):
            self.lib.hpt_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # scenes
    def upload_scene(self, sc):
        keep = [_arr(sc["tri"], np.float32), _arr(sc["tri_mat"], np.uint32),
                _arr(sc["sph"], np.float32), _arr(sc["sph_mat"], np.uint32),
                _arr(sc["mat_type"], np.uint32), _arr(sc["mat_rgb"], np.float32),
                _arr(sc["mat_rough"], np.float32), _arr(sc["mat_ior"], np.float32),
                _arr(sc["mat_emit"], np.float32), _arr(sc["env"], np.float32)]
        pbr = sc.get("mat_pbr")
        keep.append(_arr(pbr, np.float32) if pbr is not None else None)
        pts = _arr(sc.get("pts", np.zeros((0, 6))), np.float32).reshape(-1, 6)
        keep.append(pts)
        d = SceneDesc(keep[0].ctypes.data, len(keep[1]), keep[1].ctypes.data,
                      keep[2].ctypes.data, len(keep[3]), keep[3].ctypes.data,
                      len(keep[4]), keep[4].ctypes.data, keep[5].ctypes.data,
                      keep[6].ctypes.data, keep[7].ctypes.data, keep[8].ctypes.data,
                      keep[9].ctypes.data, keep[10].ctypes.data if keep[10] is not None else None,
                      pts.ctypes.data if len(pts) else None, len(pts))
        sid = C.c_uint64()
        _check(self.lib.hpt_scene_upload(self.h, C.byref(d), C.byref(sid)))
        return sid.value

    def scene_info(self, sid):
        i = SceneInfo()
        _check(self.lib.hpt_scene_info_get(self.h, sid, C.byref(i)))
        return dict(n_nodes=i.n_nodes, n_prims=i.n_prims, max_depth=i.max_depth,
                    device_bytes=i.device_bytes, build_ms=i.build_ms, bounds=list(i.bounds))

    def release_scene(self, sid):
        _check(self.lib.hpt_scene_release(self.h, sid))

    def build_cache(self, sid, res=64, bins=8, spb=4, max_bounces=6, seed=7):
        d = CacheDesc(res, bins, spb, max_bounces, seed)
        _check(self.lib.hpt_cache_build(self.h, sid, C.byref(d)))

    def export_cache(self, sid, res, bins):
        out = np.zeros((3, res ** 3, bins * bins), dtype=np.uint16)
        _check(self.lib.hpt_cache_export(self.h, sid, out.ctypes.data, out.size))
        return out

    def import_cache(self, sid, entries, res=64, bins=8, spb=4, max_bounces=6, seed=7):
        a = _arr(entries, np.uint16)
        d = CacheDesc(res, bins, spb, max_bounces, seed)
        _check(self.lib.hpt_cache_import(self.h, sid, C.byref(d), a.ctypes.data, a.size))

    def _stream(self, stream, tensors):
        """hipStream_t handle to order a call after: an int handle, a torch
        stream, or (None) torch's current stream when a tensor is passed."""
        if stream is not None:
            return stream if isinstance(stream, int) else stream.cuda_stream
        if any(t is not None and not isinstance(t, int) for t in tensors):
            import torch
            return torch.cuda.current_stream(self.device).cuda_stream
        return None

    def _dev_ptr(self, t, n_elems, dtype_name, what):
        """Device pointer of a caller buffer: an int is taken as is; a torch
        tensor must be contiguous, on this context's device, of the given dtype
        and element count."""
        if isinstance(t, int):
            return t
        import torch
        want = getattr(torch, dtype_name)
        if t.dtype != want or not t.is_contiguous() or t.device.type != "cuda" or \
                (t.device.index or 0) != self.device or t.numel() != n_elems:
            raise ValueError("%s must be a contiguous %s tensor on cuda:%d with %d elements (got %s %s on %s, %d)"
                             % (what, dtype_name, self.device, n_elems, t.dtype,
                                "contiguous" if t.is_contiguous() else "strided", t.device, t.numel()))
        return t.data_ptr()

    # jobs
    def submit(self, sid, job, field=None, stream=None):
        """Queue a job; `field` may be a device pointer (int) or a torch
        tensor on the context's device with n_ch*T*h*w complex64 elements
        (kept alive until wait() or release_job()). The job starts after the
        work already enqueued on `stream` (default: torch's current stream
        when a tensor is passed)."""
        d = job_desc(job)
        ptr = None
        if field is not None:
            w, h = crop_dims(job)
            ptr = self._dev_ptr(field, len(job["lambdas"]) * job["T"] * w * h, "complex64", "field")
        st = self._stream(stream, [field])
        jid = C.c_uint64()
        _check(self.lib.hpt_trace_submit(self.h, sid, C.byref(d), ptr, st, C.byref(jid)))
        if field is not None and not isinstance(field, int):
            self._held[jid.value] = field
        return jid.value

    def wait(self, jid, timeout_ms=-1):
        _check(self.lib.hpt_job_wait(self.h, jid, timeout_ms))
        self._held.pop(jid, None)

    def stats(self, jid):
        s = JobStats()
        _check(self.lib.hpt_job_stats_get(self.h, jid, C.byref(s)))
        return {k: getattr(s, k) for k, _ in JobStats._fields_}

    def ctx_stats(self):
        s = CtxStats()
        _check(self.lib.hpt_ctx_stats_get(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in CtxStats._fields_}

    def read_field(self, jid, job):
        w, h = crop_dims(job)
        out = np.zeros((len(job["lambdas"]), job["T"], h, w), dtype=np.complex64)
        _check(self.lib.hpt_field_read(self.h, jid, out.ctypes.data, out.size * 2))
        return out

    def read_paths(self, jid, job):
        w, h = crop_dims(job)
        out = np.zeros((len(job["lambdas"]), h, w, n_samples(job)), dtype=PATH_RECORD)
        _check(self.lib.hpt_paths_read(self.h, jid, out.ctypes.data, out.size))
        return out

    def read_contrib(self, jid, job):
        w, h = crop_dims(job)
        out = np.zeros((len(job["lambdas"]), h, w, n_samples(job), job["T"]), dtype=np.complex64)
        _check(self.lib.hpt_contrib_read(self.h, jid, out.ctypes.data, out.size * 2))
        return out

    def read_sigsum(self, jid, job):
        w, h = crop_dims(job)
        out = np.zeros((len(job["lambdas"]), h, w), dtype=np.uint64)
        _check(self.lib.hpt_sigsum_read(self.h, jid, out.ctypes.data, out.size))
        return out

    def field_ptr(self, jid):
        p = C.c_void_p()
        _check(self.lib.hpt_field_device_ptr(self.h, jid, C.byref(p)))
        return p.value

    def cancel(self, jid):
        _check(self.lib.hpt_job_cancel(self.h, jid))

    def release_job(self, jid):
        _check(self.lib.hpt_job_release(self.h, jid))
        self._held.pop(jid, None)

    def debug_fail_batches(self, n):
        _check(self.lib.hpt_debug_fail_batches(self.h, n))

    def grf(self, gw, gh, T, seed):
        out = np.zeros((gh, gw, T), dtype=np.complex64)
        _check(self.lib.hpt_grf_read(self.h, gw, gh, T, seed, out.ctypes.data, out.size * 2))
        return out

    def asm_propagate(self, src, dst, n_fields, width, height, pitch, lam, distance, band_limit=True,
                      stream=None):
        """Angular-spectrum propagation of n_fields complex64 [height][width]
        fields; src, dst: device pointers (int) or torch tensors."""
        n = n_fields * width * height
        ps = self._dev_ptr(src, n, "complex64", "src")
        pd = self._dev_ptr(dst, n, "complex64", "dst")
        _check(self.lib.hpt_asm_propagate(self.h, ps, pd, n_fields, width, height, float(pitch), float(lam),
                                          float(distance), ASM_BAND_LIMIT if band_limit else 0,
                                          self._stream(stream, [src, dst])))

    def reconstruct(self, fields, n_ch, T, width, height, pitch, lambdas, distances, na, out, band_limit=True,
                    stream=None):
        """Focal stack: mean over the T frames of the intensity of each of the
        n_ch x T complex64 [height][width] fields carried to each distance,
        through a pupil of numerical aperture na (<= 0: none); fields: device
        [n_ch][T][h][w] complex64, out: device [n_ch][n_planes][h][w] float32
        (device pointers (int) or torch tensors)."""
        if len(lambdas) != n_ch:
            raise ValueError("one wavelength per channel")
        pf = self._dev_ptr(fields, n_ch * T * width * height, "complex64", "fields")
        po = self._dev_ptr(out, n_ch * len(distances) * width * height, "float32", "out")
        lam = (C.c_double * len(lambdas))(*[float(x) for x in lambdas])
        dist = (C.c_double * len(distances))(*[float(x) for x in distances])
        _check(self.lib.hpt_reconstruct(self.h, pf, n_ch, T, width, height, float(pitch), lam, len(distances),
                                        dist, float(na), ASM_BAND_LIMIT if band_limit else 0, po,
                                        self._stream(stream, [fields, out])))

    def encode_phase(self, fields, phase, n_fields, width, height, pitch, lam, distance, iterations, lr,
                     band_limit=True, warm_start=False, stream=None):
        """Phase-only encoding of n_fields complex64 [height][width] fields
        into float32 phases (device pointers (int) or torch tensors); returns
        the final relative loss of each field."""
        n = n_fields * width * height
        pf = self._dev_ptr(fields, n, "complex64", "fields")
        pp = self._dev_ptr(phase, n, "float32", "phase")
        loss = (C.c_double * n_fields)()
        flags = (ASM_BAND_LIMIT if band_limit else 0) | (ENCODE_WARM_START if warm_start else 0)
        _check(self.lib.hpt_encode_phase(self.h, pf, n_fields, width, height, float(pitch), float(lam),
                                         float(distance), int(iterations), float(lr), flags, pp, loss,
                                         self._stream(stream, [fields, phase])))
        return np.array(loss[:], dtype=np.float64)

    # profiling
    def profile(self, level):
        _check(self.lib.hpt_profile_set(self.h, level))

    def profile_reset(self):
        _check(self.lib.hpt_profile_reset(self.h))

    def kernel_times(self):
        arr = (KernelTime * len(KERNEL_KINDS))()
        nv, nt = C.c_uint64(), C.c_uint64()
        _check(self.lib.hpt_profile_get(self.h, arr, C.byref(nv), C.byref(nt)))
        out = {k: dict(launches=arr[i].launches, items=arr[i].items, total_ms=arr[i].total_ms)
               for i, k in enumerate(KERNEL_KINDS)}
        out["node_visits"] = nv.value
        out["prim_tests"] = nt.value
        return out

    def trace(self, sid, job, records=False, contrib=False, sigsum=False):
        """Submit, wait and read back: field [n_ch, T, h, w] complex64 and the
        optional debug outputs."""
        j = dict(job)
        j["debug"] = (1 if records else 0) | (2 if contrib else 0) | (4 if sigsum else 0)
        jid = self.submit(sid, j)
        try:
            self.wait(jid)
            out = [self.read_field(jid, j)]
            if records:
                out.append(self.read_paths(jid, j))
            if contrib:
                out.append(self.read_contrib(jid, j))
            if sigsum:
                out.append(self.read_sigsum(jid, j))
        finally:
            self.release_job(jid)
        return out[0] if len(out) == 1 else tuple(out)
