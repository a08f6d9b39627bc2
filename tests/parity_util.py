"""Helpers for comparing the GPU library with the FP64 oracle on the same
seeded inputs (test infrastructure)."""
import numpy as np

import oracle


def oracle_run(sc, job, cache=None, threads=0):
    o = oracle.OracleScene(sc)
    grf = oracle.grf_table(job["grf_w"], job["grf_h"], job["T"], job["grf_seed"])
    U, rec, rt = oracle.trace(o, job, grf=grf, cache=cache, records=True, per_frame=True,
                              threads=threads)
    return U, rec, rt


def gpu_run(ctx, sid, job):
    U, rec, ct = ctx.trace(sid, job, records=True, contrib=True)
    return U, rec, ct


def cache_agree(recg, reco, comps, gpu_cache, ocache):
    """For paths that ended in the radiance cache, whether the GPU's entry and
    the oracle's entry for that (component, cell, bin) are the same binary16
    value. comps: colour component per channel."""
    ok = np.ones(recg.shape, dtype=bool)
    used = reco["cache_cell"] >= 0
    if not used.any():
        return ok
    ch = np.broadcast_to(np.arange(recg.shape[0]).reshape(-1, 1, 1, 1), recg.shape)[used]
    comp = np.asarray(comps)[ch]
    cell = reco["cache_cell"][used]
    b = reco["cache_bin"][used]
    g = np.ascontiguousarray(gpu_cache[comp, cell, b]).view(np.float16).astype(np.float64)
    o = ocache.entries(comp, cell, b)
    ok[used] = g == o
    return ok


def compare(Ug, recg, ctg, Uo, reco, cto, tol=1e-4, min_match=0.999, extra_match=None):
    """Path signatures must agree on >= min_match of the paths; on matched
    paths the per-pixel complex field error must be <= tol * RMS(field).
    extra_match: further per-path agreement (e.g. identical cache entries)."""
    match = recg["sig"] == reco["sig"]
    if extra_match is not None:
        match = match & extra_match
    frac = float(match.mean())
    # remove unmatched paths' contributions from both fields: [ch,h,w,s,T] -> [ch,T,h,w]
    um = ~match
    dg = np.einsum("chwst,chws->cthw", ctg.astype(np.complex128), um)
    do = np.einsum("chwst,chws->cthw", cto, um)
    Ugm = Ug.astype(np.complex128) - dg
    Uom = Uo - do
    rms = float(np.sqrt(np.mean(np.abs(Uom) ** 2)))
    err = float(np.abs(Ugm - Uom).max() / rms) if rms > 0 else float(np.abs(Ugm).max())
    # per-path phase error of image points on matched paths (radians)
    img = match & (reco["bP"] > 0) & (reco["amp"] != 0)
    dphi = np.angle(np.exp(2j * np.pi * (recg["rev"][img] - reco["rev"][img])))
    ph = (np.percentile(np.abs(dphi), [50, 99]).tolist() + [float(np.abs(dphi).max())]
          if dphi.size else [0.0, 0.0, 0.0])
    # the library's field equals the sum of its own per-path contributions
    self_err = float(np.abs(ctg.astype(np.complex128).sum(3).transpose(0, 3, 1, 2) - Ug).max()
                     / max(rms, 1e-300))
    return dict(match=frac, err=err, rms=rms, phase=ph, self_err=self_err,
                n_paths=int(match.size), ok=frac >= min_match and err <= tol)
