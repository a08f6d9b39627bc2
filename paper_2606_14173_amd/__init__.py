"""MI355X (gfx950) wave path tracer: Monte Carlo estimation of the rendering
equation and the Rayleigh-Sommerfeld integral together, T time-multiplexed
random-phase holograms from one path set (HoloPathTracer, Sec. 4).

The C ABI is include/hpt.h; this package is its ctypes binding."""
from ._binding import (  # noqa: F401
    Context, HptError, load, job_desc, PATH_RECORD, SIGNATURES, LIB_PATH, STATUS, ASM_BAND_LIMIT,
    ENCODE_WARM_START,
    PHASE_FP64, PHASE_SPLIT, PHASE_FP32,
)
