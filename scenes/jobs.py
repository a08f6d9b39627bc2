"""Job parameter presets for the synthetic workloads (inputs only).

A job dict carries what the paper's problem statement fixes: the recording
plane (resolution, pitch d), the wavelengths, the hologram-from-world
transform of Eq. 3, the sample budget, the number of time-multiplexed frames
T and the random-phase tables' seed, plus the precision mode and the
radiance-cache switch.
"""
import math

PHASE_FP64, PHASE_SPLIT, PHASE_FP32 = 0, 1, 2

JOB_DEFAULTS = dict(
    width=64, height=64, pitch=8e-6,
    lambdas=[520e-9], comps=[1],
    spp=16, max_bounces=2, T=1,
    seed=0, grf_seed=0, grf_w=0, grf_h=0,
    phase_mode=PHASE_FP64, random_phase=1,
    use_cache=0, cache_depth=1, nee=0,
    crop=(0, 0, 0, 0), spp_begin=0, spp_end=0,
    holo_from_world=(1.0, 0.0, 0.0, 0.0,
                     0.0, 1.0, 0.0, 0.0,
                     0.0, 0.0, 1.0, 0.0),
)

CACHE_DEFAULTS = dict(res=64, bins=8, spb=4, max_bounces=6, seed=7)

RGB = [638e-9, 520e-9, 450e-9]


def grf_size(width, height, pitch, lam_max, z_max, align=32):
    """Periodic random-phase grid: the SLM plus a margin of the widest cone
    footprint (z_max * tan(theta_max)) on each side, rounded up to `align`."""
    s = lam_max / (2 * pitch)
    margin = math.ceil(z_max * s / math.sqrt(1 - s * s) / pitch)
    gw = width + 2 * margin
    gh = height + 2 * margin
    return (-(-gw // align) * align, -(-gh // align) * align)


def job_for_config(idx, **over):
    """Job dict for the workload presets: 0 tiny (64x64 mono), 1 mid (512^2
    RGB T=8), 2 full (1920x1080 RGB T=24 with radiance cache)."""
    j = dict(JOB_DEFAULTS)
    if idx == 0:
        j.update(width=64, height=64, lambdas=[520e-9], comps=[1], spp=16, max_bounces=2,
                 T=1, phase_mode=PHASE_FP64, seed=0, grf_seed=0)
        j["grf_w"], j["grf_h"] = grf_size(64, 64, 8e-6, 520e-9, 17e-3)
    elif idx == 1:
        j.update(width=512, height=512, lambdas=list(RGB), comps=[0, 1, 2], spp=64,
                 max_bounces=4, T=8, phase_mode=PHASE_SPLIT, seed=1, grf_seed=1)
        j["grf_w"], j["grf_h"] = grf_size(512, 512, 8e-6, RGB[0], 32e-3)
    elif idx == 2:
        j.update(width=1920, height=1080, lambdas=list(RGB), comps=[0, 1, 2], spp=256,
                 max_bounces=6, T=24, phase_mode=PHASE_SPLIT, use_cache=1, seed=2,
                 grf_seed=2)
        j["grf_w"], j["grf_h"] = grf_size(1920, 1080, 8e-6, RGB[0], 50e-3)
    else:
        raise KeyError(idx)
    j.update(over)
    return j
