/*
 * hpt.h -- C ABI of the MI355X wave path tracer (HoloPathTracer, ACM TOG
 * 45(4) 2026, Sec. 4).
 *
 * The library renders the T time-multiplexed complex fields U_m of a scene on
 * a recording plane (SLM): every pixel sends rays into its recordable cone
 * (Sec. 4.1), delta lobes extend a coherent path and add n_i L_i to the
 * optical path length, the first non-delta hit is the real image point P
 * whose amplitude comes from incoherent radiance rays (Sec. 4.2, Eq. 1), and
 * every frame m accumulates A exp(i(k r + phi_m(Q))) with phi_m from a
 * band-limited random field (Eq. 4, Eq. 5); all frames reuse one path set
 * (Path Reuse, Sec. 4.3).
 *
 * Conventions
 *  - Units are metres. The SLM is the plane z = 0 of hologram space, normal
 *    +z; pixel (i, j) has its centre at ((i+1/2) - W/2) d, ((j+1/2) - H/2) d.
 *  - Every call returns an hpt_status (0 = ok, < 0 = error) and never
 *    throws. hpt_last_error() returns a thread-local message for the last
 *    failing call of the calling thread.
 *  - "host" pointers are ordinary CPU memory, owned by the caller and copied
 *    before the call returns. "device" pointers are HIP device memory on the
 *    context's device.
 *  - Output fields are complex64 stored as interleaved (re, im) float pairs,
 *    layout [channel][frame][crop_h][crop_w], normalised by 1/spp. The RS
 *    prefactor 1/(i lambda) of Eq. 2 is left out (a global constant).
 *  - Calls on one context are thread-safe. Jobs run asynchronously on the
 *    context's own HIP stream; a caller-provided output buffer must stay
 *    alive and untouched until hpt_job_wait() has returned HPT_OK.
 */
#ifndef HPT_H
#define HPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HPT_OK = 0,
  HPT_EINVAL = -1,     /* invalid argument; nothing was changed */
  HPT_ENOMEM = -2,     /* device allocation failed */
  HPT_EBUDGET = -3,    /* the request can never fit the context's HBM budget */
  HPT_ENOTFOUND = -4,  /* unknown scene or job handle */
  HPT_EBUSY = -5,      /* resource still used by a running job */
  HPT_EDEVICE = -6,    /* HIP runtime or kernel error */
  HPT_ETIMEOUT = -7,   /* hpt_job_wait timed out; the job keeps running */
  HPT_ECANCELED = -8,  /* the job was cancelled */
  HPT_ENODEV = -9      /* no usable gfx950 device */
} hpt_status;

typedef struct hpt_ctx hpt_ctx;

/* Create a context on HIP device `device` with a device-memory budget in
 * bytes for scenes, caches, random-phase tables, fields and path state
 * (0 = 90% of the device's free memory). The batch buffers (path state and
 * traversal stack spill) take at most a quarter of it, which sets the batch
 * capacity in paths (a power of two, 2^16 to 2^26); EBUDGET if even 2^16
 * paths do not fit. Spawns the scheduler thread. */
hpt_status hpt_create(int device, uint64_t hbm_budget_bytes, hpt_ctx **out);
/* Cancel queued work, wait for running batches, free everything. */
void hpt_destroy(hpt_ctx *ctx);
const char *hpt_last_error(void);
const char *hpt_version(void);

/* ---------------------------------------------------------------- scenes
 * A scene is triangles (world space, any winding: the geometric normal is
 * (v1-v0) x (v2-v0)) and analytic spheres, each with a material index.
 * Primitive ids are global: spheres [0, n_sph), triangles [n_sph, n_sph +
 * n_tri). Light sources are EMITTER triangles; they emit radiance `emit`
 * on the side of their geometric normal and are black otherwise. */
enum { HPT_LAMBERT = 0, HPT_GGX = 1, HPT_MIRROR = 2, HPT_DIELECTRIC = 3, HPT_EMITTER = 4,
       HPT_PRINCIPLED = 5 };

typedef struct {
  const float *tri;        /* host, [n_tri][3][3] vertex positions */
  uint32_t n_tri;
  const uint32_t *tri_mat; /* host, [n_tri] material index */
  const float *sph;        /* host, [n_sph][4] centre xyz, radius > 0 */
  uint32_t n_sph;
  const uint32_t *sph_mat; /* host, [n_sph] */
  uint32_t n_mat;
  const uint32_t *mat_type;  /* host, [n_mat] HPT_LAMBERT .. HPT_EMITTER */
  const float *mat_rgb;      /* host, [n_mat][3] Lambert albedo / GGX Schlick F0 */
  const float *mat_rough;    /* host, [n_mat] GGX alpha in (0, 1] */
  const float *mat_ior;      /* host, [n_mat] dielectric index > 1 */
  const float *mat_emit;     /* host, [n_mat][3] emitter radiance >= 0 */
  const float *env;          /* host, [3] radiance of rays leaving the scene */
  const float *mat_pbr;      /* host, [n_mat][4] (nullable: 0, 0.5, 0, 1 for every material):
                                HPT_PRINCIPLED metallic, specular, clearcoat, clearcoat gloss,
                                each in [0, 1]. A principled material (Burley 2012, metallic-
                                roughness core) reflects with a Burley diffuse lobe weighted
                                1 - metallic (albedo mat_rgb), a GGX lobe with alpha =
                                mat_rough^2 and Schlick F0 = (1 - metallic) 0.08 specular +
                                metallic mat_rgb, and a GTR1 clearcoat lobe (alpha = 0.1 (1 -
                                gloss) + 0.001 gloss, F0 0.04, Smith masking alpha 0.25) weighted
                                0.25 clearcoat; a lobe is sampled with probability proportional
                                to (1 - metallic, 1, 0.25 clearcoat) and weighted by the full
                                f cos over the combined pdf. */
  const float *pts;          /* host, [n_pts][6] (nullable when n_pts = 0): point emitters, a test
                                primitive with a closed-form field (Eq. 2 for a source concentrated
                                at one point y, isotropic, so the obliquity factor is 1): world
                                position xyz, then the amplitude a >= 0 per colour component.
                                Pixel p receives a exp(i (k r + phi_m(Q))) / r in every frame m,
                                Q = T y, r = |Q - x_p|, when Q is in front of the plane inside the
                                recordable cone (the direction cosines of Q - x_p within the disc
                                of radius lambda/2d, boundary included) and no primitive lies on
                                the segment from T^-1 x_p to y. The term is exact, not sampled; a
                                job adds it once, in its sample range only if that starts at 0. */
  uint32_t n_pts;            /* 0 .. 4096 */
} hpt_scene_desc;

typedef struct {
  uint32_t n_nodes, n_prims, max_depth, reserved;
  uint64_t device_bytes;
  double build_ms;
  double bounds[6]; /* lo xyz, hi xyz of all primitives */
} hpt_scene_info;

/* Validate (finite coordinates, indices in range, positive radii, known
 * material types), build the BVH on the host and copy the scene to the
 * device. Errors: EINVAL, EBUDGET, ENOMEM, EDEVICE. */
hpt_status hpt_scene_upload(hpt_ctx *ctx, const hpt_scene_desc *desc, uint64_t *scene_out);
hpt_status hpt_scene_info_get(hpt_ctx *ctx, uint64_t scene, hpt_scene_info *out);
/* EBUSY while a job that uses the scene is queued or running. */
hpt_status hpt_scene_release(hpt_ctx *ctx, uint64_t scene);

/* ---------------------------------------------------------------- radiance cache
 * Ambient radiance cache ("texture baking", Sec. 4.2; the paper defers its
 * layout to a supplement). Grid: the scene bounds inflated by 1e-3 of their
 * largest extent, res^3 cells; bins: a bins x bins octahedral map of
 * direction. Entry (comp, cell, bin) = mean over spb paths of the radiance
 * seen from a point uniform in the cell along a direction uniform in the
 * bin's octahedral square, traced without the cache up to max_bounces
 * interactions; stored as binary16 (round to nearest even), layout
 * [comp 0..2][cell][bin], cell = (iz*res + iy)*res + ix, bin = bv*bins + bu.
 * A job with use_cache != 0 ends its incoherent tail at the first non-delta
 * lobe whose tail depth >= cache_depth with throughput * entry. */
typedef struct {
  uint32_t res, bins, spb, max_bounces;
  uint64_t seed;
} hpt_cache_desc;

/* Build (or rebuild) the cache of `scene` on the device. Blocks until done. */
hpt_status hpt_cache_build(hpt_ctx *ctx, uint64_t scene, const hpt_cache_desc *desc);
/* Copy the cache to host memory: n = 3 * res^3 * bins^2 binary16 values. */
hpt_status hpt_cache_export(hpt_ctx *ctx, uint64_t scene, uint16_t *host_out, size_t n);
/* Install a cache built elsewhere (e.g. exported from a scene with the same
 * geometry): desc gives its res and bins (spb, max_bounces and seed are
 * recorded only); host: n = 3 * res^3 * bins^2 binary16 values in the layout
 * above, copied before the call returns. The grid is this scene's bounds
 * inflated as for hpt_cache_build. EINVAL on a size mismatch or
 * out-of-range desc, EBUSY while a job uses the scene, EBUDGET, ENOMEM. */
hpt_status hpt_cache_import(hpt_ctx *ctx, uint64_t scene, const hpt_cache_desc *desc, const uint16_t *host,
                            size_t n);

/* ---------------------------------------------------------------- jobs */
enum { HPT_PHASE_FP64 = 0, HPT_PHASE_SPLIT = 1, HPT_PHASE_FP32 = 2 };

typedef struct {
  uint32_t width, height;   /* SLM resolution */
  double pitch;             /* SLM pixel pitch d (m); cone: sin(theta) <= lambda/(2d) */
  uint32_t n_ch;            /* 1..3 wavelengths, traced independently */
  double lambda[3];         /* m */
  uint32_t comp[3];         /* colour component (0..2) of materials used by channel c */
  uint32_t spp;             /* samples per pixel (normalisation 1/spp) */
  uint32_t max_bounces;     /* surface interactions per path, prefix + tail (1..31) */
  uint32_t T;               /* time-multiplexed frames, 1..64 (Eq. 5) */
  uint64_t seed;            /* path random numbers */
  uint64_t grf_seed;        /* spectral phases of the random fields (Eq. 4) */
  uint32_t grf_w, grf_h;    /* periodic random-field grid (texels at pitch d), >= W, H */
  uint32_t phase_mode;      /* HPT_PHASE_FP64 / SPLIT / FP32: precision of the OPL/phase chain */
  uint32_t random_phase;    /* 1: phi_m from the random fields; 0: phi = 0 */
  uint32_t use_cache, cache_depth; /* radiance cache (built beforehand) */
  uint32_t crop[4];         /* x0, y0, w, h of the rendered window; w = h = 0: whole SLM */
  uint32_t spp_begin, spp_end;     /* sample range of this job ([0,0): all); resumable chunks */
  double holo_from_world[12];      /* Eq. 3: affine T, row-major 3x4, x_holo = T x_world */
  uint32_t debug;           /* bit 0: per-path records (<= 2^22 paths); bit 1: per-path
                               per-frame contributions; bit 2: per-pixel signature sums */
  uint32_t nee;             /* 1: next-event estimation in the incoherent tail. At every
                               non-delta tail vertex that is not ended by the radiance cache
                               and has interactions left, one emitter triangle is chosen with
                               probability proportional to area and a point uniform on it;
                               its unoccluded one-sided emission times f cos / pdf_light is
                               added with the power-heuristic weight against the lobe pdf,
                               and emission reached by a lobe sample from such a vertex gets
                               the complementary weight (Eq. 1 by two combined estimators).
                               Random numbers: Philox counter (interaction << 8) | 1.
                               0: BSDF sampling only. */
  uint32_t weight_mode;     /* HPT_WEIGHT_RS_AREA (0): every path is weighted W = r / p(v),
                               p(v) = v_z / (pi s^2) the density of the cone directions per unit
                               solid angle, so A W exp(i k r) is an unbiased sample of Eq. 2's
                               integrand; HPT_WEIGHT_PAPER_LITERAL (1): W = 1, Eq. 5 as printed
                               (the same paths and phases, amplitudes without the weight). */
} hpt_job_desc;
enum { HPT_WEIGHT_RS_AREA = 0, HPT_WEIGHT_PAPER_LITERAL = 1 };

typedef struct {
  uint64_t paths;            /* (channel, pixel, sample) paths traced */
  uint64_t rays;             /* traversal queries */
  uint64_t batches;
  double queued_ms, run_ms;  /* submit -> first batch, first batch -> done */
  double trace_gpu_ms;       /* device time of this job's batches (shared batches split by paths) */
} hpt_job_stats;

/* Per-path debug record, layout [channel][crop_h][crop_w][sample]. */
typedef struct {
  uint64_t sig;              /* FNV-1a over the path's events */
  int32_t kind, bP, first_gid, n_hits;
  double ell, r, A, W, amp, qx, qy, rev;
  int32_t cache_cell, cache_bin;  /* radiance-cache entry used, -1: none */
} hpt_path_record;

/* Queue a job. d_field: device buffer of n_ch*T*crop_h*crop_w complex64
 * (nullable: the library allocates it). hip_stream (a hipStream_t on the
 * context's device, nullable): the job's device work starts only after all
 * work enqueued on that stream before this call (an event is recorded on it
 * here), so a caller may submit right after its own kernels that produce or
 * still use d_field, without synchronising; completion is reported by
 * hpt_job_wait. Validation (EINVAL): sizes zero,
 * T not in [1,64], n_ch not in [1,3], lambda <= 0, lambda/(2 pitch) >= 1,
 * grf smaller than the SLM, crop outside the SLM, spp range empty,
 * max_bounces not in [1,31], non-finite or singular T, use_cache without a
 * built cache. EBUDGET if the job can never fit the budget; otherwise it
 * waits in the queue until memory frees up. */
hpt_status hpt_trace_submit(hpt_ctx *ctx, uint64_t scene, const hpt_job_desc *job,
                            void *d_field, void *hip_stream, uint64_t *job_out);
/* Wait for completion; timeout_ms < 0 waits forever. */
hpt_status hpt_job_wait(hpt_ctx *ctx, uint64_t job, int64_t timeout_ms);
hpt_status hpt_job_stats_get(hpt_ctx *ctx, uint64_t job, hpt_job_stats *out);
/* Copy the finished field to host memory (n_floats = 2 * elements). */
hpt_status hpt_field_read(hpt_ctx *ctx, uint64_t job, float *host_out, size_t n_floats);
/* Device pointer of the field (library-allocated or the caller's). */
hpt_status hpt_field_device_ptr(hpt_ctx *ctx, uint64_t job, void **d_out);
/* Copy per-path records (debug bit 0) / per-frame contributions (bit 1,
 * complex64 [channel][crop_h][crop_w][sample][T]) / per-pixel signature sums
 * (bit 2, uint64 [channel][crop_h][crop_w]) to host memory. */
hpt_status hpt_paths_read(hpt_ctx *ctx, uint64_t job, hpt_path_record *host_out, size_t n);
hpt_status hpt_contrib_read(hpt_ctx *ctx, uint64_t job, float *host_out, size_t n_floats);
hpt_status hpt_sigsum_read(hpt_ctx *ctx, uint64_t job, uint64_t *host_out, size_t n);
/* Remove a queued job or stop a running one at its next batch boundary. */
hpt_status hpt_job_cancel(hpt_ctx *ctx, uint64_t job);
/* Free the job's library-owned memory (its field too, unless caller-owned). */
hpt_status hpt_job_release(hpt_ctx *ctx, uint64_t job);

/* Random-phase table of Eq. 4 as the jobs use it: complex64 [grf_h][grf_w][T],
 * r_t(x, y) = sum over DFT bins with f_x^2 + f_y^2 <= (1/2d)^2 of
 * exp(i xi_t) exp(2 pi i (f_x x + f_y y)) / sqrt(#bins). Builds it (resident,
 * shared by jobs with the same grid, T and seed) and copies it out. */
hpt_status hpt_grf_read(hpt_ctx *ctx, uint32_t grf_w, uint32_t grf_h, uint32_t T,
                        uint64_t grf_seed, float *host_out, size_t n_floats);

/* Context-wide counters: bytes in use against the budget, batches run. */
typedef struct {
  uint64_t budget_bytes, used_bytes, batch_capacity_paths;
  uint64_t batches, jobs_done, jobs_queued, jobs_running;
} hpt_ctx_stats;
hpt_status hpt_ctx_stats_get(hpt_ctx *ctx, hpt_ctx_stats *out);

/* ---------------------------------------------------------------- propagation
 * Angular-spectrum propagation (second stage of the two-stage scheme, Sec.
 * 4.4; angular spectrum as the field's Fourier transform, Sec. 3): carries
 * fields recorded on one plane (e.g. a wave recording plane near the scene)
 * a distance `distance` further from the scene (metres; negative: back
 * towards it). Each field is zero-padded on each axis to the next power of two
 * >= twice its size (field in the top-left corner), Fourier transformed,
 * multiplied by H(f) = exp(+i 2 pi distance sqrt(1/lambda^2 - |f|^2)) (0 for
 * evanescent frequencies; with HPT_ASM_BAND_LIMIT also 0 where
 * |f_x| > 1 / (lambda sqrt((2 distance / (P_x pitch))^2 + 1)), likewise y, the
 * band limit of Matsushima and Shimobaba 2009), transformed back, and cropped
 * to its window. FP32 transforms; the transfer function's phase in FP64.
 *   d_in, d_out: device, complex64 [n_fields][height][width] (interleaved
 *     re, im), row-major; may be the same buffer. Caller-owned.
 *   width, height: 1..4096; pitch, lambda > 0 (metres); distance finite.
 * hip_stream (nullable): the propagation starts after all work enqueued on
 * that stream before the call. Synchronous (returns when d_out is written). Scratch (two [height][P_x]
 * complex64 buffers per field of a chunk of fields, at most 1 GiB, and the
 * transforms' twiddle tables) is taken from the context's budget for the call. EINVAL on bad arguments, EBUDGET if
 * one field's scratch does not fit, EDEVICE on a HIP error. */
#define HPT_ASM_BAND_LIMIT 1u
hpt_status hpt_asm_propagate(hpt_ctx *ctx, const void *d_in, void *d_out, uint32_t n_fields,
                             uint32_t width, uint32_t height, double pitch, double lambda,
                             double distance, uint32_t flags, void *hip_stream);

/* The same propagation without any device allocation, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): it allocates nothing, host or device, and
 * its kernels (those of hpt_asm_propagate) work in a static scratch of
 * 9437184 complex64 (72 MiB) that each device holds from the library's first
 * context until the process ends. Limit: 2 height P_x + P_x + P_y <= 9437184
 * (P_x, P_y: the padded sizes), e.g. one 1920 x 1080 field at a time; larger
 * fields return EINVAL. hip_stream non-null: the work is enqueued on that
 * stream and the call returns without waiting (d_out is ready in stream
 * order); null: it runs on the context's stream and the call returns when
 * d_out is written. The scratch needs no clearing (the transforms pad in
 * LDS). All calls on one device share its scratch and keep the last call's
 * contents: calls that overlap on one device (different streams or threads)
 * race and must be ordered by the caller. Arguments and other errors as for
 * hpt_asm_propagate. */
hpt_status hpt_asm_propagate_noalloc(hpt_ctx *ctx, const void *d_in, void *d_out, uint32_t n_fields,
                                     uint32_t width, uint32_t height, double pitch, double lambda,
                                     double distance, uint32_t flags, void *hip_stream);

/* Reconstruction (simulated viewing of the hologram; the paper's focal
 * stacks and time multiplexing, Sec. 5.3, physical configuration): each of the
 * n_ch x T fields is carried to each of n_planes distances by the ASM of
 * hpt_asm_propagate (padding, evanescent cut and HPT_ASM_BAND_LIMIT as
 * there), low-pass filtered by a circular pupil of numerical aperture na
 * (spatial frequencies with lambda |f| > na removed, na <= 0: no pupil), and
 * the intensities |u|^2 are averaged over the T frames of each channel:
 *   out[c][p] = (1/T) sum_t |ASM_{lambda_c, d_p, na}(U[c][t])|^2.
 *   d_fields: device, complex64 [n_ch][T][height][width]; d_out: device,
 *     float32 [n_ch][n_planes][height][width]; caller-owned, not aliasing.
 *   lambdas (n_ch entries), distances (n_planes entries): host arrays,
 *     metres; lambdas > 0, distances finite; width, height: 1..4096;
 *     n_ch, T >= 1; 1 <= n_planes <= 64; na finite.
 * The forward transforms of a chunk of frames are computed once and reused
 * for every plane. hip_stream (nullable): starts after the work enqueued on
 * it before the call. Synchronous. Scratch (three [height][P_x] complex64
 * buffers per frame of a chunk, at most 1 GiB, and twiddle tables) from the
 * context's budget for the call. EINVAL on bad arguments, EBUDGET if one
 * frame's scratch does not fit, EDEVICE on a HIP error. */
hpt_status hpt_reconstruct(hpt_ctx *ctx, const void *d_fields, uint32_t n_ch, uint32_t T, uint32_t width,
                           uint32_t height, double pitch, const double *lambdas, uint32_t n_planes,
                           const double *distances, double na, uint32_t flags, void *d_out,
                           void *hip_stream);

/* Phase-only encoding (the paper's hologram encoding: SGD under
 * complex-amplitude supervision on one plane with a phase-shift-invariant
 * scale factor; abstract, Sec. 2, Sec. 5.3). For each field U (a rendered
 * SLM-plane field) the phase phi of a phase-only SLM is optimised so that
 * its field A = P exp(i phi) at the supervision plane matches the target
 * V = P U up to one complex factor: loss L = ||A - s V||^2 with the optimal
 * s = <V, A> / <V, V>; P = the ASM of hpt_asm_propagate over `distance`
 * (HPT_ASM_BAND_LIMIT as there). Gradient 2 Im(G conj(exp(i phi))) with
 * G = P^H (A - s V), P^H being the ASM over -distance; Adam (Kingma and Ba
 * 2015: beta1 0.9, beta2 0.999, eps 1e-8, step `lr`) for `iterations` steps.
 * Start: phi = arg U (0 where U = 0), or the contents of d_phase with
 * HPT_ENCODE_WARM_START (Adam's moments start at zero either way).
 *   d_fields: device complex64 [n_fields][height][width]; d_phase: device
 *     float32 [n_fields][height][width] (radians, not wrapped), written;
 *     caller-owned, not aliasing.
 *   loss_out: host, n_fields doubles (nullable): the final relative loss
 *     1 - |<V, A>|^2 / (<V, V> <A, A>) in [0, 1].
 *   width, height 1..4096; pitch, lambda > 0; distance finite;
 *   iterations 0..100000; lr > 0.
 * hip_stream (nullable): starts after the work enqueued on it before the
 * call. Synchronous. Scratch (five [height][width] buffers and two [height][P_x]
 * complex64 buffers per field of a chunk, at most 1 GiB) from the
 * context's budget for the call. EINVAL, EBUDGET, EDEVICE as for
 * hpt_asm_propagate. */
#define HPT_ENCODE_WARM_START 2u
hpt_status hpt_encode_phase(hpt_ctx *ctx, const void *d_fields, uint32_t n_fields, uint32_t width,
                            uint32_t height, double pitch, double lambda, double distance,
                            uint32_t iterations, double lr, uint32_t flags, void *d_phase, double *loss_out,
                            void *hip_stream);

/* ---------------------------------------------------------------- profiling
 * Level 1: HIP events around every kernel launch on the context stream,
 * summed per kernel kind. Level 2: also counts BVH node visits and primitive
 * tests in the traversal kernel (slower; for work accounting only). */
enum { HPT_K_RAYGEN = 0, HPT_K_TRACE = 1, HPT_K_SHADE = 2, HPT_K_ACCUMULATE = 3,
       HPT_K_CACHE_REDUCE = 4, HPT_K_COMPACT = 5 /* ray ordering between interactions */, HPT_K_KINDS = 6 };
typedef struct {
  uint64_t launches;  /* kernel launches timed */
  uint64_t items;     /* rays (trace, shade), paths (raygen), pixel-units (accumulate) */
  double total_ms;    /* sum of event-measured launch durations */
} hpt_kernel_time;
hpt_status hpt_profile_set(hpt_ctx *ctx, uint32_t level);
/* out: HPT_K_KINDS entries; node_visits / prim_tests: level-2 counters (nullable). */
hpt_status hpt_profile_get(hpt_ctx *ctx, hpt_kernel_time *out, uint64_t *node_visits, uint64_t *prim_tests);
hpt_status hpt_profile_reset(hpt_ctx *ctx);

/* ---------------------------------------------------------------- testing
 * Failure injection for tests of the error paths: the next n batches the
 * scheduler packs fail at launch, before any of their work is enqueued,
 * exactly as a launch error would (their jobs end with HPT_EDEVICE once no
 * other batch holds their units). n = 0 turns it off. */
hpt_status hpt_debug_fail_batches(hpt_ctx *ctx, uint32_t n);

#ifdef __cplusplus
}
#endif
#endif /* HPT_H */
