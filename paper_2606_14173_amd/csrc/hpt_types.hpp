// Plain data shared by the host runtime and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hpt.h"

namespace hpt {

constexpr int kMaxT = 64;
constexpr int kStackMax = 64;        // BVH depth bound enforced by the builder
// LDS per traversal workgroup: kStackLds x 256 entries of the stack plus
// kLdsNodes 64-byte nodes (8 KB + 14 KB), so that seven workgroups share a
// CU's 160 KB at seven waves per SIMD
#ifndef HPT_STACK_LDS
#define HPT_STACK_LDS 8
#endif
#ifndef HPT_LDS_NODES
#define HPT_LDS_NODES 224
#endif
// top BVH nodes a traversal workgroup keeps in LDS (the builder stores the
// first levels first; at most its kBvhTopNodes)
constexpr uint32_t kLdsNodes = HPT_LDS_NODES;
constexpr int kStackLds = HPT_STACK_LDS;           // traversal stack entries per lane in LDS
constexpr int kStackSpill = kStackMax - kStackLds;  // further entries per lane in global memory
#ifndef HPT_TRACE_CHUNK
#define HPT_TRACE_CHUNK 64
#endif
constexpr int kTraceChunk = HPT_TRACE_CHUNK;  // queue entries a traversal wave claims at a time
#ifndef HPT_TRACE_GRID
#define HPT_TRACE_GRID 2048
#endif
#ifndef HPT_TRACE_PRIO
#define HPT_TRACE_PRIO 2  // wave issue priority of the traversal (0..3)
#endif
#ifndef HPT_STRAGGLERS
#define HPT_STRAGGLERS 24
#endif
constexpr uint32_t kTraceGridMax = HPT_TRACE_GRID;  // traversal workgroups per launch (8 per CU)
constexpr int kTraceStragglers = HPT_STRAGGLERS;    // lanes a wave's descent stops waiting for
#ifndef HPT_CLAIM_CLASSES
#define HPT_CLAIM_CLASSES 8
#endif
constexpr uint32_t kClaimClasses = HPT_CLAIM_CLASSES;  // chunk classes, one claim counter each
static_assert(kTraceGridMax % kClaimClasses == 0 && kClaimClasses % 8 == 0,
              "the traversal grid (a multiple of 8, capped) must give every class workgroups");
constexpr uint32_t kClaimStride = 32;         // words between claim counters (own 128-byte line)
constexpr float kTmin = 1e-7f;       // self-intersection guard (metres)
constexpr double kTminD = 1e-7;

enum Stage : uint32_t { STAGE_PREFIX = 0, STAGE_TAIL = 1 };
// A queue entry's slot word: the path slot (batches hold at most 2^26
// paths) | stage << 26 | bP << 27 (the interaction of the image point, at
// most 31). The interaction count b of every ray in a queue is the pass
// index, so it is not stored.
constexpr uint32_t kSlotBits = 26, kSlotMask = (1u << kSlotBits) - 1u;
enum UnitKind : uint32_t { UNIT_HOLO = 0, UNIT_CACHE = 1 };

// Lanes per pixel in the accumulation: one per two frames.
__host__ __device__ inline uint32_t frame_group(uint32_t T) { return (T + 1) / 2; }

// Path events hashed into the signature (same codes as the FP64 reference).
enum : uint32_t { EV_MIRROR = 1, EV_DIEL_REFL = 2, EV_DIEL_REFR = 3, EV_LAMBERT = 4, EV_GGX = 5,
                  EV_ABSORB = 6, EV_EMIT = 7, EV_IMAGE_POINT = 8, EV_PRIN_DIFFUSE = 9,
                  EV_PRIN_SPECULAR = 10, EV_PRIN_CLEARCOAT = 11 };
enum : int32_t { K_NONE = 0, K_ESCAPE_PREFIX = 1, K_MAXB_PREFIX = 2, K_EMITTER = 3, K_ENV = 4,
                 K_MAXB_TAIL = 5, K_CACHE = 6, K_ABSORBED = 7 };

struct MaterialDev {
  uint32_t type;
  float rgb[3];
  float rough, ior;
  float emit[3];
  float metallic, specular, clearcoat, clearcoat_gloss;  // HPT_PRINCIPLED
  float pad[3];
};

// What shading needs of a hit primitive, one record per primitive in leaf
// order (the traversal reports the leaf-order index of the closest hit), so
// that a hit costs one 64-byte read. Triangle: unit normal (v1-v0)x(v2-v0)
// and offset n.v0 of its plane in FP64. Sphere: centre and radius (the
// float32 input, exact in FP64).
struct alignas(64) HitRec {
  double g[4];
  int32_t gid;     // global id: spheres [0, n_sph), then triangles
  uint32_t mat;    // material index
  uint32_t pad[6];
};
static_assert(sizeof(HitRec) == 64, "HitRec is one 64-byte record");

// Device view of one resident scene.
struct SceneDev {
  const float4 *nodes;       // BVH2: 4 x float4 per node (two child boxes + links)
  const float4 *prims;       // 3 x float4 per primitive in leaf order
  const HitRec *hits;        // [n_sph + n_tri] in leaf order
  const MaterialDev *mats;
  uint32_t n_sph, n_tri, n_mat, n_nodes;
  float env[3];
  uint32_t pad0;
  // radiance cache
  const uint16_t *cache;     // [3][res^3][bins^2] binary16, or null
  uint32_t cache_res, cache_bins;
  float cache_lo[3], cache_scale[3];   // cell index = floor((x - lo) * scale)
  double cache_lo_d[3], cache_hi_d[3];
  // emitter triangles for next-event estimation, in primitive id order
  const float4 *lights;      // 4 x float4 per light: v0, v1, v2, unit normal (w: material index bits)
  const double *light_cdf;   // running sum of the light areas
  uint32_t n_lights, pad2;
  double light_area;
  // point emitters (a test primitive with a closed-form field)
  const float4 *pts;         // 2 x float4 per emitter: world position (w unused), amplitude rgb (w unused)
  uint32_t n_pts, pad3;
};

// Device view of a job (or of a cache build).
struct JobDev {
  uint32_t width, height;
  double pitch;
  uint32_t crop_x0, crop_y0, crop_w, crop_h;
  uint32_t n_ch;
  uint32_t comp[3];
  double lambda[3], inv_lambda[3], s_cone[3];
  float lambda_f[3], inv_lambda_f[3], s_cone_f[3];
  uint32_t spp, max_bounces, T, phase_mode, random_phase, use_cache, cache_depth, debug;
  uint64_t seed;
  double Tm[12], Ti[12];
  uint32_t identity_T;
  uint32_t grf_w, grf_h;
  const float2 *grf;         // [grf_h][grf_w][T]
  float2 *field;             // [n_ch][T][crop_h][crop_w]
  hpt_path_record *rec;      // debug bit 0
  float2 *contrib;           // debug bit 1: [n_ch][crop_h][crop_w][n_s][T]
  unsigned long long *sigsum;// debug bit 2: [n_ch][crop_h][crop_w]
  uint32_t spp_lo, n_s;      // sample range of the job
  const SceneDev *scene;
  // cache build
  uint16_t *cache_out;       // [3][res^3][bins^2]
  uint32_t cache_res, cache_bins, cache_spb;
  uint32_t nee;              // next-event estimation with MIS in the tail
  uint32_t weight_mode;      // HPT_WEIGHT_RS_AREA: W = r / p(v); HPT_WEIGHT_PAPER_LITERAL: W = 1
};

// A contiguous block of paths of one job: pixels [p_lo, p_lo + p_n) of the
// crop (row-major) x samples [s_lo, s_lo + s_n) of one channel; or cache
// entries x paths per entry of one colour component.
struct UnitDev {
  uint32_t kind, ch;
  uint32_t p_lo, p_n, s_lo, s_n;
  uint32_t slot_base, acc_base;
  const JobDev *job;
  const SceneDev *scene;
};

// One ray queue: entry k is a live ray with the state its path carries from
// bounce to bounce (structure of arrays, so each field is read and written
// coalesced). The FP64 fields are read and written only while the ray is in
// the coherent prefix.
struct RayQueue {
  uint32_t *slot, *unit;
  unsigned long long *sig;         // path signature so far
  float *bpre;                     // beta_pre: product of the delta weights
  float *wt;                       // medium index in the prefix, then the weight W
  float *beta, *L;                 // tail throughput and radiance
  float *pdf;                      // lobe pdf of the ray if next-event estimation covers it (MIS), else 0
  double *ox, *oy, *oz, *dx, *dy, *dz, *ell;  // FP64 ray and optical path length of the coherent prefix
  float4 *ray;                     // 2 per entry: (o, tmin), (d, exclude id bits), traversal input
  float *t;                        // hit distance
  int32_t *prim;                   // leaf-order primitive index of the hit, -1: none
  // A queue filled by shading is compacted per 256-entry chunk of the
  // source queue (entries [256 c, 256 c + cnt[c]) hold rays); off holds the
  // exclusive prefix sums of cnt and idx the entries in order (idx[v] = the
  // entry of ray v), which the next traversal and shading passes read. The
  // first queue (ray generation) is dense and read without idx.
  uint32_t *idx, *cnt, *off;
  uint32_t *tile_sum;              // totals of the counts per tile of 4096 chunks (at most 64)
};

// What the accumulation reads of a path: one 32-byte record per path slot,
// written where the path finds its image point and where it ends, so that
// the scattered writes of a shading pass touch one cache line per path.
struct alignas(32) PathRes {
  uint32_t tex;   // random-field texel of the image point: i0 | j0 << 16
  float amp;      // hologram path: amplitude weight A W / spp; cache path: radiance (0: none)
  float2 cs;      // unit phasor exp(i k r) (FP32 and split phase)
  double fx, fy;  // position of the image point in the texel (FP64: the lookup's
                  // phase is ill-conditioned near zeros of the random field)
};
static_assert(sizeof(PathRes) == 32, "PathRes is one 32-byte record");

struct BatchDev {
  const UnitDev *units;
  uint32_t n_units, n_paths, n_acc, lds_unused;
  // per path slot
  unsigned long long *s_sig;  // final signature (debug records and signature sums only)
  int32_t *s_first;           // first hit (debug records only)
  PathRes *res;                 // results consumed by the accumulation
  double2 *r_cs64;              // unit phasor exp(i k r) in FP64 (FP64 phase)
  RayQueue Q[2];
  uint32_t *counters;        // [0], [1]: queue lengths; [2]: rays traced
  uint32_t *claims;          // traversal claim counters: queue q, class c at [(8 q + c) * kClaimStride]
  unsigned long long *work;  // [0] node visits, [1] primitive tests (counting traversal)
  int32_t *stack_spill;      // [kStackSpill][spill_threads] traversal stack beyond the LDS part
  uint32_t spill_threads;    // threads the spill has a column for
  const SceneDev *scene_uniform;  // the one scene of every unit, or null for mixed batches
  const JobDev *job_uniform;      // the one job of every unit, or null
};

}  // namespace hpt
