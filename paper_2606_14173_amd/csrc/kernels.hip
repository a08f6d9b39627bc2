// gfx950 kernels of the wave path tracer (wavefront organisation).
//
// One batch = a set of units (blocks of (channel, pixel, sample) paths of
// one or several jobs). Per batch:
//   k_raygen        s1-s2: cone directions from Philox, world-space rays
//   k_trace/k_shade  s3-s5, once per interaction: FP32 closest hit, then the
//                   coherent delta prefix (FP64 or split OPL), the image
//                   point (s6-s7) and the incoherent radiance tail; shading
//                   compacts the live rays of each 256-entry chunk into the
//                   next queue (ballots, no atomics)
//   k_scan/k_index  order the chunks of the next queue (prefix sums of the
//                   chunk counts, then the index list the next pass reads)
//   k_accumulate    s8-s9: Eq. 5 for all T frames of every path (Path Reuse)
//   k_points        exact terms of point emitters, after the accumulation
// Random-phase tables (Eq. 4) are built by k_grf_* once per grid/T/seed.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "kernels.hpp"

namespace hpt {

constexpr int kBlock = 256;

__device__ __forceinline__ uint32_t find_unit(const UnitDev *U, uint32_t n, uint32_t i, bool acc) {
  uint32_t lo = 0, hi = n;  // last unit with base <= i
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    uint32_t base = acc ? U[mid].acc_base : U[mid].slot_base;
    if (base <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// Workgroup index remapped so that each of the 8 XCDs (which receive
// workgroups round-robin) works on one contiguous range of the grid.
__device__ __forceinline__ uint32_t xcd_block() {
  uint32_t g = gridDim.x, b = blockIdx.x;
  if (g % 8u) return b;
  return (b % 8u) * (g / 8u) + b / 8u;
}

// FP32 geometric normal at x of the primitive of record H (unnormalised
// input never reaches here: planes are stored unit length).
__device__ __forceinline__ F3 hit_normal32(const SceneDev &S, const HitRec &H, F3 x) {
  if (H.gid < (int32_t)S.n_sph)
    return (1.0f / (float)H.g[3]) * (x - f3((float)H.g[0], (float)H.g[1], (float)H.g[2]));
  return f3((float)H.g[0], (float)H.g[1], (float)H.g[2]);
}

// Pixel order of a crop: 8x8 tiles, tiles row-major, pixels row-major inside
// a tile (narrower / shorter tiles at the right and bottom edges). Units own
// ranges of this order, so the rays of a unit's first wave groups come from
// one small tile.
__device__ __forceinline__ void crop_xy(const JobDev &J, uint32_t p, uint32_t &cx, uint32_t &cy) {
  uint32_t w = J.crop_w, h = J.crop_h;
  uint32_t band = p / (8u * w);                 // 8-row band
  uint32_t rows = min(8u, h - 8u * band);
  uint32_t o = p - band * 8u * w;
  uint32_t full = (w / 8u) * 8u * rows;         // pixels in the band's full-width tiles
  uint32_t tx, ix, iy;
  if (o < full) {
    tx = o / (8u * rows);
    uint32_t in = o - tx * 8u * rows;
    iy = in / 8u; ix = in - iy * 8u;
    cx = tx * 8u + ix;
  } else {
    uint32_t wp = w - (w / 8u) * 8u;              // width of the last, partial tile
    uint32_t in = o - full;
    iy = in / wp; ix = in - iy * wp;
    cx = (w / 8u) * 8u + ix;
  }
  cy = band * 8u + iy;
}

// Slots of a unit are pixel-major: slot = slot_base + p_local * s_n + s_local.
__device__ __forceinline__ void slot_decode(const UnitDev &U, uint32_t slot, uint32_t &p_local,
                                            uint32_t &s_local) {
  uint32_t l = slot - U.slot_base;
  p_local = l / U.s_n;
  s_local = l - p_local * U.s_n;
}

// Philox key words of path slot `slot` of unit U: (global pixel index,
// sample index) for a hologram path, (cell, bin << 16 | sample) for a cache
// path. A function of the slot, so the ray queues do not carry them.
__device__ __forceinline__ void path_keys(const UnitDev &U, const JobDev &J, uint32_t slot, uint32_t &ka,
                                          uint32_t &kb) {
  uint32_t p_local, s_local;
  slot_decode(U, slot, p_local, s_local);
  if (U.kind == UNIT_HOLO) {
    uint32_t cx, cy;
    crop_xy(J, U.p_lo + p_local, cx, cy);
    ka = (J.crop_y0 + cy) * J.width + J.crop_x0 + cx;
    kb = U.s_lo + s_local;
  } else {
    const uint32_t nb = J.cache_bins * J.cache_bins, e = U.p_lo + p_local, cell = e / nb;
    ka = cell;
    kb = ((e - cell * nb) << 16) | (U.s_lo + s_local);
  }
}

__device__ __forceinline__ size_t rec_index(const JobDev &J, const UnitDev &U, uint32_t p_local,
                                            uint32_t s_local) {
  uint32_t cx, cy;
  crop_xy(J, U.p_lo + p_local, cx, cy);
  return ((size_t)U.ch * J.crop_h * J.crop_w + (size_t)cy * J.crop_w + cx) * J.n_s +
         (U.s_lo + s_local - J.spp_lo);
}

// Morton index of a point of [-1,1]^2 on a grid of 2^kSortBits cells a side
// (ray-sorting key).
constexpr int kSortBits = 5;  // 3 and 4 order the first bounce less coherently
constexpr uint32_t kSortBins = 1u << (2 * kSortBits);
__device__ __forceinline__ uint32_t morton_key(float u, float v) {
  constexpr int n = 1 << kSortBits;
  const int a = min(max((int)floorf((u + 1.f) * (0.5f * n)), 0), n - 1);
  const int b = min(max((int)floorf((v + 1.f) * (0.5f * n)), 0), n - 1);
  uint32_t k = 0;
  for (int i = 0; i < kSortBits; ++i)
    k |= (((uint32_t)a >> i) & 1u) << (2 * i) | (((uint32_t)b >> i) & 1u) << (2 * i + 1);
  return k;
}

// State of one live ray that shading changes, loaded from entry i of queue
// q; the Philox key words are read with it, the direction cosines stay in the
// source entry, are read where they are used, and are copied to the ray's
// next entry when the path continues.
struct RayState {
  uint32_t slot, unit, meta;
  uint32_t ka, kb;           // Philox key words of the path
  unsigned long long sig;
  float bpre, wt, beta, L;   // wt: medium index while in the prefix, then the weight W
  float pdf;                 // lobe pdf of this ray when next-event estimation covers it, else 0
  D3 o, d;                   // FP64 ray of the coherent prefix
  double ell;
};

// The path signature is carried only for jobs that keep per-path records
// or signature sums (sig); the others never read it.
template <bool EXT>
__device__ __forceinline__ void load_state(const RayQueue &Q, uint32_t i, RayState &r, bool sig, const UnitDev &U,
                                           const JobDev &J, uint32_t b) {
  const uint32_t w = Q.slot[i];
  r.slot = w & kSlotMask;
  r.meta = ((w >> kSlotBits) & 1u) | (b << 1) | ((w >> (kSlotBits + 1)) << 7);
  path_keys(U, J, r.slot, r.ka, r.kb);
  r.sig = sig ? Q.sig[i] : kSigInit;
  r.bpre = Q.bpre[i]; r.wt = Q.wt[i];
  // a prefix ray's tail throughput and radiance are 1 and 0: not stored
  const bool tail = (r.meta & 1u) == STAGE_TAIL;
  r.beta = tail ? Q.beta[i] : 1.f;
  r.L = tail ? Q.L[i] : 0.f;
  r.pdf = (EXT && tail) ? Q.pdf[i] : 0.f;
  if ((r.meta & 1u) == STAGE_PREFIX) {
    r.o = D3{Q.ox[i], Q.oy[i], Q.oz[i]};
    r.d = D3{Q.dx[i], Q.dy[i], Q.dz[i]};
    r.ell = Q.ell[i];
  }
}

// s1: cone direction cosines (al, be) of a hologram path with Philox key
// words (gpix, smp): uniform on the disc of radius lambda/(2d), from the
// path's first two uniforms (FP32 phase draws them in FP32). A function of
// the key words, so the passes that need the direction recompute it rather
// than carrying it in the queues.
// The two Philox words the cone direction of path (gpix, smp) is drawn from.
__device__ __forceinline__ U4 cone_words(const UnitDev &U, const JobDev &J, uint32_t gpix, uint32_t smp) {
  return philox(gpix, smp, 0u, J.comp[U.ch] << 16, (uint32_t)J.seed, (uint32_t)(J.seed >> 32));
}

// (al, be) from those words.
__device__ __forceinline__ void cone_from_words(const UnitDev &U, const JobDev &J, uint32_t wx, uint32_t wy,
                                                double &al, double &be) {
  if (J.phase_mode != HPT_PHASE_FP32) {
    const double rad = J.s_cone[U.ch] * sqrt(ud(wx));
    double sn, cs;
    sincospi(2.0 * ud(wy), &sn, &cs);
    al = rad * cs; be = rad * sn;
  } else {
    const float rad = J.s_cone_f[U.ch] * sqrtf(uf(wx));
    float sn, cs;
    sincospif(2.0f * uf(wy), &sn, &cs);
    al = rad * cs; be = rad * sn;
  }
}

__device__ __forceinline__ void cone_cosines(const UnitDev &U, const JobDev &J, uint32_t gpix, uint32_t smp,
                                             double &al, double &be) {
  const U4 w = cone_words(U, J, gpix, smp);
  cone_from_words(U, J, w.x, w.y, al, be);
}

// Entry k of the first queue: what the first shading pass cannot rebuild
// (slot, unit) and the FP32 ray. The start state (signature, throughputs,
// medium, stage) is the same for every path, and the key words and the FP64
// primary ray are functions of the slot, so the first shading pass rebuilds
// them (load_first) instead of reading them.
__device__ __forceinline__ void store_first(const RayQueue &Q, uint32_t k, const RayState &r, F3 o, F3 d) {
  Q.slot[k] = r.slot; Q.unit[k] = r.unit;
  Q.ray[2 * k] = make_float4(o.x, o.y, o.z, kTmin);
  Q.ray[2 * k + 1] = make_float4(d.x, d.y, d.z, __int_as_float(-1));
}

// ------------------------------------------------------------------ raygen
// A block of kRaygenBlock threads takes kRaygenWindow consecutive slots
// (kRaygenSlots per thread: 32 neighbouring pixels x their 256 samples;
// slots are pixel-major) and counting-sorts their rays by direction (32x32
// Morton bins over the cone, or over the octahedral square for cache paths)
// before writing the first queue, so that each wave traces rays of similar
// origin and direction. The queue order changes nothing but the traversal's
// coherence: every path keeps its slot.
constexpr int kRaygenBlock = 1024;
constexpr uint32_t kRaygenSlots = 8;                              // 2 and 4 sort less coherently
constexpr uint32_t kRaygenWindow = kRaygenSlots * kRaygenBlock;  // slots a block sorts

// A batch of one job with at most kLdsUnits units (and, for shading, a scene
// of at most kLdsMats materials) has its descriptors copied to LDS once per
// workgroup and read from there with LDS instructions; otherwise they are
// read from global memory. (Reached through a pointer that may address
// either, they would be read with flat instructions, each of which waits for
// every load in flight.)
constexpr uint32_t kLdsMats = 64;
constexpr uint32_t kLdsUnits = 128;
// Workgroups of a shading launch at most (a multiple of 8): each copies the
// descriptors once and then walks its chunks of the queue.
constexpr uint32_t kShadeGridMax = 32768;

// s1-s2: the primary ray of SLM pixel (px, py) with cone direction cosines
// (al, be): origin at the pixel, direction (al, be, sqrt(1 - al^2 - be^2)),
// both carried into world space by the inverse of T (Eq. 3). FP32 phase
// builds it in FP32 (al, be hold FP32 values there).
__device__ __forceinline__ void primary_ray(const JobDev &J, uint32_t px, uint32_t py, double al, double be,
                                            D3 &O, D3 &d) {
  D3 xp = {((double)px + 0.5 - 0.5 * (double)J.width) * J.pitch,
           ((double)py + 0.5 - 0.5 * (double)J.height) * J.pitch, 0.0};
  if (J.phase_mode != HPT_PHASE_FP32) {
    D3 v = {al, be, sqrt(1.0 - al * al - be * be)};
    if (J.identity_T) {
      O = xp;
      d = normalize(v);
    } else {
      const double *M = J.Ti;
      O = {M[0] * xp.x + M[1] * xp.y + M[2] * xp.z + M[3], M[4] * xp.x + M[5] * xp.y + M[6] * xp.z + M[7],
           M[8] * xp.x + M[9] * xp.y + M[10] * xp.z + M[11]};
      d = normalize(D3{M[0] * v.x + M[1] * v.y + M[2] * v.z, M[4] * v.x + M[5] * v.y + M[6] * v.z,
                       M[8] * v.x + M[9] * v.y + M[10] * v.z});
    }
  } else {
    const float alf = (float)al, bef = (float)be;
    F3 v = f3(alf, bef, sqrtf(1.0f - alf * alf - bef * bef));
    F3 O32, d32;
    if (J.identity_T) {
      O32 = to_f(xp);
      d32 = normalize(v);
    } else {
      float M[12];
      for (int k = 0; k < 12; ++k) M[k] = (float)J.Ti[k];
      F3 x = to_f(xp);
      O32 = f3(M[0] * x.x + M[1] * x.y + M[2] * x.z + M[3], M[4] * x.x + M[5] * x.y + M[6] * x.z + M[7],
               M[8] * x.x + M[9] * x.y + M[10] * x.z + M[11]);
      d32 = normalize(f3(M[0] * v.x + M[1] * v.y + M[2] * v.z, M[4] * v.x + M[5] * v.y + M[6] * v.z,
                         M[8] * v.x + M[9] * v.y + M[10] * v.z));
    }
    O = to_d(O32); d = to_d(d32);
  }
}

// A radiance-cache path: a point uniform in the cell, a direction uniform in
// the bin's octahedral square.
__device__ __forceinline__ void gen_cache_path(const UnitDev &U, const JobDev &J, uint32_t p_local,
                                               uint32_t s_local, RayState &st, uint32_t &ska, uint32_t &skb,
                                               F3 &ro, F3 &rd, uint32_t &key) {
  const SceneDev &S = *J.scene;
  uint32_t comp = U.ch;
  uint32_t e = U.p_lo + p_local, j = U.s_lo + s_local;
  uint32_t nb = J.cache_bins * J.cache_bins;
  uint32_t cell = e / nb, bin = e - cell * nb;
  uint32_t res = J.cache_res;
  uint32_t ix = cell % res, iy = (cell / res) % res, iz = cell / (res * res);
  uint32_t bu = bin % J.cache_bins, bv = bin / J.cache_bins;
  uint32_t ka = cell, kb = (bin << 16) | j;
  uint32_t sw = (comp << 16) | 2u;
  U4 w0 = philox(ka, kb, 0u, sw, (uint32_t)J.seed, (uint32_t)(J.seed >> 32));
  U4 w1 = philox(ka, kb, 1u, sw, (uint32_t)J.seed, (uint32_t)(J.seed >> 32));
  D3 lo = {S.cache_lo_d[0], S.cache_lo_d[1], S.cache_lo_d[2]};
  D3 ext = {S.cache_hi_d[0] - lo.x, S.cache_hi_d[1] - lo.y, S.cache_hi_d[2] - lo.z};
  D3 x = {lo.x + (ix + ud(w0.x)) / res * ext.x, lo.y + (iy + ud(w0.y)) / res * ext.y,
          lo.z + (iz + ud(w0.z)) / res * ext.z};
  double pu = -1.0 + 2.0 * (bu + ud(w0.w)) / J.cache_bins;
  double pv = -1.0 + 2.0 * (bv + ud(w1.x)) / J.cache_bins;
  D3 d = oct_decode64(pu, pv);
  ska = ka;
  skb = kb;
  st.meta = STAGE_TAIL;  // b = 0, bP = 0
  ro = to_f(x); rd = to_f(d);
  key = morton_key((float)pu, (float)pv);
}

// s1-s2 for path slot i (or a cache path) of unit u of the batch: its
// state, read-only key words, FP32 ray and direction-sort key.
__device__ __forceinline__ void gen_path(const UnitDev &U, const JobDev &J, uint32_t u, uint32_t i,
                                         RayState &st, uint32_t &ska, uint32_t &skb, F3 &ro, F3 &rd,
                                         uint32_t &key) {
  uint32_t p_local, s_local;
  slot_decode(U, i, p_local, s_local);
  st.slot = i;
  st.unit = u;
  st.sig = kSigInit;
  st.bpre = 1.f;
  st.wt = 1.0f;  // refractive index of the current medium while in the prefix
  st.beta = 1.f;
  st.L = 0.f;
  st.pdf = 0.f;
  if (U.kind == UNIT_HOLO) {
    uint32_t comp = J.comp[U.ch];
    uint32_t cx, cy;
    crop_xy(J, U.p_lo + p_local, cx, cy);
    uint32_t px = J.crop_x0 + cx, py = J.crop_y0 + cy;
    uint32_t gpix = py * J.width + px, smp = U.s_lo + s_local;
    ska = gpix;
    skb = smp;
    double al, be;
    cone_cosines(U, J, gpix, smp, al, be);
    D3 O, d;
    primary_ray(J, px, py, al, be, O, d);
    st.o = O; st.d = d;
    st.ell = 0.0;
    st.meta = STAGE_PREFIX;
    ro = to_f(O); rd = to_f(d);
    key = morton_key((float)(al / J.s_cone[U.ch]), (float)(be / J.s_cone[U.ch]));
  } else {
    // radiance-cache path: a point uniform in the cell, a direction uniform
    // in the bin's octahedral square
    gen_cache_path(U, J, p_local, s_local, st, ska, skb, ro, rd, key);
  }
}


// State of entry i of the first queue, as gen_path made it (store_first).
__device__ __forceinline__ void load_first(const RayQueue &Q, uint32_t i, RayState &r, const UnitDev &U,
                                           const JobDev &J) {
  r.slot = Q.slot[i];
  path_keys(U, J, r.slot, r.ka, r.kb);
  r.sig = kSigInit;
  r.bpre = 1.f; r.wt = 1.f; r.beta = 1.f; r.L = 0.f; r.pdf = 0.f;
  if (U.kind == UNIT_HOLO) {
    r.meta = STAGE_PREFIX;
    double al, be;
    cone_cosines(U, J, r.ka, r.kb, al, be);
    primary_ray(J, r.ka % J.width, r.ka / J.width, al, be, r.o, r.d);
    r.ell = 0.0;
  } else {
    r.meta = STAGE_TAIL;
  }
}

// Direction-sort key of path slot i of unit u: for a hologram path the
// 32x32 Morton cell of its cone direction cosines over s (from the same
// uniforms as gen_path, in FP32: the key only orders the queue), with the
// pixel (px | py << 16) and the two Philox words of the direction, which ray
// generation keeps for the path's second pass; for a cache path the key
// gen_path gives.
__device__ __forceinline__ uint32_t sort_key(const UnitDev &U, const JobDev &J, uint32_t u, uint32_t i,
                                             uint32_t &pxy, uint32_t &wx, uint32_t &wy) {
  uint32_t p_local, s_local;
  slot_decode(U, i, p_local, s_local);
  pxy = wx = wy = 0u;
  if (U.kind == UNIT_HOLO) {
    uint32_t cx, cy;
    crop_xy(J, U.p_lo + p_local, cx, cy);
    const uint32_t px = J.crop_x0 + cx, py = J.crop_y0 + cy;
    const U4 w = cone_words(U, J, py * J.width + px, U.s_lo + s_local);
    pxy = px | (py << 16);
    wx = w.x; wy = w.y;
    const float rad = sqrtf(uf(w.x));
    float sn, cs;
    sincospif(2.0f * uf(w.y), &sn, &cs);
    return morton_key(rad * cs, rad * sn);
  }
  RayState st;
  uint32_t ska, skb, key;
  F3 ro, rd;
  gen_cache_path(U, J, p_local, s_local, st, ska, skb, ro, rd, key);
  return key;
}

template <bool UNI>
__global__ void __launch_bounds__(kRaygenBlock) k_raygen(BatchDev B) {
  static_assert(kSortBins <= kRaygenBlock, "one thread per sort bin");
  __shared__ uint32_t hist[kSortBins], wsum[kRaygenBlock / 64];
  __shared__ uint16_t perm[kRaygenWindow];
  // what the first pass learnt of each slot of the window, for the second:
  // unit, pixel, the Philox words of the cone direction (the workgroup is
  // alone on its CU, so this LDS costs no occupancy)
  __shared__ uint16_t s_unit[kRaygenWindow];
  __shared__ uint32_t s_pxy[kRaygenWindow], s_wx[kRaygenWindow], s_wy[kRaygenWindow];
  __shared__ JobDev lds_job[1];
  __shared__ UnitDev lds_units[UNI ? kLdsUnits : 1];
  static_assert(kRaygenWindow <= 65536, "sorted positions fit 16 bits");
  const uint32_t g0 = blockIdx.x * kRaygenWindow;
  if (blockIdx.x == 0 && threadIdx.x == 0) { B.counters[0] = B.n_paths; B.counters[1] = 0; }
  if (threadIdx.x < kSortBins) hist[threadIdx.x] = 0;
  if (UNI) {
    const uint32_t t = threadIdx.x;
    const uint32_t *jsrc = (const uint32_t *)B.job_uniform, *usrc = (const uint32_t *)B.units;
    for (uint32_t k = t; k < sizeof(JobDev) / 4; k += blockDim.x) ((uint32_t *)lds_job)[k] = jsrc[k];
    for (uint32_t k = t; k < B.n_units * (uint32_t)(sizeof(UnitDev) / 4); k += blockDim.x)
      ((uint32_t *)lds_units)[k] = usrc[k];
  }
  __syncthreads();
  const UnitDev *Us = UNI ? lds_units : B.units;
  const uint32_t nv = min(kRaygenWindow, B.n_paths - g0);  // slots of this block
  uint32_t key[kRaygenSlots], rank[kRaygenSlots];
#pragma unroll
  for (uint32_t r = 0; r < kRaygenSlots; ++r) {
    const uint32_t w = r * blockDim.x + threadIdx.x, i = g0 + w;
    key[r] = 0;
    rank[r] = 0;
    if (w < nv) {
      // the result record needs no clearing: every path ends in finish(),
      // which writes its amplitude, and the rest of the record is read only
      // where the amplitude is non-zero; the first-hit word only feeds the
      // per-path records of a debug job
      const uint32_t u = find_unit(Us, B.n_units, i, false);
      const JobDev &Jr = UNI ? lds_job[0] : *Us[u].job;
      if (Jr.debug & 1u) B.s_first[i] = -1;
      uint32_t pxy, wx, wy;
      key[r] = sort_key(Us[u], Jr, u, i, pxy, wx, wy);
      s_unit[w] = (uint16_t)u; s_pxy[w] = pxy; s_wx[w] = wx; s_wy[w] = wy;
      rank[r] = atomicAdd(&hist[key[r]], 1u);
    }
  }
  __syncthreads();
  // exclusive prefix sum of the bin counts (thread k owns bin k): within
  // each wave by shuffles, then over the waves' totals
  const uint32_t lane = __lane_id(), wv = threadIdx.x / 64u;
  const uint32_t own = threadIdx.x < kSortBins ? hist[threadIdx.x] : 0u;
  uint32_t inc = own;
  for (uint32_t off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(inc, off);
    if (lane >= off) inc += y;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  uint32_t before = 0;
  for (uint32_t k = 0; k < wv; ++k) before += wsum[k];
  __syncthreads();
  if (threadIdx.x < kSortBins) hist[threadIdx.x] = before + inc - own;  // the bin's first sorted position
  __syncthreads();
#pragma unroll
  for (uint32_t r = 0; r < kRaygenSlots; ++r) {
    const uint32_t w = r * blockDim.x + threadIdx.x;
    if (w < nv) perm[hist[key[r]] + rank[r]] = (uint16_t)w;
  }
  __syncthreads();
  // entry g0 + w of the first queue: the path at sorted position w, its
  // ray built again from what the first pass kept (a hologram path) or
  // generated again (a cache path), so that the queue entries are written in
  // order
  for (uint32_t r = 0; r < kRaygenSlots; ++r) {
    const uint32_t w = r * blockDim.x + threadIdx.x;
    if (w >= nv) break;
    const uint32_t wi = perm[w], k = g0 + wi, u = s_unit[wi];
    const UnitDev &U = Us[u];
    const JobDev &J = UNI ? lds_job[0] : *U.job;
    RayState st;
    F3 ro, rd;
    if (U.kind == UNIT_HOLO) {
      double al, be;
      cone_from_words(U, J, s_wx[wi], s_wy[wi], al, be);
      const uint32_t pxy = s_pxy[wi];
      D3 O, d;
      primary_ray(J, pxy & 0xFFFFu, pxy >> 16, al, be, O, d);
      st.slot = k; st.unit = u;
      ro = to_f(O); rd = to_f(d);
    } else {
      uint32_t ska = 0, skb = 0, kk;
      gen_path(U, J, u, k, st, ska, skb, ro, rd, kk);
    }
    store_first(B.Q[0], g0 + w, st, ro, rd);
  }
}

// ------------------------------------------------------------------ trace
// FP32 closest hit for every ray of queue q (rays in order: entries 0..n-1
// of the dense first queue, else the entries idx lists). The queue is cut into chunks of
// kTraceChunk entries; chunk j belongs to class j mod kClaimClasses, and the
// waves of workgroups with blockIdx mod kClaimClasses = c claim the chunks of
// class c one at a time from that class's counter (zeroed by the shading pass
// of the previous use of the queue), so the claim atomics are spread over
// kClaimClasses addresses (all atomics on one counter serialise). A lane that
// finishes its ray takes the next entry of the wave's chunk, so lanes do not
// idle while the wave's longest ray finishes, and the launch ends when the
// queue is drained, however short the queue. The grid is a multiple of
// kClaimClasses workgroups, so every class is drained.
// The traversal stack is kStackLds entries per lane in LDS, then the lane's
// column of the global spill. Seven waves per SIMD (72 VGPRs, a few spilled
// to scratch outside the node loop) hide more of the node-fetch latency than
// six with no spill.
template <bool COUNT>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7))) k_trace(BatchDev B, int q, int dense) {
  // issue priority over the previous batch's accumulation waves that share
  // the SIMDs (the traversal is on the step's critical path, the
  // accumulation beside it is not)
  __builtin_amdgcn_s_setprio(HPT_TRACE_PRIO);
  __shared__ int32_t stack[kStackLds * kBlock];
  __shared__ v4f top_nodes[4 * (kLdsNodes ? kLdsNodes : 1)];
  // the top levels of the BVH (its first kLdsNodes nodes) in LDS, when every
  // ray of the batch traverses the same scene
  const uint32_t n_top = (kLdsNodes && B.scene_uniform) ? min(kLdsNodes, B.scene_uniform->n_nodes) : 0u;
  if (n_top) {
    const GF4 src = as_global(B.scene_uniform->nodes);
    for (uint32_t k = threadIdx.x; k < 4 * n_top; k += blockDim.x) {
      const float4 v = ld4(src + k);
      top_nodes[k] = v4f{v.x, v.y, v.z, v.w};
    }
    __syncthreads();
  }
  const uint32_t n = B.counters[q];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    B.counters[q ^ 1] = 0;
    B.counters[2] += n;
  }
  const uint32_t cls = blockIdx.x % kClaimClasses;
  uint32_t *claim = B.claims + ((uint32_t)q * kClaimClasses + cls) * kClaimStride;
  const uint32_t n_chunks = (n + kTraceChunk - 1) / kTraceChunk;
  const uint32_t lane = __lane_id();
  const Stack St{(LdsI32)(stack + threadIdx.x), kBlock,
                 (GlbI32)(B.stack_spill + xcd_block() * blockDim.x + threadIdx.x), B.spill_threads,
                 (LF4)top_nodes, n_top};
  uint32_t nv = 0, nt = 0;
  uint32_t next = 0, end = 0;  // unassigned entries of the wave's chunk
  bool more = true;            // the queue may hold unclaimed entries
  int64_t i = -1;              // queue entry of this lane's ray, -1: none
  Trav T;
  const SceneDev *S = B.scene_uniform;
  GF4 N = as_global(S ? S->nodes : nullptr), P = as_global(S ? S->prims : nullptr);
  uint32_t nn = S ? S->n_nodes : 0;
  for (;;) {
    if (more && next >= end && __any(i < 0)) {  // claim the next chunk
      uint32_t k = 0;
      if (lane == 0) k = atomicAdd(claim, 1u);
      const uint32_t j = __shfl(k, 0) * kClaimClasses + cls;  // chunk index
      if (j >= n_chunks) {
        more = false;
      } else {
        next = j * (uint32_t)kTraceChunk;
        end = min(n, next + (uint32_t)kTraceChunk);
      }
    }
    // refill idle lanes from the chunk, in lane order
    unsigned long long need = __ballot(i < 0 && next < end);
    if (need) {
      if (i < 0) {
        uint32_t k = next + (uint32_t)__popcll(need & ((1ull << lane) - 1ull));
        if (k < end) {
          if (!dense) k = B.Q[q].idx[k];   // the k-th ray of a compacted queue
          i = k;
          if (!B.scene_uniform) {
            S = B.units[B.Q[q].unit[k]].scene;
            N = as_global(S->nodes); P = as_global(S->prims); nn = S->n_nodes;
          }
          float4 r0 = B.Q[q].ray[2 * k], r1 = B.Q[q].ray[2 * k + 1];
          trav_init(T, f3(r0.x, r0.y, r0.z), f3(r1.x, r1.y, r1.z), r0.w, __float_as_int(r1.w), nn == 0);
        }
      }
      next = min(end, next + (uint32_t)__popcll(need));
    }
    if (!__any(i >= 0)) {
      if (!more) break;
      continue;
    }
    if (i >= 0) {
      if (T.node != kDone) trav_step<COUNT>(T, N, P, St, nv, nt);
      if (T.node == kDone) {
        B.Q[q].t[i] = T.best.t;
        B.Q[q].prim[i] = T.best.prim;
        i = -1;
      }
    }
  }
  if (COUNT) {
    for (int off = 32; off > 0; off >>= 1) {
      nv += __shfl_xor(nv, off);
      nt += __shfl_xor(nt, off);
    }
    if (lane == 0 && (nv | nt)) {
      atomicAdd(&B.work[0], (unsigned long long)nv);
      atomicAdd(&B.work[1], (unsigned long long)nt);
    }
  }
}

// ------------------------------------------------------------------ shade
struct Emit { bool on, sig; };  // the ray continues; its signature is carried

// A workgroup's continuing rays, staged in LDS (one column per lane, field by
// field so that lanes never share a bank) from the point where shading
// finalises them until the compaction has given them their entry in the next
// queue; this keeps the new state out of registers for the rest of the pass.
struct StageLds {
  uint32_t slot[kBlock], unit[kBlock], meta[kBlock];
  unsigned long long sig[kBlock];
  float bpre[kBlock], wt[kBlock], beta[kBlock], L[kBlock], pdf[kBlock];
  double ox[kBlock], oy[kBlock], oz[kBlock], dx[kBlock], dy[kBlock], dz[kBlock], ell[kBlock];
  float rox[kBlock], roy[kBlock], roz[kBlock], rdx[kBlock], rdy[kBlock], rdz[kBlock];
  int32_t excl[kBlock];
};

__device__ __forceinline__ void stage_put(StageLds &G, const RayState &r, F3 o, F3 d, int32_t excl, Emit &e) {
  const uint32_t t = threadIdx.x;
  G.slot[t] = r.slot; G.unit[t] = r.unit; G.meta[t] = r.meta;
  G.sig[t] = r.sig;
  G.bpre[t] = r.bpre; G.wt[t] = r.wt; G.beta[t] = r.beta; G.L[t] = r.L; G.pdf[t] = r.pdf;
  if ((r.meta & 1u) == STAGE_PREFIX) {
    G.ox[t] = r.o.x; G.oy[t] = r.o.y; G.oz[t] = r.o.z;
    G.dx[t] = r.d.x; G.dy[t] = r.d.y; G.dz[t] = r.d.z;
    G.ell[t] = r.ell;
  }
  G.rox[t] = o.x; G.roy[t] = o.y; G.roz[t] = o.z;
  G.rdx[t] = d.x; G.rdy[t] = d.y; G.rdz[t] = d.z;
  G.excl[t] = excl;
  e.on = true;
}

// Entry k of queue Q from this lane's staged ray (the signature only if
// its job reads signatures).
template <bool EXT>
__device__ __forceinline__ void stage_store(const StageLds &G, const RayQueue &Q, uint32_t k, bool sig) {
  const uint32_t t = threadIdx.x, meta = G.meta[t];
  Q.slot[k] = G.slot[t] | ((meta & 1u) << kSlotBits) | (((meta >> 7) & 31u) << (kSlotBits + 1));
  Q.unit[k] = G.unit[t];
  if (sig) Q.sig[k] = G.sig[t];
  Q.bpre[k] = G.bpre[t]; Q.wt[k] = G.wt[t];
  if ((meta & 1u) == STAGE_TAIL) {  // a prefix ray's are 1 and 0
    Q.beta[k] = G.beta[t]; Q.L[k] = G.L[t];
    if (EXT) Q.pdf[k] = G.pdf[t];
  }
  if ((meta & 1u) == STAGE_PREFIX) {
    Q.ox[k] = G.ox[t]; Q.oy[k] = G.oy[t]; Q.oz[k] = G.oz[t];
    Q.dx[k] = G.dx[t]; Q.dy[k] = G.dy[t]; Q.dz[k] = G.dz[t];
    Q.ell[k] = G.ell[t];
  }
  Q.ray[2 * k] = make_float4(G.rox[t], G.roy[t], G.roz[t], kTmin);
  Q.ray[2 * k + 1] = make_float4(G.rdx[t], G.rdy[t], G.rdz[t], __int_as_float(G.excl[t]));
}

__device__ __forceinline__ void write_rec_tail(const JobDev &J, const UnitDev &U, const BatchDev &B,
                                               uint32_t slot, int32_t kind, uint32_t b, float A,
                                               float amp, unsigned long long sig) {
  uint32_t p_local, s_local;
  slot_decode(U, slot, p_local, s_local);
  auto R = glb(J.rec) + rec_index(J, U, p_local, s_local);
  R->sig = sig; R->kind = kind; R->n_hits = (int32_t)b; R->A = A; R->amp = amp;
  R->first_gid = B.s_first[slot];
  if (kind != K_CACHE) { R->cache_cell = -1; R->cache_bin = -1; }
}

// End of a hologram path or a cache path.
__device__ __forceinline__ void finish(const BatchDev &B, const UnitDev &U, const JobDev &J,
                                       const RayState &r, int32_t kind, uint32_t b, float L,
                                       unsigned long long sig, bool has_image) {
  const uint32_t slot = r.slot;
  sig_add(sig, 0x100u | (uint32_t)kind);
  if (J.debug & 5u) B.s_sig[slot] = sig;  // records and signature sums
  if (U.kind == UNIT_CACHE) { B.res[slot].amp = L; return; }
  float A = 0.f, amp = 0.f;
  if (has_image) {
    A = sqrtf(r.bpre * L);
    amp = A * r.wt / (float)J.spp;
  }
  B.res[slot].amp = amp;
  if (J.debug & 1u) write_rec_tail(J, U, B, slot, kind, b, A, amp, sig);
}

// s6-s7: image point of a path whose coherent prefix ended at a non-delta
// hit after optical path length ell: P' = O + ell v, Q = T P',
// r = |Q - x_p|, weight W = r / p(v) with p(v) = v_z / (pi s^2); phase
// record and the random-field texel that Q falls in.
__device__ __forceinline__ void image_point(const BatchDev &B, const RayQueue &Q, const UnitDev &U,
                                            const JobDev &J, RayState &st, double ell, uint32_t bP) {
  const uint32_t slot = st.slot;
  uint32_t gpix = st.ka;
  uint32_t px = gpix % J.width, py = gpix / J.width;
  double al, be;
  cone_cosines(U, J, st.ka, st.kb, al, be);
  double s = J.s_cone[U.ch];
  double r, qx, qy, u, v, rev;
  float W;
  if (J.phase_mode != HPT_PHASE_FP32) {
    D3 xp = {((double)px + 0.5 - 0.5 * (double)J.width) * J.pitch,
             ((double)py + 0.5 - 0.5 * (double)J.height) * J.pitch, 0.0};
    double vz = sqrt(1.0 - al * al - be * be);
    D3 Q;
    if (J.identity_T) {
      D3 dv = normalize(D3{al, be, vz});
      Q = xp + ell * dv;
    } else {
      const double *Ti = J.Ti, *M = J.Tm;
      D3 O = {Ti[0] * xp.x + Ti[1] * xp.y + Ti[2] * xp.z + Ti[3],
              Ti[4] * xp.x + Ti[5] * xp.y + Ti[6] * xp.z + Ti[7],
              Ti[8] * xp.x + Ti[9] * xp.y + Ti[10] * xp.z + Ti[11]};
      D3 dw = normalize(D3{Ti[0] * al + Ti[1] * be + Ti[2] * vz, Ti[4] * al + Ti[5] * be + Ti[6] * vz,
                           Ti[8] * al + Ti[9] * be + Ti[10] * vz});
      D3 P = O + ell * dw;
      Q = {M[0] * P.x + M[1] * P.y + M[2] * P.z + M[3], M[4] * P.x + M[5] * P.y + M[6] * P.z + M[7],
           M[8] * P.x + M[9] * P.y + M[10] * P.z + M[11]};
    }
    D3 dq = Q - xp;
    r = sqrt(dot(dq, dq));
    W = J.weight_mode == HPT_WEIGHT_PAPER_LITERAL ? 1.0f : (float)(r * (M_PI * s * s) / vz);
    double x = r * J.inv_lambda[U.ch];
    rev = x - floor(x);
    qx = Q.x; qy = Q.y;
    u = Q.x / J.pitch + 0.5 * (double)J.width - 0.5;
    v = Q.y / J.pitch + 0.5 * (double)J.height - 0.5;
  } else {
    float alf = (float)al, bef = (float)be;
    float vz = sqrtf(1.0f - alf * alf - bef * bef);
    F3 xp = f3(((float)px + 0.5f - 0.5f * (float)J.width) * (float)J.pitch,
               ((float)py + 0.5f - 0.5f * (float)J.height) * (float)J.pitch, 0.f);
    F3 Q;
    float ellf = (float)ell;
    if (J.identity_T) {
      Q = xp + ellf * normalize(f3(alf, bef, vz));
    } else {
      float Ti[12], M[12];
      for (int k = 0; k < 12; ++k) { Ti[k] = (float)J.Ti[k]; M[k] = (float)J.Tm[k]; }
      F3 O = f3(Ti[0] * xp.x + Ti[1] * xp.y + Ti[2] * xp.z + Ti[3],
                Ti[4] * xp.x + Ti[5] * xp.y + Ti[6] * xp.z + Ti[7],
                Ti[8] * xp.x + Ti[9] * xp.y + Ti[10] * xp.z + Ti[11]);
      F3 dw = normalize(f3(Ti[0] * alf + Ti[1] * bef + Ti[2] * vz, Ti[4] * alf + Ti[5] * bef + Ti[6] * vz,
                           Ti[8] * alf + Ti[9] * bef + Ti[10] * vz));
      F3 P = O + ellf * dw;
      Q = f3(M[0] * P.x + M[1] * P.y + M[2] * P.z + M[3], M[4] * P.x + M[5] * P.y + M[6] * P.z + M[7],
             M[8] * P.x + M[9] * P.y + M[10] * P.z + M[11]);
    }
    F3 dq = Q - xp;
    float rf = sqrtf(dot(dq, dq));
    float sf = J.s_cone_f[U.ch];
    W = J.weight_mode == HPT_WEIGHT_PAPER_LITERAL ? 1.0f : rf * (3.14159265358979f * sf * sf) / vz;
    float x = rf * J.inv_lambda_f[U.ch];
    rev = x - floorf(x);
    r = rf; qx = Q.x; qy = Q.y;
    u = Q.x / (float)J.pitch + 0.5f * (float)J.width - 0.5f;
    v = Q.y / (float)J.pitch + 0.5f * (float)J.height - 0.5f;
  }
  double fu = floor(u), fv = floor(v);
  int64_t i0 = (int64_t)fu % (int64_t)J.grf_w, j0 = (int64_t)fv % (int64_t)J.grf_h;
  if (i0 < 0) i0 += J.grf_w;
  if (j0 < 0) j0 += J.grf_h;
  PathRes &res = B.res[slot];
  res.tex = (uint32_t)i0 | ((uint32_t)j0 << 16);
  res.fx = u - fu;
  res.fy = v - fv;
  // unit phasor exp(i k r) of the path (the same for all T frames), in the
  // precision the accumulation of this mode sums in
  if (J.phase_mode == HPT_PHASE_FP64) {
    double sn, cs;
    sincospi(2.0 * rev, &sn, &cs);
    B.r_cs64[slot] = make_double2(cs, sn);
  } else {
    float sn, cs;
    sincospif(2.0f * (float)rev, &sn, &cs);
    res.cs = make_float2(cs, sn);
  }
  st.wt = W;
  if (J.debug & 1u) {
    uint32_t p_local, s_local;
    slot_decode(U, slot, p_local, s_local);
    auto R = glb(J.rec) + rec_index(J, U, p_local, s_local);
    R->bP = (int32_t)bP; R->ell = ell; R->r = r; R->W = W; R->qx = qx; R->qy = qy; R->rev = rev;
  }
}

// One interaction of the incoherent tail at x (index b), reached along d_in
// on primitive gid. Returns a ray to trace in `e`, or finishes the path.
// Next-event estimate at the non-delta tail vertex x (material m, primitive
// gid, reached along d_in): an emitter triangle chosen with probability
// proportional to area, a point uniform on it; its unoccluded one-sided
// emission times f cos over the light pdf dist^2 / (cos_y A_total), with
// the power-heuristic weight against the lobe pdf. The occlusion query is a
// traversal of the whole BVH limited to the segment (stack St). The light
// index and visibility enter the signature.
__device__ float next_event(const SceneDev &S, const MaterialDev *M, const MaterialDev &m, uint32_t comp, F3 x,
                            F3 d_in, F3 ng, int32_t gid, U4 w, const Stack &St, unsigned long long &sig) {
  const auto cdf = glb(S.light_cdf);
  const double u0 = ud(w.x) * S.light_area;
  uint32_t lo = 0, hi = S.n_lights;  // first light whose running area exceeds u0
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (cdf[mid] > u0) hi = mid; else lo = mid + 1;
  }
  const uint32_t li = min(lo, S.n_lights - 1u);
  const GF4 Lp = as_global(S.lights + 4 * li);
  const float4 v0 = ld4(Lp), v1 = ld4(Lp + 1), v2 = ld4(Lp + 2), nn = ld4(Lp + 3);
  const float su = sqrtf(uf(w.y)), u2 = uf(w.z);
  const F3 y = (1.0f - su) * f3(v0.x, v0.y, v0.z) + (su * (1.0f - u2)) * f3(v1.x, v1.y, v1.z) +
               (su * u2) * f3(v2.x, v2.y, v2.z);
  F3 om = y - x;
  const float dist = sqrtf(dot(om, om));
  om = (1.0f / dist) * om;
  const float cos_y = -dot(om, f3(nn.x, nn.y, nn.z));
  const BsdfEval e = eval_lobe<true>(m, comp, d_in, ng, om);
  bool vis = false;
  float c = 0.f;
  if (cos_y > 0.f && e.fcos > 0.f) {
    Trav T;
    trav_init(T, x, om, kTmin, gid >= (int32_t)S.n_sph ? gid : -1, S.n_nodes == 0);
    T.best.t = dist * (1.0f - 1e-4f);
    const GF4 N = as_global(S.nodes), P = as_global(S.prims);
    uint32_t nv = 0, nt = 0;
    while (T.node != kDone && T.best.prim < 0) trav_step<false>(T, N, P, St, nv, nt);
    vis = T.best.prim < 0;
    if (vis) {
      const float pl = dist * dist / (cos_y * (float)S.light_area);
      const float wl = pl * pl / (pl * pl + e.pdf * e.pdf);
      const MaterialDev &lm = M[__float_as_uint(nn.w)];
      const float le = comp == 0 ? lm.emit[0] : (comp == 1 ? lm.emit[1] : lm.emit[2]);
      c = le * e.fcos * wl / pl;
    }
  }
  sig_add(sig, 0x60000000u | (vis ? 0x800000u : 0u) | li);
  return c;
}

template <bool EXT>
__device__ __forceinline__ void tail_interaction(const BatchDev &B, const RayQueue &Q, StageLds &G,
                                                 const UnitDev &U, const JobDev &J, const SceneDev &S,
                                                 const MaterialDev *M, RayState &st, F3 x, F3 d_in,
                                                 const HitRec &H, uint32_t b, uint32_t bP, uint32_t comp,
                                                 uint32_t stream, float beta, float L,
                                                 unsigned long long sig, float t_seg, const Stack *St,
                                                 Emit &e) {
  const int32_t gid = H.gid;
  const MaterialDev &m = M[H.mat];
  F3 ng = hit_normal32(S, H, x);
  bool holo = U.kind == UNIT_HOLO;
  const bool nee = EXT && J.nee && S.n_lights > 0;
  if (m.type == HPT_EMITTER) {
    sig_add(sig, EV_EMIT);
    const float cos_y = -dot(d_in, ng);
    if (cos_y > 0.f) {
      float wb = 1.f;  // power-heuristic weight of a lobe sample that next-event estimation also covers
      if (nee && st.pdf > 0.f && gid >= (int32_t)S.n_sph) {
        const float pl = t_seg * t_seg / (cos_y * (float)S.light_area);
        wb = st.pdf * st.pdf / (st.pdf * st.pdf + pl * pl);
      }
      L += beta * (comp == 0 ? m.emit[0] : (comp == 1 ? m.emit[1] : m.emit[2])) * wb;
    }
    finish(B, U, J, st, K_EMITTER, b, L, sig, holo);
    return;
  }
  if (b >= J.max_bounces) { finish(B, U, J, st, K_MAXB_TAIL, b, L, sig, holo); return; }
  U4 w = philox(st.ka, st.kb, b << 8, stream, (uint32_t)J.seed, (uint32_t)(J.seed >> 32));
  Lobe lb = sample_lobe<EXT>(m, comp, d_in, ng, uf(w.x), uf(w.y), uf(w.z));
  sig_add(sig, lb.ev);
  const bool cache_here = holo && J.use_cache && !lb.delta && (b - bP + 1) >= J.cache_depth;
  const bool nee_here = nee && !lb.delta && !cache_here;
  if (EXT && nee_here) {
    U4 wn = philox(st.ka, st.kb, (b << 8) | 1u, stream, (uint32_t)J.seed, (uint32_t)(J.seed >> 32));
    L += beta * next_event(S, M, m, comp, x, d_in, ng, gid, wn, *St, sig);
  }
  if (lb.w == 0.f) { finish(B, U, J, st, K_ABSORBED, b, L, sig, holo); return; }
  st.pdf = (EXT && nee_here) ? eval_lobe<EXT>(m, comp, d_in, ng, lb.d).pdf : 0.f;
  beta *= lb.w;
  if (cache_here) {
    uint32_t res = S.cache_res, nb = S.cache_bins * S.cache_bins;
    int ix = (int)floorf((x.x - S.cache_lo[0]) * S.cache_scale[0]);
    int iy = (int)floorf((x.y - S.cache_lo[1]) * S.cache_scale[1]);
    int iz = (int)floorf((x.z - S.cache_lo[2]) * S.cache_scale[2]);
    ix = min(max(ix, 0), (int)res - 1); iy = min(max(iy, 0), (int)res - 1); iz = min(max(iz, 0), (int)res - 1);
    uint32_t cell = ((uint32_t)iz * res + (uint32_t)iy) * res + (uint32_t)ix;
    uint32_t bin = oct_bin(lb.d, S.cache_bins);
    sig_add(sig, 0x40000000u | cell);
    sig_add(sig, 0x50000000u | bin);
    if (J.debug & 1u) {
      uint32_t p_local, s_local;
      slot_decode(U, st.slot, p_local, s_local);
      auto R = glb(J.rec) + rec_index(J, U, p_local, s_local);
      R->cache_cell = (int32_t)cell;
      R->cache_bin = (int32_t)bin;
    }
    size_t ce = (size_t)comp * res * res * res * nb + (size_t)cell * nb + bin;
    L += beta * __half2float(__ushort_as_half(glb(S.cache)[ce]));
    finish(B, U, J, st, K_CACHE, b, L, sig, true);
    return;
  }
  st.beta = beta;
  st.L = L;
  st.sig = sig;
  st.meta = STAGE_TAIL | (b << 1) | (bP << 7);
  stage_put(G, st, x, lb.d, gid >= (int32_t)S.n_sph ? gid : -1, e);
}

// Shade entry i of queue q, whose state is st; st is updated in place for a
// path that continues (e.on). U, J, S, M: its unit, job, scene and the
// scene's materials; t, hp: the hit the traversal reported, H its record
// (read when hp >= 0).
template <bool EXT>
__device__ __forceinline__ void shade_one(const BatchDev &B, int q, uint32_t i, RayState &st, StageLds &G,
                                          const UnitDev &U, const JobDev &J, const SceneDev &S,
                                          const MaterialDev *M, float t, int32_t hp, const HitRec &H,
                                          const Stack *St, Emit &e) {
  const RayQueue &Q = B.Q[q];
  uint32_t meta = st.meta;
  uint32_t stage = meta & 1u, b = (meta >> 1) & 63u, bP = (meta >> 7) & 63u;
  unsigned long long sig = st.sig;
  bool holo = U.kind == UNIT_HOLO;
  uint32_t comp = holo ? J.comp[U.ch] : U.ch;
  uint32_t stream = (comp << 16) | (holo ? 0u : 2u);
  const int32_t gid = hp >= 0 ? H.gid : -1;
  if (stage == STAGE_PREFIX) {
    if (gid < 0) {
      sig_add(sig, 0xFFFFFFFFu);
      finish(B, U, J, st, K_ESCAPE_PREFIX, b, 0.f, sig, false);
      return;
    }
    b += 1;
    if (b == 1 && (J.debug & 1u)) B.s_first[st.slot] = gid;
    sig_add(sig, (uint32_t)gid + 1u);
    if (b > J.max_bounces) { finish(B, U, J, st, K_MAXB_PREFIX, b, 0.f, sig, false); return; }
    D3 o = st.o, d = st.d;
    double ell = st.ell;
    float ncur = st.wt;
    bool tri = gid >= (int32_t)S.n_sph;
    const MaterialDev &m = M[H.mat];
    bool delta = m.type == HPT_MIRROR || m.type == HPT_DIELECTRIC;
    double t64;
    const double4 pl = make_double4(H.g[0], H.g[1], H.g[2], H.g[3]);  // plane, or centre and radius
    if (J.phase_mode == HPT_PHASE_FP32) {
      t64 = (double)t;
      ell = (double)((float)ell + ncur * t);
    } else {
      t64 = tri ? tri_t64(pl, o, d) : sph_t64(pl, o, d, kTminD);
      ell += (double)ncur * t64;
    }
    D3 x = o + t64 * d;
    if (J.phase_mode == HPT_PHASE_FP32) x = to_d(to_f(o) + t * to_f(d));
    if (delta) {
      U4 w = philox(st.ka, st.kb, b << 8, stream, (uint32_t)J.seed, (uint32_t)(J.seed >> 32));
      D3 ng;
      if (tri) ng = D3{pl.x, pl.y, pl.z};
      else ng = (1.0 / pl.w) * (x - D3{pl.x, pl.y, pl.z});
      double dn = dot(d, ng);
      D3 nf = dn < 0 ? ng : (-1.0) * ng;
      double wgt = 1.0;
      uint32_t ev;
      if (m.type == HPT_MIRROR) {
        d = reflect(d, nf); ev = EV_MIRROR;
      } else {
        bool entering = dn < 0;
        double eta_i = entering ? 1.0 : (double)m.ior, eta_t = entering ? (double)m.ior : 1.0;
        double cos_i = fabs(dn), cos_t;
        double F = fresnel64(cos_i, eta_i, eta_t, cos_t);
        if (ud(w.x) < F) {
          d = reflect(d, nf); ev = EV_DIEL_REFL;
        } else {
          double et = eta_i / eta_t;
          d = normalize(et * d + (et * cos_i - cos_t) * nf);
          wgt = et * et; ev = EV_DIEL_REFR;
          ncur = (float)eta_t;
        }
      }
      if (J.phase_mode == HPT_PHASE_FP32) d = to_d(normalize(to_f(d)));
      sig_add(sig, ev);
      st.bpre *= (float)wgt;
      st.o = x;
      st.d = d;
      st.ell = ell;
      st.wt = ncur;
      st.sig = sig;
      st.meta = STAGE_PREFIX | (b << 1);
      stage_put(G, st, to_f(x), to_f(d), tri ? gid : -1, e);
      return;
    }
    // first non-delta hit: the real image point P
    sig_add(sig, EV_IMAGE_POINT);
    image_point(B, Q, U, J, st, ell, b);
    tail_interaction<EXT>(B, Q, G, U, J, S, M, st, to_f(x), to_f(d), H, b, b, comp, stream, 1.0f, 0.0f, sig, t,
                          St, e);
    return;
  }
  // incoherent tail (or cache path)
  float beta = st.beta, L = st.L;
  float4 r0 = Q.ray[2 * i], r1 = Q.ray[2 * i + 1];
  if (gid < 0) {
    L += beta * S.env[comp];
    sig_add(sig, 0xFFFFFFFEu);
    finish(B, U, J, st, K_ENV, b, L, sig, holo);
    return;
  }
  b += 1;
  sig_add(sig, (uint32_t)gid + 1u);
  F3 d_in = f3(r1.x, r1.y, r1.z);
  F3 x = f3(r0.x, r0.y, r0.z) + t * d_in;
  tail_interaction<EXT>(B, Q, G, U, J, S, M, st, x, d_in, H, b, bP, comp, stream, beta, L, sig, t, St, e);
}

// EXT: batches that use next-event estimation or principled materials (the
// base kernel leaves both out to keep its registers). Shading then may run
// occlusion queries: the traversal stack takes kStackLds entries per lane in
// LDS and the lane's column of the traversal spill, so the grid is capped at
// the spill's columns and walks the queue with a plain grid stride.
// UNI: a batch of one job whose scene has at most kLdsMats materials and
// which has at most kLdsUnits units; its job, scene, material and unit
// descriptors are read from LDS.
template <bool FIRST, bool EXT, bool UNI>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(EXT ? 2 : 3))) k_shade(BatchDev B, int q, uint32_t pass) {
  // FIRST: queue 0 as ray generation wrote it (dense); else a compacted
  // queue, read through its index list
  __shared__ StageLds G;
  __shared__ int32_t nee_stack[EXT ? kStackLds * kBlock : 1];
  __shared__ JobDev lds_job[1];
  __shared__ SceneDev lds_scene[1];
  __shared__ MaterialDev lds_mats[UNI ? kLdsMats : 1];
  __shared__ UnitDev lds_units[UNI ? kLdsUnits : 1];
  __shared__ uint32_t wave_cnt[kBlock / 64], wave_base[kBlock / 64 + 1];
  uint32_t n = B.counters[q];
  int qo = q ^ 1;
  if (blockIdx.x == 0 && threadIdx.x < kClaimClasses)  // traversal claims of queue q
    B.claims[((uint32_t)q * kClaimClasses + threadIdx.x) * kClaimStride] = 0;
  // The queue is cut into chunks of blockDim entries. Neighbouring entries
  // touch the same slot windows, so each XCD (the hardware deals workgroups
  // to the 8 XCDs in turn; the grid is a multiple of 8) takes one contiguous
  // eighth of the chunks, which its workgroups walk with a stride of their
  // number; the extended kernel walks all chunks with a plain grid stride.
  const uint32_t nb8 = ((n + blockDim.x - 1) / blockDim.x + 7u) & ~7u;
  const uint32_t b = blockIdx.x, per = nb8 / 8u;
  const uint32_t c0 = EXT ? b : (b % 8u) * per + b / 8u;
  const uint32_t cstep = EXT ? gridDim.x : gridDim.x / 8u;
  const uint32_t cend = EXT ? nb8 : (b % 8u + 1u) * per;
  if (c0 >= cend || c0 * blockDim.x >= n) return;  // no entries for this workgroup
  const Stack St{(LdsI32)(nee_stack + (EXT ? threadIdx.x : 0u)), kBlock,
                 (GlbI32)(B.stack_spill + blockIdx.x * blockDim.x + threadIdx.x), B.spill_threads, nullptr, 0u};
  if (UNI) {
    const uint32_t t = threadIdx.x;
    const uint32_t *jsrc = (const uint32_t *)B.job_uniform, *ssrc = (const uint32_t *)B.scene_uniform;
    for (uint32_t k = t; k < sizeof(JobDev) / 4; k += blockDim.x) ((uint32_t *)lds_job)[k] = jsrc[k];
    for (uint32_t k = t; k < sizeof(SceneDev) / 4; k += blockDim.x) ((uint32_t *)lds_scene)[k] = ssrc[k];
    const uint32_t nm = B.scene_uniform->n_mat;
    const uint32_t *msrc = (const uint32_t *)B.scene_uniform->mats;
    for (uint32_t k = t; k < nm * (uint32_t)(sizeof(MaterialDev) / 4); k += blockDim.x)
      ((uint32_t *)lds_mats)[k] = msrc[k];
    const uint32_t *usrc = (const uint32_t *)B.units;
    for (uint32_t k = t; k < B.n_units * (uint32_t)(sizeof(UnitDev) / 4); k += blockDim.x)
      ((uint32_t *)lds_units)[k] = usrc[k];
    __syncthreads();
  }
  for (uint32_t c = c0; c < cend && c * blockDim.x < n; c += cstep) {
    const uint32_t v = c * blockDim.x + threadIdx.x;  // v-th ray of the queue
    const bool live = v < n;
    Emit e;
    e.on = false;
    e.sig = false;
    if (live) {
      const uint32_t i = FIRST ? v : B.Q[q].idx[v];
      // the hit record is requested first: it is the longest chain
      // (entry -> primitive -> record); the rest of the state is loaded
      // while it is in flight
      const RayQueue &Qc = B.Q[q];
      const int32_t hp = Qc.prim[i];
      const uint32_t unit = Qc.unit[i];
      const float t = Qc.t[i];
      const UnitDev &U = UNI ? lds_units[unit] : B.units[unit];
      const JobDev &J = UNI ? lds_job[0] : *U.job;
      const SceneDev &S = UNI ? lds_scene[0] : *J.scene;
      const MaterialDev *M = UNI ? lds_mats : S.mats;
      HitRec H;
      if (hp >= 0) H = glb(S.hits)[hp];
      RayState st;
      st.unit = unit;
      e.sig = (J.debug & 5u) != 0;
      if (FIRST) load_first(Qc, i, st, U, J);
      else load_state<EXT>(Qc, i, st, e.sig, U, J, pass);
      shade_one<EXT>(B, q, i, st, G, U, J, S, M, t, hp, H, &St, e);
    }
    // compaction within the chunk: the continuing rays of chunk c take
    // entries [256 c, 256 c + count) of the next queue in lane order (wave
    // counts from ballots, their prefix in LDS), and the count is recorded
    // for the scan that orders the chunks; no atomic leaves the workgroup
    unsigned long long m = __ballot(e.on);
    const uint32_t lane = __lane_id(), wv = threadIdx.x / 64u;
    if (lane == 0) wave_cnt[wv] = (uint32_t)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t tot = 0;
      for (uint32_t k = 0; k < kBlock / 64; ++k) { wave_base[k] = tot; tot += wave_cnt[k]; }
      B.Q[qo].cnt[c] = tot;
    }
    __syncthreads();
    const uint32_t before = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
    if (e.on) stage_store<EXT>(G, B.Q[qo], c * kBlock + wave_base[wv] + before, e.sig);
  }
}

// Ordering of queue qo after the shading pass over the n rays of queue q
// (ceil(n / 256) chunks with a count each). k_scan: each workgroup takes a
// tile of kScanTile consecutive chunk counts, writes their exclusive prefix
// sums within the tile to off and the tile's total to tile_sum. k_index:
// the entries of chunk c are idx[base(c) + off[c] + k] = 256 c + k, k <
// cnt[c], with base(c) the sum of the totals of the tiles before c's (at
// most 64 tiles: one wave adds them); it also records qo's ray count.
constexpr uint32_t kScanPer = 16, kScanTile = kBlock * kScanPer;
__global__ void __launch_bounds__(kBlock) k_scan(BatchDev B, int q) {
  __shared__ uint32_t wsum[kBlock / 64];
  const int qo = q ^ 1;
  const uint32_t nc = (B.counters[q] + kBlock - 1) / kBlock;
  const uint32_t c0 = blockIdx.x * kScanTile + threadIdx.x * kScanPer;
  if (blockIdx.x * kScanTile >= nc) return;
  const auto cnt = glb(B.Q[qo].cnt);
  const auto off = glb(B.Q[qo].off);
  const uint32_t lane = __lane_id(), wv = threadIdx.x / 64u;
  uint32_t v[kScanPer], sum = 0;
#pragma unroll
  for (uint32_t j = 0; j < kScanPer; ++j) {
    v[j] = c0 + j < nc ? cnt[c0 + j] : 0u;
    sum += v[j];
  }
  uint32_t inc = sum;  // inclusive scan of the thread sums: in the wave, then over the waves
  for (uint32_t o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  uint32_t before = inc - sum;
  for (uint32_t k = 0; k < wv; ++k) before += wsum[k];
#pragma unroll
  for (uint32_t j = 0; j < kScanPer; ++j) {
    if (c0 + j < nc) off[c0 + j] = before;
    before += v[j];
  }
  if (threadIdx.x == kBlock - 1) B.Q[qo].tile_sum[blockIdx.x] = before;
}

__global__ void __launch_bounds__(kBlock) k_index(BatchDev B, int q) {
  const int qo = q ^ 1;
  const uint32_t nc = (B.counters[q] + kBlock - 1) / kBlock;
  const uint32_t n_tiles = (nc + kScanTile - 1) / kScanTile;
  const auto cnt = glb(B.Q[qo].cnt);
  const auto off = glb(B.Q[qo].off);
  const auto idx = glb(B.Q[qo].idx);
  const auto ts = glb(B.Q[qo].tile_sum);
  const uint32_t lane = __lane_id();
  if (blockIdx.x == 0 && threadIdx.x < 64) {  // the queue's ray count
    uint32_t t = lane < n_tiles ? ts[lane] : 0u;
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
    if (lane == 0) B.counters[qo] = t;
  }
  for (uint32_t c = xcd_block(); c < nc; c += gridDim.x) {
    const uint32_t tile = c / kScanTile;
    uint32_t base = lane < tile ? ts[lane] : 0u;   // every wave sums the earlier tiles
    for (int o = 32; o > 0; o >>= 1) base += __shfl_xor(base, o);
    const uint32_t k = threadIdx.x;
    if (k < cnt[c]) idx[base + off[c] + k] = c * kBlock + k;
  }
}

// ------------------------------------------------------------------ accumulate
// s8-s9 and Path Reuse. A group of ceil(T/2) consecutive lanes owns one
// pixel of a unit; lane t of the group owns frames 2t and 2t + 1 (the second
// when T > 2t + 1). The group walks the unit's samples in order; for each
// path it forms A W exp(i k r) / spp from the amplitude and the phasor the
// shading stored (the same value in every lane) and multiplies it by the
// unit phasors of its two frames at Q. The T frames of a texel are
// contiguous, so a lane reads its two frames of a table corner with one
// 16-byte load (two 8-byte loads when T is odd, where the pairs are not
// 16-byte aligned): what the gathers cost is their number of load
// instructions, not their bytes. Partial sums are added to the field at the
// end.
constexpr uint32_t kAccBatch = 4;  // paths whose loads are in flight together

// Bilinear weights of the corners (i0, j0), (i1, j0), (i0, j1), (i1, j1) at
// offsets (x, y).
struct BiW { double w00, w10, w01, w11; };

__device__ __forceinline__ BiW bilinear_weights(double x, double y) {
  return {(1.0 - x) * (1.0 - y), x * (1.0 - y), (1.0 - x) * y, x * y};
}

// 1 / sqrt(m2) for m2 > 0 from the hardware FP32 reciprocal square root
// (1 ulp; the result only scales the phasor, whose argument comes from the
// FP64 sums). Below the normal FP32 range m2 is first scaled by an even
// power of two into [0.5, 2).
__device__ __forceinline__ double inv_norm(double m2) {
  double inv = (double)__builtin_amdgcn_rsqf((float)m2);
  if (m2 < 1e-37 && m2 > 0.0) {  // rare: below the normal FP32 range
    const int h = ilogb(m2) / 2;  // m2 = m' 2^(2h), m' in [0.5, 4)
    inv = (double)__builtin_amdgcn_rsqf((float)ldexp(m2, -2 * h)) * ldexp(1.0, -h);
  }
  return inv;
}

// Unit phasor of the interpolated table value at weights W: in FP64 on the
// stored values (the phase is ill-conditioned where the interpolated value
// is small), normalised through FP32 (which only scales it); FP32
// throughout in the FP32 comparison mode. 1 where the value vanishes.
template <class R>
__device__ __forceinline__ void corner_phasor(bool f32_lookup, const BiW &W, float ar, float ai, float br,
                                              float bi, float cr, float ci, float dr, float di, R &pr, R &pi) {
  if (!f32_lookup) {
    const double zr = W.w00 * ar + W.w10 * br + W.w01 * cr + W.w11 * dr;
    const double zi = W.w00 * ai + W.w10 * bi + W.w01 * ci + W.w11 * di;
    const double m2 = zr * zr + zi * zi;
    const double inv = inv_norm(m2);  // inf for m2 = 0, not used then
    const bool nz = m2 > 0.0;
    pr = nz ? (R)(zr * inv) : (R)1;
    pi = nz ? (R)(zi * inv) : (R)0;
  } else {
    const float w00 = (float)W.w00, w10 = (float)W.w10, w01 = (float)W.w01, w11 = (float)W.w11;
    const float zr = w00 * ar + w10 * br + w01 * cr + w11 * dr;
    const float zi = w00 * ai + w10 * bi + w01 * ci + w11 * di;
    const float m2 = zr * zr + zi * zi;
    const float inv = m2 > 0.f ? rsqrtf(m2) : 0.f;
    pr = m2 > 0.f ? (R)(zr * inv) : (R)1;
    pi = (R)(zi * inv);
  }
}

template <bool F64>
__global__ void __launch_bounds__(kBlock) k_accumulate(BatchDev B, uint32_t lane0, uint32_t lane_end) {
  uint32_t idx = lane0 + xcd_block() * blockDim.x + threadIdx.x;
  if (idx >= lane_end) return;
  uint32_t u = find_unit(B.units, B.n_units, idx, true);
  const UnitDev U = B.units[u];
  if (U.kind != UNIT_HOLO) return;
  const JobDev &J = *U.job;
  if (F64 != (J.phase_mode == HPT_PHASE_FP64)) return;
  const uint32_t T = J.T, G = frame_group(T);
  const uint32_t local = idx - U.acc_base;
  const uint32_t p_local = local / G, t = local - p_local * G;
  const uint32_t f0 = 2 * t;                 // this lane's frames: f0 and, if two, f0 + 1
  const bool two = f0 + 1 < T;
  const bool pairs = (T & 1u) == 0;          // every (texel, f0) pair is 16-byte aligned
  uint32_t cx, cy;
  crop_xy(J, U.p_lo + p_local, cx, cy);
  using R = typename std::conditional<F64, double, float>::type;
  const uint32_t gw = J.grf_w, gh = J.grf_h;
  const auto G2 = glb(J.grf);
  const auto G4 = glb(reinterpret_cast<const float4 *>(J.grf));
  const size_t plane = (size_t)J.crop_h * J.crop_w;
  R ar0 = 0, ai0 = 0, ar1 = 0, ai1 = 0;
  unsigned long long sigsum = 0;
  const bool dbg_c = (J.debug & 2u) != 0, dbg_s = (J.debug & 4u) != 0 && t == 0;
  const bool rp = J.random_phase != 0;
  const bool f32_lookup = J.phase_mode == HPT_PHASE_FP32;  // the FP32 comparison mode looks up in FP32
  const uint32_t n = U.s_n, slot0 = U.slot_base + p_local * n;
  // frames f0, f0 + 1 at table element e (texel x T + f0, below 2^30 for
  // grids up to 4096^2 and T <= 64): one 16-byte load, or two 8-byte ones
  auto corner = [&](uint32_t e) -> float4 {
    if (pairs) return G4[e >> 1];
    const float2 a = G2[e];
    float2 b = make_float2(0.f, 0.f);
    if (two) b = G2[e + 1];
    return make_float4(a.x, a.y, b.x, b.y);
  };
  const uint32_t rowT = gw * T;  // elements per table row
  // Paths are taken kAccBatch at a time: the records of all of them are
  // requested, then the table corners of all of them, before the first is
  // used, so a wave has several gathers in flight instead of two dependent
  // round trips per path. The sum still runs in sample order.
  for (uint32_t k0 = 0; k0 < n; k0 += kAccBatch) {
    uint32_t tex[kAccBatch];
    float amp[kAccBatch];
    double fx[kAccBatch], fy[kAccBatch];
    R csr[kAccBatch], csi[kAccBatch];
    float4 qa[kAccBatch], qb[kAccBatch], qc[kAccBatch], qd[kAccBatch];
#pragma unroll
    for (uint32_t u = 0; u < kAccBatch; ++u) {
      const bool v = k0 + u < n;
      const uint32_t slot = slot0 + k0 + u;
      PathRes pr{};
      if (v) pr = B.res[slot];
      amp[u] = pr.amp;
      if (F64) {
        const double2 cs = v ? B.r_cs64[slot] : make_double2(0.0, 0.0);
        csr[u] = (R)cs.x; csi[u] = (R)cs.y;
      } else {
        csr[u] = (R)pr.cs.x; csi[u] = (R)pr.cs.y;
      }
      tex[u] = rp ? pr.tex : 0u;
      fx[u] = rp ? pr.fx : 0.0;
      fy[u] = rp ? pr.fy : 0.0;
    }
#pragma unroll
    for (uint32_t u = 0; u < kAccBatch; ++u) {
      if (rp && amp[u] != 0.f) {  // the texel is written only for paths with an image point
        // corners (i0, j0), (i0 + 1, j0), (i0, j0 + 1), (i0 + 1, j0 + 1),
        // the +1 wrapping to 0 on the periodic grid: 32-bit element offsets,
        // the steps to the next column and row as (modular) differences
        const uint32_t i0 = tex[u] & 0xFFFFu, j0 = tex[u] >> 16;
        const uint32_t e00 = j0 * rowT + i0 * T + f0;
        const uint32_t di = i0 + 1 == gw ? 0u - i0 * T : T;
        const uint32_t dj = j0 + 1 == gh ? 0u - j0 * rowT : rowT;
        qa[u] = corner(e00); qb[u] = corner(e00 + di);
        qc[u] = corner(e00 + dj); qd[u] = corner(e00 + di + dj);
      }
    }
#pragma unroll
    for (uint32_t u = 0; u < kAccBatch; ++u) {
      const uint32_t s = k0 + u;
      if (s >= n) break;
      if (dbg_s) sigsum += B.s_sig[slot0 + s];
      R c0r = 0, c0i = 0, c1r = 0, c1i = 0;
      if (amp[u] != 0.f) {
        R br, bi;
        if (F64) {
          br = (R)((double)amp[u] * csr[u]); bi = (R)((double)amp[u] * csi[u]);
        } else {
          br = (R)(amp[u] * csr[u]); bi = (R)(amp[u] * csi[u]);
        }
        if (rp) {
          R pr, pi;
          const BiW W = bilinear_weights(fx[u], fy[u]);
          corner_phasor<R>(f32_lookup, W, qa[u].x, qa[u].y, qb[u].x, qb[u].y, qc[u].x, qc[u].y,
                           qd[u].x, qd[u].y, pr, pi);
          c0r = br * pr - bi * pi; c0i = br * pi + bi * pr;
          if (two) {
            corner_phasor<R>(f32_lookup, W, qa[u].z, qa[u].w, qb[u].z, qb[u].w, qc[u].z, qc[u].w,
                             qd[u].z, qd[u].w, pr, pi);
            c1r = br * pr - bi * pi; c1i = br * pi + bi * pr;
          }
        } else {
          c0r = br; c0i = bi;
          c1r = br; c1i = bi;
        }
        ar0 += c0r; ai0 += c0i;
        ar1 += c1r; ai1 += c1i;
      }
      if (dbg_c) {
        const size_t ci = rec_index(J, U, p_local, s) * T + f0;
        J.contrib[ci] = make_float2((float)c0r, (float)c0i);
        if (two) J.contrib[ci + 1] = make_float2((float)c1r, (float)c1i);
      }
    }
  }
  const auto F = glb(J.field) + ((size_t)U.ch * T + f0) * plane + (size_t)cy * J.crop_w + cx;
  float2 v = F[0];
  v.x += (float)ar0; v.y += (float)ai0;
  F[0] = v;
  if (two) {
    v = F[plane];
    v.x += (float)ar1; v.y += (float)ai1;
    F[plane] = v;
  }
  if (dbg_s) J.sigsum[(size_t)U.ch * plane + (size_t)cy * J.crop_w + cx] += sigsum;
}

// ------------------------------------------------------------------ point emitters
// Closest-hit-free occlusion query: whether any primitive lies on the ray
// (o, d) at a distance in (kTmin, tmax). Plain stack traversal with the
// whole stack (kStackMax entries per lane) in LDS, so that it needs no
// global spill; `st` is this lane's column (stride kPtsBlock).
constexpr int kPtsBlock = 64;
__device__ bool segment_blocked(const SceneDev &S, F3 o, F3 d, float tmax, int32_t *st) {
  if (S.n_nodes == 0) return false;
  const RayPre r = ray_pre(o, d);
  const GF4 N = as_global(S.nodes), P = as_global(S.prims);
  int32_t node = 0;
  int sp = 0;
  for (;;) {
    if (node >= 0) {
      const float4 a = ld4(N + 4 * node), b = ld4(N + 4 * node + 1), c = ld4(N + 4 * node + 2),
                   l4 = ld4(N + 4 * node + 3);
      float t0, t1;
      bool h0, h1;
      box2(r, a, b, c, kTmin, tmax, t0, t1, h0, h1);
      const int32_t c0 = __float_as_int(l4.x), c1 = __float_as_int(l4.y);
      if (h0 && h1) {
        st[sp * kPtsBlock] = t0 <= t1 ? c1 : c0;
        ++sp;
        node = t0 <= t1 ? c0 : c1;
        continue;
      }
      if (h0 || h1) { node = h0 ? c0 : c1; continue; }
    } else {
      const uint32_t v = (uint32_t)(~node), first = v >> 3, cnt = (v & 7u) + 1u;
      for (uint32_t k = 0; k < cnt; ++k) {
        const GF4 p = P + 3 * (size_t)(first + k);
        const float4 p0 = ld4(p), p1 = ld4(p + 1);
        float t;
        const bool h = __float_as_int(p1.w) == 1
                           ? sph_hit(r, f3(p0.x, p0.y, p0.z), p1.x, kTmin, tmax, t)
                           : tri_hit(r, f3(p0.x, p0.y, p0.z), f3(p1.x, p1.y, p1.z),
                                     f3(ld4(p + 2).x, ld4(p + 2).y, ld4(p + 2).z), kTmin, tmax, t);
        if (h && t < tmax) return true;
      }
    }
    if (sp == 0) return false;
    node = st[--sp * kPtsBlock];
  }
}

// Unit phasor of frame t at hologram-space (qx, qy): bilinear interpolation
// of the random field (texel (i, j) on pixel centre (i, j), periodic) in
// FP64, then normalised (1 where it vanishes), as the accumulation does.
__device__ __forceinline__ float2 grf_unit(const JobDev &J, uint32_t t, double qx, double qy) {
  const double u = qx / J.pitch + 0.5 * (double)J.width - 0.5;
  const double v = qy / J.pitch + 0.5 * (double)J.height - 0.5;
  const double fu = floor(u), fv = floor(v);
  int64_t i0 = (int64_t)fu % (int64_t)J.grf_w, j0 = (int64_t)fv % (int64_t)J.grf_h;
  if (i0 < 0) i0 += J.grf_w;
  if (j0 < 0) j0 += J.grf_h;
  const uint32_t i1 = i0 + 1 == J.grf_w ? 0 : (uint32_t)i0 + 1, j1 = j0 + 1 == J.grf_h ? 0 : (uint32_t)j0 + 1;
  const auto G2 = glb(J.grf) + t;
  const size_t gw = J.grf_w, T = J.T;
  const float2 qa = G2[((size_t)j0 * gw + i0) * T], qb = G2[((size_t)j0 * gw + i1) * T],
               qc = G2[((size_t)j1 * gw + i0) * T], qd = G2[((size_t)j1 * gw + i1) * T];
  const double x = u - fu, y = v - fv;
  const double w00 = (1.0 - x) * (1.0 - y), w10 = x * (1.0 - y), w01 = (1.0 - x) * y, w11 = x * y;
  const double zr = w00 * qa.x + w10 * qb.x + w01 * qc.x + w11 * qd.x;
  const double zi = w00 * qa.y + w10 * qb.y + w01 * qc.y + w11 * qd.y;
  const double m2 = zr * zr + zi * zi;
  if (!(m2 > 0.0)) return make_float2(1.f, 0.f);
  const double inv = inv_norm(m2);  // also where m2 is below the FP32 range
  return make_float2((float)(zr * inv), (float)(zi * inv));
}

// Point emitters: pixel p of a unit that starts at sample 0 receives, for
// every emitter y in front of the plane inside its recordable cone and not
// occluded, a exp(i (k r + phi_t(Q))) / r in frame t, Q = T y, r = |Q - x_p|
// (Eq. 2 for a point source, obliquity 1). Grid: x over a unit's pixels,
// y over the batch's units. The cone test and r are FP64 in every mode; the
// phase is carried like a path's (FP64 reduction frac(r / lambda), sin/cos
// in FP64 for FP64 phase, FP32 otherwise; all FP32 in FP32 phase).
__global__ void __launch_bounds__(kPtsBlock) k_points(BatchDev B) {
  __shared__ int32_t stack[kStackMax * kPtsBlock];
  const UnitDev U = B.units[blockIdx.y];
  if (U.kind != UNIT_HOLO || U.s_lo != 0) return;
  const uint32_t pl = blockIdx.x * kPtsBlock + threadIdx.x;
  if (pl >= U.p_n) return;
  const JobDev &J = *U.job;
  const SceneDev &S = *J.scene;
  if (S.n_pts == 0) return;
  uint32_t cx, cy;
  crop_xy(J, U.p_lo + pl, cx, cy);
  const uint32_t px = J.crop_x0 + cx, py = J.crop_y0 + cy;
  const uint32_t comp = J.comp[U.ch];
  const D3 xp = {((double)px + 0.5 - 0.5 * (double)J.width) * J.pitch,
                 ((double)py + 0.5 - 0.5 * (double)J.height) * J.pitch, 0.0};
  const double *Ti = J.Ti, *M = J.Tm;
  const D3 O = {Ti[0] * xp.x + Ti[1] * xp.y + Ti[2] * xp.z + Ti[3], Ti[4] * xp.x + Ti[5] * xp.y + Ti[6] * xp.z + Ti[7],
                Ti[8] * xp.x + Ti[9] * xp.y + Ti[10] * xp.z + Ti[11]};
  const double s = J.s_cone[U.ch];
  const size_t plane = (size_t)J.crop_h * J.crop_w;
  const auto F = glb(J.field) + (size_t)U.ch * J.T * plane + (size_t)cy * J.crop_w + cx;
  const auto E = as_global(S.pts);
  for (uint32_t e = 0; e < S.n_pts; ++e) {
    const float4 pos = ld4(E + 2 * e), amp4 = ld4(E + 2 * e + 1);
    const float a = comp == 0 ? amp4.x : (comp == 1 ? amp4.y : amp4.z);
    if (a == 0.f) continue;
    const D3 y = {pos.x, pos.y, pos.z};
    const D3 Q = {M[0] * y.x + M[1] * y.y + M[2] * y.z + M[3], M[4] * y.x + M[5] * y.y + M[6] * y.z + M[7],
                  M[8] * y.x + M[9] * y.y + M[10] * y.z + M[11]};
    const D3 dq = Q - xp;
    const double r = sqrt(dot(dq, dq));
    if (!(dq.z > 0.0) || dq.x * dq.x + dq.y * dq.y > s * s * r * r) continue;
    const D3 seg = y - O;
    const double dist = sqrt(dot(seg, seg));
    if (segment_blocked(S, to_f(O), to_f((1.0 / dist) * seg), (float)dist, stack + threadIdx.x)) continue;
    double cr, ci;
    if (J.phase_mode == HPT_PHASE_FP32) {
      const float rf = (float)r, x = rf * J.inv_lambda_f[U.ch];
      float sn, cs;
      sincospif(2.0f * (x - floorf(x)), &sn, &cs);
      cr = (double)(a / rf * cs); ci = (double)(a / rf * sn);
    } else {
      const double x = r * J.inv_lambda[U.ch], rev = x - floor(x);
      if (J.phase_mode == HPT_PHASE_FP64) {
        double sn, cs;
        sincospi(2.0 * rev, &sn, &cs);
        cr = a / r * cs; ci = a / r * sn;
      } else {
        float sn, cs;
        sincospif(2.0f * (float)rev, &sn, &cs);
        const float ar = (float)(a / r);
        cr = (double)(ar * cs); ci = (double)(ar * sn);
      }
    }
    for (uint32_t t = 0; t < J.T; ++t) {
      double zr = cr, zi = ci;
      if (J.random_phase) {
        const float2 ph = grf_unit(J, t, Q.x, Q.y);
        zr = cr * ph.x - ci * ph.y;
        zi = cr * ph.y + ci * ph.x;
      }
      float2 v = F[(size_t)t * plane];
      v.x += (float)zr; v.y += (float)zi;
      F[(size_t)t * plane] = v;
    }
  }
}

// Mean radiance of each cache entry over its paths, rounded to binary16.
__global__ void __launch_bounds__(kBlock) k_cache_reduce(BatchDev B) {
  uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= B.n_acc) return;
  uint32_t u = find_unit(B.units, B.n_units, idx, true);
  const UnitDev U = B.units[u];
  if (U.kind != UNIT_CACHE) return;
  const JobDev &J = *U.job;
  uint32_t e_local = idx - U.acc_base;
  float sum = 0.f;
  for (uint32_t s = 0; s < U.s_n; ++s) sum += B.res[U.slot_base + e_local * U.s_n + s].amp;
  float mean = sum / (float)J.cache_spb;
  size_t n_entries = (size_t)J.cache_res * J.cache_res * J.cache_res * J.cache_bins * J.cache_bins;
  J.cache_out[(size_t)U.ch * n_entries + U.p_lo + e_local] = __half_as_ushort(__float2half_rn(mean));
}

// ------------------------------------------------------------------ Eq. 4 tables
// Spectrum: exp(i xi_t(jx, jy)) inside the passband (sx/gw)^2 + (sy/gh)^2 <= 1/4
// (exact integer test), 0 outside; xi = 2 pi u from Philox stream 3.
__global__ void k_grf_spectrum(double2 *spec, uint32_t gw, uint32_t gh, uint32_t T, uint64_t seed) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t n = (size_t)T * gh * gw;
  if (idx >= n) return;
  uint32_t jx = idx % gw, jy = (idx / gw) % gh, t = idx / ((size_t)gw * gh);
  int64_t sx = jx < (gw + 1) / 2 ? (int64_t)jx : (int64_t)jx - gw;
  int64_t sy = jy < (gh + 1) / 2 ? (int64_t)jy : (int64_t)jy - gh;
  bool in = 4 * (sx * sx * (int64_t)gh * gh + sy * sy * (int64_t)gw * gw) <= (int64_t)gw * gw * (int64_t)gh * gh;
  double2 v = make_double2(0.0, 0.0);
  if (in) {
    U4 w = philox(jx, jy, t, 3u, (uint32_t)seed, (uint32_t)(seed >> 32));
    double sn, cs;
    sincospi(2.0 * ud(w.x), &sn, &cs);
    v = make_double2(cs, sn);
  }
  spec[idx] = v;
}

// Inverse DFT along x of one spectrum row (t, jy): only passband bins.
__global__ void k_grf_rows(const double2 *spec, double2 *rows, uint32_t gw, uint32_t gh) {
  extern __shared__ double2 tw[];  // exp(2 pi i m / gw)
  uint32_t row = blockIdx.x;       // t * gh + jy
  for (uint32_t m = threadIdx.x; m < gw; m += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * (double)m / (double)gw, &sn, &cs);
    tw[m] = make_double2(cs, sn);
  }
  __syncthreads();
  uint32_t jy = row % gh;
  int64_t sy = jy < (gh + 1) / 2 ? (int64_t)jy : (int64_t)jy - gh;
  // passband half-width along x for this row
  int64_t lim2 = (int64_t)gw * gw * (int64_t)gh * gh - 4 * sy * sy * (int64_t)gw * gw;  // >= 4 sx^2 gh^2
  int64_t smax = 0;
  while (4 * (smax + 1) * (smax + 1) * (int64_t)gh * gh <= lim2 && smax + 1 <= (int64_t)gw / 2) ++smax;
  // signed bins [lo, hi]; an even grid's Nyquist bin is -gw/2 only
  int64_t lo = -(smax < (int64_t)gw / 2 ? smax : (int64_t)gw / 2);
  int64_t hi = smax < ((int64_t)gw - 1) / 2 ? smax : ((int64_t)gw - 1) / 2;
  const double2 *S = spec + (size_t)row * gw;
  for (uint32_t x = threadIdx.x; x < gw; x += blockDim.x) {
    double re = 0.0, im = 0.0;
    uint32_t jx = (uint32_t)(lo < 0 ? lo + gw : lo);
    uint32_t m = (uint32_t)(((uint64_t)jx * x) % gw);  // jx * x mod gw, then stepped
    for (int64_t sx = lo; sx <= hi; ++sx) {
      double2 a = S[jx];
      double2 w = tw[m];
      re += a.x * w.x - a.y * w.y;
      im += a.x * w.y + a.y * w.x;
      jx = jx + 1 == gw ? 0 : jx + 1;
      m += x;
      if (m >= gw) m -= gw;
    }
    rows[(size_t)row * gw + x] = make_double2(re, im);
  }
}

// Inverse DFT along y, scaling by 1/sqrt(#passband bins), written as
// complex64 into the table [gh][gw][T].
__global__ void k_grf_cols(const double2 *rows, float2 *table, uint32_t gw, uint32_t gh, uint32_t T,
                           double scale) {
  extern __shared__ double2 tw[];
  uint32_t x = blockIdx.x % gw, t = blockIdx.x / gw;
  for (uint32_t m = threadIdx.x; m < gh; m += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * (double)m / (double)gh, &sn, &cs);
    tw[m] = make_double2(cs, sn);
  }
  __syncthreads();
  const double2 *Rr = rows + (size_t)t * gh * gw + x;
  for (uint32_t y = threadIdx.x; y < gh; y += blockDim.x) {
    double re = 0.0, im = 0.0;
    uint32_t m = 0;
    for (uint32_t jy = 0; jy < gh; ++jy) {
      double2 a = Rr[(size_t)jy * gw];
      double2 w = tw[m];
      re += a.x * w.x - a.y * w.y;
      im += a.x * w.y + a.y * w.x;
      m += y;
      if (m >= gh) m -= gh;
    }
    table[((size_t)y * gw + x) * T + t] = make_float2((float)(re * scale), (float)(im * scale));
  }
}

// ------------------------------------------------------------------ host launchers
static inline uint32_t grid_for(uint64_t n) { return (uint32_t)((n + kBlock - 1) / kBlock); }
static inline uint32_t round8(uint32_t g) { return (g + 7u) & ~7u; }

hipError_t launch_raygen(const BatchDev &B, bool uni, hipStream_t st) {
  uint32_t g = (uint32_t)(((uint64_t)B.n_paths + kRaygenWindow - 1) / kRaygenWindow);
  if (uni)
    hipLaunchKernelGGL(k_raygen<true>, dim3(g), dim3(kRaygenBlock), 0, st, B);
  else
    hipLaunchKernelGGL(k_raygen<false>, dim3(g), dim3(kRaygenBlock), 0, st, B);
  return hipGetLastError();
}

uint32_t trace_grid(uint32_t n_paths) {
  // enough waves to fill every CU; waves beyond the resident ones find the
  // queue drained and exit
  uint64_t waves = ((uint64_t)n_paths + kTraceChunk - 1) / kTraceChunk;
  uint32_t g = (uint32_t)((waves * 64 + kBlock - 1) / kBlock);
  g = (g + kClaimClasses - 1) / kClaimClasses * kClaimClasses;  // every class has workgroups
  return g < kTraceGridMax ? g : kTraceGridMax;
}

uint32_t trace_block() { return kBlock; }

hipError_t launch_trace(const BatchDev &B, int q, bool dense, bool count, hipStream_t st) {
  uint32_t g = trace_grid(B.n_paths);
  if ((uint64_t)g * kBlock > B.spill_threads) return hipErrorInvalidValue;
  if (count) hipLaunchKernelGGL(k_trace<true>, dim3(g), dim3(kBlock), 0, st, B, q, dense ? 1 : 0);
  else hipLaunchKernelGGL(k_trace<false>, dim3(g), dim3(kBlock), 0, st, B, q, dense ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_compact(const BatchDev &B, int q, hipStream_t st) {
  const uint32_t max_chunks = (B.n_paths + kBlock - 1) / kBlock;
  const uint32_t tiles = (max_chunks + kScanTile - 1) / kScanTile;
  if (tiles > 64) return hipErrorInvalidValue;   // k_index sums the tile totals with one wave
  hipLaunchKernelGGL(k_scan, dim3(tiles), dim3(kBlock), 0, st, B, q);
  const uint32_t g = min(round8((B.n_paths + kBlock - 1) / kBlock), 4096u);
  hipLaunchKernelGGL(k_index, dim3(g), dim3(kBlock), 0, st, B, q);
  return hipGetLastError();
}

uint32_t shade_lds_mats() { return kLdsMats; }
uint32_t shade_lds_units() { return kLdsUnits; }

hipError_t launch_shade(const BatchDev &B, int q, uint32_t pass, bool ext, bool uni, hipStream_t st) {
  const bool first = pass == 0;
  const uint32_t g = min(round8(grid_for(B.n_paths)), kShadeGridMax);
  const uint32_t gn = ext ? min(g, B.spill_threads / (uint32_t)kBlock) : g;  // one spill column per lane
  auto k = ext ? (first ? (uni ? k_shade<true, true, true> : k_shade<true, true, false>)
                        : (uni ? k_shade<false, true, true> : k_shade<false, true, false>))
               : (first ? (uni ? k_shade<true, false, true> : k_shade<true, false, false>)
                        : (uni ? k_shade<false, false, true> : k_shade<false, false, false>));
  hipLaunchKernelGGL(k, dim3(gn), dim3(kBlock), 0, st, B, q, pass);
  return hipGetLastError();
}

// One launch per precision present in the batch.
hipError_t launch_accumulate(const BatchDev &B, bool has_f64, bool has_f32, uint32_t lane0, uint32_t lane_end,
                             hipStream_t st) {
  if (lane_end <= lane0) return hipSuccess;
  uint32_t g = round8(grid_for(lane_end - lane0));
  if (has_f32) hipLaunchKernelGGL(k_accumulate<false>, dim3(g), dim3(kBlock), 0, st, B, lane0, lane_end);
  if (has_f64) hipLaunchKernelGGL(k_accumulate<true>, dim3(g), dim3(kBlock), 0, st, B, lane0, lane_end);
  return hipGetLastError();
}

hipError_t launch_points(const BatchDev &B, uint32_t max_pn, hipStream_t st) {
  if (B.n_units == 0 || max_pn == 0) return hipSuccess;
  hipLaunchKernelGGL(k_points, dim3((max_pn + kPtsBlock - 1) / kPtsBlock, B.n_units), dim3(kPtsBlock), 0, st, B);
  return hipGetLastError();
}

hipError_t launch_cache_reduce(const BatchDev &B, hipStream_t st) {
  hipLaunchKernelGGL(k_cache_reduce, dim3(grid_for(B.n_acc)), dim3(kBlock), 0, st, B);
  return hipGetLastError();
}

hipError_t launch_grf(double2 *spec, double2 *rows, float2 *table, uint32_t gw, uint32_t gh, uint32_t T,
                      uint64_t seed, double scale, hipStream_t st) {
  size_t n = (size_t)T * gh * gw;
  hipLaunchKernelGGL(k_grf_spectrum, dim3(grid_for(n)), dim3(kBlock), 0, st, spec, gw, gh, T, seed);
  hipLaunchKernelGGL(k_grf_rows, dim3(T * gh), dim3(kBlock), gw * sizeof(double2), st, spec, rows, gw, gh);
  hipLaunchKernelGGL(k_grf_cols, dim3(T * gw), dim3(kBlock), gh * sizeof(double2), st, rows, table, gw, gh, T,
                     scale);
  return hipGetLastError();
}

}  // namespace hpt
