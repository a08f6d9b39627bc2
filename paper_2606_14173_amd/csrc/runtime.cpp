// Host runtime of the wave path tracer: context, resident scenes, radiance
// caches and random-phase tables, and a continuous-batching scheduler.
//
// A job is split, once and independently of other jobs, into units of
// (channel, pixel block, sample chunk). The scheduler thread admits queued
// jobs while their device memory fits the budget, packs units of all
// running jobs into batches of at most `capacity` paths, runs the kernel
// sequence of a batch on the context stream and retires units. Units of one
// (channel, pixel block) never share a batch and retire in sample order, so
// a job's field is bitwise the same whether it runs alone or among others.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/hpt.h"
#include "asm.hpp"
#include "encode.hpp"
#include "bvh_build.hpp"
#include "hpt_types.hpp"
#include "kernels.hpp"

using namespace hpt;
using Clock = std::chrono::steady_clock;

namespace {

thread_local std::string g_err;

hpt_status fail(hpt_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

constexpr uint32_t kMaxUnitsPerBatch = 4096;
// per path, in two sets: final signature, first hit, results; per queue
// entry (two queues): state (32 B), FP64 prefix ray (56 B), FP32 ray (32 B),
// hit (8 B), index list (4 B; chunk counts and offsets: 8 B per 256 entries)
#ifndef HPT_ACC_PARTS
#define HPT_ACC_PARTS 3
#endif
constexpr uint32_t kAccParts = HPT_ACC_PARTS;  // accumulation launches per batch
static_assert(kAccParts >= 1 && kAccParts <= 4, "part k starts beside the next batch's traversal k + 1");

constexpr size_t kBytesPerPath = 2 * (8 + 4 + 32 + 16) + 2 * (32 + 56 + 32 + 8 + 4 + 1);

struct Scene {
  uint64_t id = 0;
  std::vector<void *> bufs;
  size_t bytes = 0;
  SceneDev host{};
  SceneDev *dev = nullptr;
  hpt_scene_info info{};
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  uint16_t *cache = nullptr;
  size_t cache_bytes = 0;
  hpt_cache_desc cache_desc{};
  int users = 0;
  bool principled = false;   // some material is HPT_PRINCIPLED
};

struct Grf {
  uint32_t gw = 0, gh = 0, T = 0;
  uint64_t seed = 0;
  float2 *d = nullptr;
  size_t bytes = 0;
  int users = 0;
};

enum JobState { JS_QUEUED, JS_RUNNING, JS_DONE, JS_FAILED, JS_CANCELED };

struct Unit {
  uint32_t kind, ch, p_lo, p_n, s_lo, s_n, key;
};

struct Job {
  uint64_t id = 0;
  hpt_job_desc desc{};
  Scene *scene = nullptr;
  Grf *grf = nullptr;
  bool cache_build = false;
  bool ext = false;       // needs the extended shading kernel: next-event estimation or principled materials
  JobDev host{};
  JobDev *dev = nullptr;
  float2 *field = nullptr;
  bool own_field = false;
  size_t field_elems = 0;
  hpt_path_record *rec = nullptr;
  float2 *contrib = nullptr;
  unsigned long long *sigsum = nullptr;
  size_t n_rec = 0, n_contrib = 0, n_sig = 0;
  std::vector<Unit> units;
  size_t next = 0, done = 0;
  uint32_t in_flight = 0;     // units in the batch the GPU may still be running
  JobState state = JS_QUEUED;
  hpt_status status = HPT_OK;
  std::string err;
  bool cancel = false;
  hpt_status fail_status = HPT_OK;  // a batch holding its units failed; retired once none is in flight
  std::string fail_err;
  hipEvent_t ready = nullptr;  // recorded on the caller's stream at submit: the job's work waits for it
  size_t bytes = 0;       // device bytes it holds while admitted (not counting the table)
  size_t grf_bytes = 0;   // bytes of its random-phase table if it must be built
  Clock::time_point t_submit, t_start, t_end;
  bool started = false;
  hpt_job_stats stats{};
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

bool affine_inverse(const double *M, double *Ti) {
  double a = M[0], b = M[1], c = M[2], d = M[4], e = M[5], f = M[6], g = M[8], h = M[9], i = M[10];
  double c00 = e * i - f * h, c01 = f * g - d * i, c02 = d * h - e * g;
  double det = a * c00 + b * c01 + c * c02;
  if (!(std::fabs(det) > 1e-300) || !std::isfinite(det)) return false;
  double inv[9] = {c00, c * h - b * i, b * f - c * e,
                   c01, a * i - c * g, c * d - a * f,
                   c02, b * g - a * h, a * e - b * d};
  for (int k = 0; k < 9; ++k) inv[k] /= det;
  for (int r = 0; r < 3; ++r) {
    for (int k = 0; k < 3; ++k) Ti[4 * r + k] = inv[3 * r + k];
    Ti[4 * r + 3] = -(inv[3 * r] * M[3] + inv[3 * r + 1] * M[7] + inv[3 * r + 2] * M[11]);
  }
  return true;
}

// One unit of a job picked into a batch.
struct Picked { Job *job; size_t unit; };

}  // namespace

struct hpt_ctx {
  int device = 0;
  hipStream_t stream = nullptr, aux = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  uint64_t budget = 0, used = 0;
  uint32_t capacity = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  bool stop = false;
  uint64_t next_id = 1;
  std::map<uint64_t, std::unique_ptr<Scene>> scenes;
  std::map<uint64_t, std::unique_ptr<Job>> jobs;
  std::deque<Job *> queue;     // submitted, not yet admitted
  std::vector<Job *> running;  // admitted, units left
  std::vector<std::unique_ptr<Grf>> grfs;
  // batch buffers: queues, counters and stack spill shared by consecutive
  // batches (one stream runs their tracing in order); per-path results and
  // unit tables in two sets, so that batch k's accumulation (on its own
  // stream) overlaps batch k+1's tracing
  std::vector<void *> batch_bufs;
  uint64_t batch_bytes = 0;   // device bytes of batch_bufs
  BatchDev batch{};
  hipStream_t acc = nullptr;  // accumulation stream
  static constexpr int kEvents = 200;   // 2 per timed launch: ray generation, 3 per interaction, accumulation
  struct Slot {
    unsigned long long *s_sig = nullptr;
    int32_t *s_first = nullptr;
    PathRes *res = nullptr;
    double2 *r_cs64 = nullptr;
    UnitDev *d_units = nullptr, *h_units = nullptr;
    uint32_t *h_cnt = nullptr;            // pinned: the batch's counters after its last shading pass
    unsigned long long *h_work = nullptr; // pinned: node visits, primitive tests
    hipEvent_t ev0 = nullptr, ev_rg = nullptr, ev_shade = nullptr, ev_done = nullptr;
    BatchDev B{};               // the batch's device view (for its accumulation)
    bool has_f64 = false, has_f32 = false, has_ext = false;
    bool acc_pending = false;   // accumulation not (fully) enqueued yet
    uint32_t acc_parts = 0;     // parts of it enqueued
    hipEvent_t ev_sh[4] = {};   // after the batch's first shading passes
    hipEvent_t pev[kEvents] = {};
    int ne = 0;
    int seg_kind[kEvents / 2] = {};
    // the batch in this slot
    std::vector<Picked> P;
    uint32_t profile = 0, paths = 0;
    bool has_holo = false, has_cache = false;
    uint32_t pts_max_pn = 0;    // largest pixel count of a unit with point-emitter terms (0: none)
    hpt_status launch_status = HPT_OK;
    std::string err;
  } slots[2];
  uint64_t batches = 0, jobs_done = 0;
  uint32_t fail_batches = 0;  // failure injection (hpt_debug_fail_batches)
  float2 *na_scratch = nullptr;  // this device's static scratch of the allocation-free propagation
  // profiling (guarded by mu; events used by the scheduler thread only)
  uint32_t profile = 0;
  hpt_kernel_time ktime[HPT_K_KINDS] = {};
  uint64_t node_visits = 0, prim_tests = 0;

  hipError_t alloc(void **p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes ? bytes : 16);
    if (e == hipSuccess) used += bytes;
    return e;
  }
  void release(void *p, size_t bytes) {
    if (p) { (void)hipFree(p); used -= std::min<uint64_t>(used, bytes); }
  }
};

namespace {

// ---------------------------------------------------------------- random tables
Grf *find_grf(hpt_ctx *C, uint32_t gw, uint32_t gh, uint32_t T, uint64_t seed) {
  for (auto &g : C->grfs)
    if (g->gw == gw && g->gh == gh && g->T == T && g->seed == seed) return g.get();
  return nullptr;
}

size_t grf_table_bytes(uint32_t gw, uint32_t gh, uint32_t T) { return (size_t)gw * gh * T * sizeof(float2); }
size_t grf_temp_bytes(uint32_t gw, uint32_t gh, uint32_t T) { return 2 * (size_t)gw * gh * T * sizeof(double2); }

uint64_t passband_bins(uint32_t gw, uint32_t gh) {
  uint64_t n = 0;
  for (uint32_t jy = 0; jy < gh; ++jy) {
    int64_t sy = jy < (gh + 1) / 2 ? (int64_t)jy : (int64_t)jy - gh;
    for (uint32_t jx = 0; jx < gw; ++jx) {
      int64_t sx = jx < (gw + 1) / 2 ? (int64_t)jx : (int64_t)jx - gw;
      if (4 * (sx * sx * (int64_t)gh * gh + sy * sy * (int64_t)gw * gw) <= (int64_t)gw * gw * (int64_t)gh * gh) ++n;
    }
  }
  return n;
}

// Drop tables no running job uses until `need` more bytes fit the budget.
void evict_grfs(hpt_ctx *C, size_t need) {
  for (size_t k = 0; k < C->grfs.size() && C->used + need > C->budget;) {
    if (C->grfs[k]->users == 0) {
      C->release(C->grfs[k]->d, C->grfs[k]->bytes);
      C->grfs.erase(C->grfs.begin() + k);
    } else {
      ++k;
    }
  }
}

// Build a table (caller holds the lock); synchronous on `st`.
hpt_status build_grf(hpt_ctx *C, uint32_t gw, uint32_t gh, uint32_t T, uint64_t seed, hipStream_t st,
                     Grf **out) {
  if (Grf *g = find_grf(C, gw, gh, T, seed)) { *out = g; return HPT_OK; }
  size_t tb = grf_table_bytes(gw, gh, T), tmp = grf_temp_bytes(gw, gh, T);
  evict_grfs(C, tb + tmp);
  if (C->used + tb + tmp > C->budget) return fail(HPT_EBUDGET, "random-phase table does not fit the budget");
  auto g = std::make_unique<Grf>();
  g->gw = gw; g->gh = gh; g->T = T; g->seed = seed; g->bytes = tb;
  void *spec = nullptr, *rows = nullptr;
  if (C->alloc((void **)&g->d, tb) != hipSuccess) return fail(HPT_ENOMEM, "table allocation failed");
  if (C->alloc(&spec, tmp / 2) != hipSuccess || C->alloc(&rows, tmp / 2) != hipSuccess) {
    C->release(spec, tmp / 2);
    C->release(g->d, tb);
    return fail(HPT_ENOMEM, "table scratch allocation failed");
  }
  double scale = 1.0 / std::sqrt((double)passband_bins(gw, gh));
  hipError_t e = launch_grf((double2 *)spec, (double2 *)rows, g->d, gw, gh, T, seed, scale, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  C->release(spec, tmp / 2);
  C->release(rows, tmp / 2);
  if (e != hipSuccess) {
    C->release(g->d, tb);
    return fail(HPT_EDEVICE, std::string("table build failed: ") + hipGetErrorString(e));
  }
  *out = g.get();
  C->grfs.push_back(std::move(g));
  return HPT_OK;
}

// ---------------------------------------------------------------- jobs
// Units of about min(2^20, batch capacity) paths: up to 256 samples of a
// block of pixels. Deep sample chunks keep a batch's pixels (consecutive
// blocks in the 8x8-tile order) in a band of rows, so that the image points
// its paths look up in the random-field table stay within a band of the table
// (the cone footprint around those rows) that the L2 and the memory-side
// cache can hold. A unit never exceeds the capacity (>= 2^16 >= 64 x 256), so
// every unit fits a batch.
void split_units(Job *J, uint32_t capacity) {
  uint32_t P = J->host.crop_w * J->host.crop_h, S = J->host.n_s;
  uint32_t Su = std::min<uint32_t>(S, 256u);
  uint32_t target = std::min<uint32_t>(1u << 20, capacity);
  uint32_t Pu = std::min<uint32_t>(P, std::max<uint32_t>(64u, target / Su));
  uint32_t nblk = (P + Pu - 1) / Pu;
  for (uint32_t s0 = 0; s0 < S; s0 += Su)
    for (uint32_t c = 0; c < J->host.n_ch; ++c)
      for (uint32_t r = 0; r < nblk; ++r) {
        Unit u;
        u.kind = UNIT_HOLO; u.ch = c;
        u.p_lo = r * Pu; u.p_n = std::min(Pu, P - r * Pu);
        u.s_lo = J->host.spp_lo + s0; u.s_n = std::min(Su, S - s0);
        u.key = c * nblk + r;
        J->units.push_back(u);
      }
}

void split_cache_units(Job *J, uint32_t capacity) {
  uint32_t E = J->host.cache_res * J->host.cache_res * J->host.cache_res * J->host.cache_bins *
               J->host.cache_bins;
  uint32_t spb = J->host.cache_spb;
  uint32_t Eu = std::max<uint32_t>(1u, std::min<uint32_t>(E, std::min<uint32_t>(1u << 20, capacity) / spb));
  uint32_t nblk = (E + Eu - 1) / Eu;
  for (uint32_t c = 0; c < 3; ++c)
    for (uint32_t r = 0; r < nblk; ++r) {
      Unit u;
      u.kind = UNIT_CACHE; u.ch = c;
      u.p_lo = r * Eu; u.p_n = std::min(Eu, E - r * Eu);
      u.s_lo = 0; u.s_n = spb;
      u.key = c * nblk + r;
      J->units.push_back(u);
    }
}

void free_job_buffers(hpt_ctx *C, Job *J) {
  if (J->own_field) C->release(J->field, J->field_elems * sizeof(float2));
  C->release(J->rec, J->n_rec * sizeof(hpt_path_record));
  C->release(J->contrib, J->n_contrib * sizeof(float2));
  C->release(J->sigsum, J->n_sig * sizeof(unsigned long long));
  C->release(J->dev, sizeof(JobDev));
  J->field = nullptr; J->rec = nullptr; J->contrib = nullptr; J->sigsum = nullptr; J->dev = nullptr;
  if (J->ready) { (void)hipEventDestroy(J->ready); J->ready = nullptr; }
}

void retire(hpt_ctx *C, Job *J, JobState st, hpt_status status, const std::string &err) {
  J->state = st;
  J->status = status;
  J->err = err;
  J->t_end = Clock::now();
  if (!J->started) J->t_start = J->t_end;
  J->stats.queued_ms = ms_between(J->t_submit, J->t_start);
  J->stats.run_ms = ms_between(J->t_start, J->t_end);
  if (J->scene) J->scene->users--;
  if (J->grf) J->grf->users--;
  C->running.erase(std::remove(C->running.begin(), C->running.end(), J), C->running.end());
  C->jobs_done++;
  C->cv.notify_all();
}

// Allocate what a queued job needs and move it to the running set.
hpt_status admit(hpt_ctx *C, Job *J) {
  if (!J->cache_build) {
    const hpt_job_desc &d = J->desc;
    hpt_status s = build_grf(C, d.grf_w, d.grf_h, d.T, d.grf_seed, C->stream, &J->grf);
    if (s != HPT_OK) return s;
    J->grf->users++;
    J->host.grf = J->grf->d;
  }
  bool ok = true;
  if (J->own_field) ok &= C->alloc((void **)&J->field, J->field_elems * sizeof(float2)) == hipSuccess;
  if (J->n_rec) ok &= C->alloc((void **)&J->rec, J->n_rec * sizeof(hpt_path_record)) == hipSuccess;
  if (J->n_contrib) ok &= C->alloc((void **)&J->contrib, J->n_contrib * sizeof(float2)) == hipSuccess;
  if (J->n_sig) ok &= C->alloc((void **)&J->sigsum, J->n_sig * sizeof(unsigned long long)) == hipSuccess;
  ok &= C->alloc((void **)&J->dev, sizeof(JobDev)) == hipSuccess;
  if (!ok) {
    free_job_buffers(C, J);
    if (J->grf) { J->grf->users--; J->grf = nullptr; }
    return fail(HPT_ENOMEM, "job allocation failed");
  }
  J->host.field = J->field;
  J->host.rec = J->rec;
  J->host.contrib = J->contrib;
  J->host.sigsum = J->sigsum;
  hipError_t e = hipSuccess;
  // the caller's stream: everything it had enqueued at submit runs before the job's first work
  if (J->ready) e = hipStreamWaitEvent(C->stream, J->ready, 0);
  if (e == hipSuccess && J->field && !J->cache_build)
    e = hipMemsetAsync(J->field, 0, J->field_elems * sizeof(float2), C->stream);
  if (e == hipSuccess && J->rec) e = hipMemsetAsync(J->rec, 0, J->n_rec * sizeof(hpt_path_record), C->stream);
  if (e == hipSuccess && J->contrib) e = hipMemsetAsync(J->contrib, 0, J->n_contrib * sizeof(float2), C->stream);
  if (e == hipSuccess && J->sigsum)
    e = hipMemsetAsync(J->sigsum, 0, J->n_sig * sizeof(unsigned long long), C->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(J->dev, &J->host, sizeof(JobDev), hipMemcpyHostToDevice, C->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(C->stream);
  if (e != hipSuccess) {
    free_job_buffers(C, J);
    return fail(HPT_EDEVICE, std::string("job set-up failed: ") + hipGetErrorString(e));
  }
  J->state = JS_RUNNING;
  C->running.push_back(J);
  return HPT_OK;
}

// Fill one batch round-robin over the running jobs. A batch holds jobs of
// one next-event-estimation mode (the shading kernel differs, and a job's
// results must not depend on what it shares a batch with); the mode is that
// of the first job with units left, counted from a start that moves with
// every batch so that neither mode waits for the other to drain.
std::vector<Picked> pick_batch(hpt_ctx *C) {
  std::vector<Picked> out;
  uint64_t paths = 0;
  std::vector<std::vector<uint32_t>> keys(C->running.size());
  std::vector<bool> blocked(C->running.size(), false);
  const size_t nr = C->running.size();
  int mode = -1;
  for (size_t k = 0; k < nr && mode < 0; ++k) {
    const Job *J = C->running[(C->batches + k) % nr];
    if (!J->cancel && J->next < J->units.size()) mode = J->ext ? 1 : 0;
  }
  for (size_t j = 0; j < nr; ++j)
    if ((C->running[j]->ext ? 1 : 0) != mode) blocked[j] = true;
  bool progress = true;
  while (progress && out.size() < kMaxUnitsPerBatch) {
    progress = false;
    for (size_t j = 0; j < C->running.size() && out.size() < kMaxUnitsPerBatch; ++j) {
      Job *J = C->running[j];
      if (blocked[j] || J->cancel || J->next >= J->units.size()) continue;
      const Unit &u = J->units[J->next];
      uint64_t np = (uint64_t)u.p_n * u.s_n;
      if (paths + np > C->capacity ||
          std::find(keys[j].begin(), keys[j].end(), u.key) != keys[j].end()) {
        blocked[j] = true;
        continue;
      }
      keys[j].push_back(u.key);
      out.push_back({J, J->next});
      J->next++;
      paths += np;
      progress = true;
    }
  }
  return out;
}

// Profiling helper: run `launch` on stream st, bracketed by an event pair of
// slot L when profiling.
template <class F>
void timed_launch(hpt_ctx::Slot &L, int kind, hipStream_t st, hipError_t &e, F &&launch) {
  if (e != hipSuccess) return;
  if (L.profile && L.ne + 2 <= hpt_ctx::kEvents) {
    e = hipEventRecord(L.pev[L.ne], st);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(L.pev[L.ne + 1], st);
    L.seg_kind[L.ne / 2] = kind;
    L.ne += 2;
  } else {
    e = launch();
  }
}

// Enqueue parts [L.acc_parts, part_end) of the accumulation (or cache
// reduction) of slot si on the accumulation stream, after the batch's last
// shading pass and after the event `after`. The accumulation is cut into
// kAccParts ranges of its lanes (each lane's sums are its own), which the
// next batch starts beside its first kAccParts traversal launches, so that
// the gather-heavy accumulation runs beside the ALU-bound tracing rather
// than beside the memory-bound ray generation or the latency-bound shading.
hipError_t launch_accumulation(hpt_ctx *C, int si, hipEvent_t after, uint32_t part_end) {
  hpt_ctx::Slot &L = C->slots[si];
  hipError_t e = hipStreamWaitEvent(C->acc, L.ev_shade, 0);
  if (e == hipSuccess && after) e = hipStreamWaitEvent(C->acc, after, 0);
  const BatchDev &B = L.B;
  for (; e == hipSuccess && L.acc_parts < part_end; ++L.acc_parts) {
    const uint32_t lo = (uint32_t)((uint64_t)B.n_acc * L.acc_parts / kAccParts);
    const uint32_t hi = (uint32_t)((uint64_t)B.n_acc * (L.acc_parts + 1) / kAccParts);
    if (L.has_holo)
      timed_launch(L, HPT_K_ACCUMULATE, C->acc, e,
                   [&] { return launch_accumulate(B, L.has_f64, L.has_f32, lo, hi, C->acc); });
  }
  if (L.acc_parts < kAccParts) return e;
  L.acc_pending = false;
  // point-emitter terms: on the same stream after the accumulation, so that
  // every read-modify-write of a pixel's field is ordered
  if (e == hipSuccess && L.pts_max_pn) e = launch_points(B, L.pts_max_pn, C->acc);
  if (L.has_cache) timed_launch(L, HPT_K_CACHE_REDUCE, C->acc, e, [&] { return launch_cache_reduce(B, C->acc); });
  if (e == hipSuccess) e = hipEventRecord(L.ev_done, C->acc);
  return e;
}

// Enqueue the batch of slot si (lock not held): raygen, then tracing and
// shading on the context stream; the batch's counters are copied to pinned
// memory after its last shading pass. The accumulation of the previous batch
// (slot `prev`, if still pending) is enqueued behind this batch's ray
// generation; this batch's own accumulation is left pending for the next
// batch or for finish_batch. The slot's result set and unit table are free:
// the batch that used them before has been finished.
hpt_status launch_batch(hpt_ctx *C, int si, int prev) {
  hpt_ctx::Slot &L = C->slots[si];
  const std::vector<Picked> &P = L.P;
  uint32_t slot = 0, acc = 0, max_b = 0;
  L.has_holo = L.has_cache = L.has_f64 = L.has_f32 = L.has_ext = false;
  L.pts_max_pn = 0;
  for (size_t k = 0; k < P.size(); ++k) {
    const Unit &u = P[k].job->units[P[k].unit];
    UnitDev &d = L.h_units[k];
    d.kind = u.kind; d.ch = u.ch; d.p_lo = u.p_lo; d.p_n = u.p_n; d.s_lo = u.s_lo; d.s_n = u.s_n;
    d.slot_base = slot; d.acc_base = acc; d.job = P[k].job->dev; d.scene = P[k].job->scene->dev;
    const JobDev &J = P[k].job->host;
    slot += u.p_n * u.s_n;
    acc += u.kind == UNIT_HOLO ? u.p_n * frame_group(J.T) : u.p_n;
    max_b = std::max(max_b, J.max_bounces);
    if (P[k].job->ext) L.has_ext = true;
    if (u.kind == UNIT_HOLO) {
      L.has_holo = true;
      if (J.phase_mode == HPT_PHASE_FP64) L.has_f64 = true; else L.has_f32 = true;
      if (u.s_lo == 0 && P[k].job->scene->host.n_pts) L.pts_max_pn = std::max(L.pts_max_pn, u.p_n);
    } else {
      L.has_cache = true;
    }
  }
  L.paths = slot;
  BatchDev &B = L.B;
  B = C->batch;
  B.s_sig = L.s_sig; B.s_first = L.s_first;
  B.res = L.res; B.r_cs64 = L.r_cs64;
  B.scene_uniform = P.empty() ? nullptr : P[0].job->scene->dev;
  B.job_uniform = P.empty() ? nullptr : P[0].job->dev;
  for (auto &p : P) {
    if (p.job->scene->dev != B.scene_uniform) B.scene_uniform = nullptr;
    if (p.job->dev != B.job_uniform) B.job_uniform = nullptr;
  }
  B.units = L.d_units;
  B.n_units = (uint32_t)P.size();
  B.n_paths = slot;
  B.n_acc = acc;
  const uint32_t profile = L.profile;
  L.ne = 0;
  hipError_t e = hipSuccess;
  hipStream_t S = C->stream;
  e = hipMemcpyAsync(L.d_units, L.h_units, P.size() * sizeof(UnitDev), hipMemcpyHostToDevice, S);
  if (e == hipSuccess) e = hipMemsetAsync(B.counters, 0, 8 * sizeof(uint32_t), S);
  if (e == hipSuccess) e = hipMemsetAsync(B.claims, 0, 2 * kClaimClasses * kClaimStride * sizeof(uint32_t), S);
  if (e == hipSuccess && profile >= 2) e = hipMemsetAsync(B.work, 0, 2 * sizeof(unsigned long long), S);
  if (e == hipSuccess) e = hipEventRecord(L.ev0, S);
  timed_launch(L, HPT_K_RAYGEN, S, e,
               [&] { return launch_raygen(B, B.job_uniform && B.n_units <= shade_lds_units(), S); });
  if (e == hipSuccess) e = hipEventRecord(L.ev_rg, S);
  if (e == hipSuccess && prev >= 0 && C->slots[prev].acc_pending) e = launch_accumulation(C, prev, L.ev_rg, 1);
  // shading copies the descriptors of a one-job batch to LDS when they fit
  const bool uni = B.job_uniform && B.scene_uniform && P[0].job->scene->host.n_mat <= shade_lds_mats() &&
                   B.n_units <= shade_lds_units();
  for (uint32_t it = 0; it <= max_b; ++it) {
    int q = (int)(it & 1u);
    timed_launch(L, HPT_K_TRACE, S, e, [&] { return launch_trace(B, q, it == 0, profile >= 2, S); });
    timed_launch(L, HPT_K_SHADE, S, e, [&] { return launch_shade(B, q, it, L.has_ext, uni, S); });
    // the last pass ends every path (interaction max_b + 1 exceeds the
    // budget), so only the earlier ones leave rays to order
    if (it < max_b) timed_launch(L, HPT_K_COMPACT, S, e, [&] { return launch_compact(B, q, S); });
    // part it + 1 of the previous batch's accumulation starts beside this
    // batch's next traversal (all that is left after the last such pass)
    if (it + 1 < kAccParts && e == hipSuccess && prev >= 0 && C->slots[prev].acc_pending) {
      e = hipEventRecord(L.ev_sh[it], S);
      const uint32_t end = (it + 2 == kAccParts || it == max_b) ? kAccParts : it + 2;
      if (e == hipSuccess) e = launch_accumulation(C, prev, L.ev_sh[it], end);
    }
  }
  if (e == hipSuccess) e = hipMemcpyAsync(L.h_cnt, B.counters, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, S);
  if (e == hipSuccess && profile >= 2)
    e = hipMemcpyAsync(L.h_work, B.work, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, S);
  if (e == hipSuccess) e = hipEventRecord(L.ev_shade, S);
  L.acc_pending = e == hipSuccess;
  L.acc_parts = 0;
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(S);
    (void)hipStreamSynchronize(C->acc);
    return fail(HPT_EDEVICE, std::string("batch failed: ") + hipGetErrorString(e));
  }
  return HPT_OK;
}

// Wait for the batch of slot si and collect its statistics (lock not held).
hpt_status finish_batch(hpt_ctx *C, int si, double &gpu_ms, uint64_t &rays, hpt_kernel_time *kt,
                        uint64_t *work) {
  hpt_ctx::Slot &L = C->slots[si];
  if (L.launch_status != HPT_OK) return L.launch_status;
  hipError_t e = L.acc_pending ? launch_accumulation(C, si, nullptr, kAccParts) : hipSuccess;
  if (e == hipSuccess) e = hipEventSynchronize(L.ev_done);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, L.ev0, L.ev_done);
  for (int k = 0; e == hipSuccess && k < L.ne; k += 2) {
    float m = 0.f;
    e = hipEventElapsedTime(&m, L.pev[k], L.pev[k + 1]);
    hpt_kernel_time &t = kt[L.seg_kind[k / 2]];
    t.launches++;
    t.total_ms += m;
  }
  if (e != hipSuccess) return fail(HPT_EDEVICE, std::string("batch failed: ") + hipGetErrorString(e));
  const uint32_t nr = L.h_cnt[2];
  if (L.profile >= 2) { work[0] = L.h_work[0]; work[1] = L.h_work[1]; }
  kt[HPT_K_RAYGEN].items += L.profile ? L.paths : 0;
  kt[HPT_K_TRACE].items += L.profile ? nr : 0;
  kt[HPT_K_SHADE].items += L.profile ? nr : 0;
  kt[HPT_K_ACCUMULATE].items += (L.profile && L.has_holo) ? L.paths : 0;
  kt[HPT_K_CACHE_REDUCE].items += (L.profile && L.has_cache) ? L.paths : 0;
  kt[HPT_K_COMPACT].items += L.profile ? nr : 0;
  gpu_ms = ms;
  rays = nr;
  return HPT_OK;
}

// Account a finished batch and retire the jobs it completed (lock held).
void account_batch(hpt_ctx *C, int si, hpt_status s, const std::string &err, double gpu_ms, uint64_t rays,
                   const hpt_kernel_time *kt, const uint64_t *work) {
  const std::vector<Picked> &P = C->slots[si].P;
  C->batches++;
  for (int k = 0; k < HPT_K_KINDS; ++k) {
    C->ktime[k].launches += kt[k].launches;
    C->ktime[k].items += kt[k].items;
    C->ktime[k].total_ms += kt[k].total_ms;
  }
  C->node_visits += work[0];
  C->prim_tests += work[1];
  uint64_t total = 0;
  for (auto &p : P) total += (uint64_t)p.job->units[p.unit].p_n * p.job->units[p.unit].s_n;
  for (auto &p : P) {
    Job *J = p.job;
    uint64_t np = (uint64_t)J->units[p.unit].p_n * J->units[p.unit].s_n;
    J->stats.paths += np;
    J->stats.rays += total ? rays * np / total : 0;
    J->stats.trace_gpu_ms += total ? gpu_ms * (double)np / (double)total : 0.0;
    J->done++;
    J->in_flight--;
  }
  std::vector<Job *> seen;
  for (auto &p : P) {
    Job *J = p.job;
    if (std::find(seen.begin(), seen.end(), J) != seen.end()) continue;
    seen.push_back(J);
    J->stats.batches++;
    if (J->state != JS_RUNNING) continue;
    if (s != HPT_OK) {
      // the job stops at its next batch boundary; a batch in the other slot
      // may still hold its units (and read its scene, table and buffers), so
      // it is retired only once none is in flight
      if (J->fail_status == HPT_OK) { J->fail_status = s; J->fail_err = err; }
      J->cancel = true;
    }
    if (J->fail_status != HPT_OK) {
      if (J->in_flight == 0) retire(C, J, JS_FAILED, J->fail_status, J->fail_err);
    } else if (J->done == J->units.size()) {
      retire(C, J, JS_DONE, HPT_OK, "");
    }
  }
  C->slots[si].P.clear();
}

// The scheduler thread: admission, batch packing and the batch pipeline
// (batch k+1 is enqueued before batch k is waited for, so the GPU always has
// the next batch queued and batch k's accumulation overlaps batch k+1's
// tracing).
void scheduler(hpt_ctx *C) {
  (void)hipSetDevice(C->device);
  std::unique_lock<std::mutex> lk(C->mu);
  int cur = 0, inflight = -1;
  for (;;) {
    C->cv.wait(lk, [&] {
      if (C->stop || inflight >= 0) return true;
      for (Job *J : C->running)
        if (J->cancel || J->next < J->units.size()) return true;
      return !C->queue.empty();
    });
    if (C->stop && inflight < 0) break;
    // cancellations at the batch boundary; a job with units in flight is
    // retired once its batch has finished
    for (size_t k = 0; k < C->running.size();) {
      Job *J = C->running[k];
      if (J->cancel && J->in_flight == 0) {
        if (J->fail_status != HPT_OK) retire(C, J, JS_FAILED, J->fail_status, J->fail_err);
        else retire(C, J, JS_CANCELED, HPT_ECANCELED, "cancelled");
      } else {
        ++k;
      }
    }
    // admission in arrival order while memory allows
    while (!C->stop && !C->queue.empty()) {
      Job *J = C->queue.front();
      if (J->cancel) {
        C->queue.pop_front();
        J->state = JS_CANCELED; J->status = HPT_ECANCELED;
        if (J->scene) J->scene->users--;
        C->cv.notify_all();
        continue;
      }
      size_t need = J->bytes + (J->cache_build || find_grf(C, J->desc.grf_w, J->desc.grf_h, J->desc.T,
                                                           J->desc.grf_seed)
                                     ? 0
                                     : J->grf_bytes);
      if (C->used + need > C->budget) evict_grfs(C, need);
      if (C->used + need > C->budget && !C->running.empty()) break;  // wait for memory
      C->queue.pop_front();
      hpt_status s = admit(C, J);
      if (s != HPT_OK) {
        J->state = JS_FAILED; J->status = s; J->err = g_err;
        if (J->scene) J->scene->users--;
        C->cv.notify_all();
      }
    }
    int launched = -1;
    if (!C->stop) {
      std::vector<Picked> P = pick_batch(C);
      if (!P.empty()) {
        for (auto &p : P) {
          if (!p.job->started) { p.job->started = true; p.job->t_start = Clock::now(); }
          p.job->in_flight++;
        }
        hpt_ctx::Slot &L = C->slots[cur];
        L.P = std::move(P);
        L.profile = C->profile;
        const bool inject = C->fail_batches > 0;
        if (inject) C->fail_batches--;
        lk.unlock();
        if (inject) {
          L.acc_pending = false;
          L.launch_status = fail(HPT_EDEVICE, "batch launch failed (injected)");
        } else {
          L.launch_status = launch_batch(C, cur, inflight);
        }
        L.err = L.launch_status == HPT_OK ? std::string() : g_err;
        lk.lock();
        launched = cur;
        cur ^= 1;
      }
    }
    if (inflight >= 0) {
      lk.unlock();
      double gpu_ms = 0.0;
      uint64_t rays = 0, work[2] = {0, 0};
      hpt_kernel_time kt[HPT_K_KINDS] = {};
      hpt_status s = finish_batch(C, inflight, gpu_ms, rays, kt, work);
      std::string err = s == HPT_OK ? std::string() : (C->slots[inflight].launch_status != HPT_OK
                                                            ? C->slots[inflight].err : g_err);
      lk.lock();
      account_batch(C, inflight, s, err, gpu_ms, rays, kt, work);
    }
    inflight = launched;
  }
  // drain: everything still queued or running is cancelled
  for (Job *J : C->queue) {
    J->state = JS_CANCELED; J->status = HPT_ECANCELED;
    if (J->scene) J->scene->users--;
  }
  C->queue.clear();
  while (!C->running.empty()) retire(C, C->running.front(), JS_CANCELED, HPT_ECANCELED, "context destroyed");
  C->cv.notify_all();
}

hpt_status alloc_batch(hpt_ctx *C) {
  uint32_t N = C->capacity;
  BatchDev &B = C->batch;
  auto A = [&](void **p, size_t bytes) {
    if (C->alloc(p, bytes) != hipSuccess) return false;
    C->batch_bufs.push_back(*p);
    C->batch_bytes += bytes;
    return true;
  };
  bool ok = true;
  for (auto &L : C->slots) {
    ok &= A((void **)&L.s_sig, 8ull * N) && A((void **)&L.s_first, 4ull * N);
    ok &= A((void **)&L.res, sizeof(PathRes) * (size_t)N) && A((void **)&L.r_cs64, 16ull * N);
    ok &= A((void **)&L.d_units, kMaxUnitsPerBatch * sizeof(UnitDev));
  }
  for (int q = 0; q < 2 && ok; ++q) {
    RayQueue &Q = B.Q[q];
    ok &= A((void **)&Q.slot, 4ull * N) && A((void **)&Q.unit, 4ull * N) &&
          A((void **)&Q.sig, 8ull * N) &&
          A((void **)&Q.bpre, 4ull * N) && A((void **)&Q.wt, 4ull * N) && A((void **)&Q.beta, 4ull * N) &&
          A((void **)&Q.L, 4ull * N) && A((void **)&Q.pdf, 4ull * N);
    ok &= A((void **)&Q.ox, 8ull * N) && A((void **)&Q.oy, 8ull * N) && A((void **)&Q.oz, 8ull * N) &&
          A((void **)&Q.dx, 8ull * N) && A((void **)&Q.dy, 8ull * N) && A((void **)&Q.dz, 8ull * N) &&
          A((void **)&Q.ell, 8ull * N);
    ok &= A((void **)&Q.ray, 32ull * N) && A((void **)&Q.t, 4ull * N) && A((void **)&Q.prim, 4ull * N);
    ok &= A((void **)&Q.idx, 4ull * N) && A((void **)&Q.cnt, 4ull * (N / 256 + 1)) &&
          A((void **)&Q.off, 4ull * (N / 256 + 1)) && A((void **)&Q.tile_sum, 4ull * 64);
  }
  ok &= A((void **)&B.counters, 64);
  ok &= A((void **)&B.claims, 2 * kClaimClasses * kClaimStride * sizeof(uint32_t));
  ok &= A((void **)&B.work, 64);
  B.spill_threads = trace_grid(N) * trace_block();
  ok &= A((void **)&B.stack_spill, (size_t)kStackSpill * B.spill_threads * sizeof(int32_t));
  if (!ok) return fail(HPT_ENOMEM, "batch buffer allocation failed");
  for (auto &L : C->slots) {
    if (hipHostMalloc((void **)&L.h_units, kMaxUnitsPerBatch * sizeof(UnitDev), hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void **)&L.h_cnt, 4 * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&L.h_work, 2 * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess)
      return fail(HPT_ENOMEM, "pinned batch table allocation failed");
    if (hipEventCreate(&L.ev0) != hipSuccess || hipEventCreate(&L.ev_rg) != hipSuccess ||
        hipEventCreate(&L.ev_shade) != hipSuccess || hipEventCreate(&L.ev_done) != hipSuccess ||
        hipEventCreateWithFlags(&L.ev_sh[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&L.ev_sh[1], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&L.ev_sh[2], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&L.ev_sh[3], hipEventDisableTiming) != hipSuccess)
      return fail(HPT_EDEVICE, "event creation failed");
    for (auto &ev : L.pev)
      if (hipEventCreate(&ev) != hipSuccess) return fail(HPT_EDEVICE, "event creation failed");
  }
  return HPT_OK;
}

Job *find_job(hpt_ctx *C, uint64_t id) {
  auto it = C->jobs.find(id);
  return it == C->jobs.end() ? nullptr : it->second.get();
}

Scene *find_scene(hpt_ctx *C, uint64_t id) {
  auto it = C->scenes.find(id);
  return it == C->scenes.end() ? nullptr : it->second.get();
}

bool finite3(const float *p) { return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]); }

}  // namespace

// =================================================================== ABI
extern "C" {

const char *hpt_last_error(void) { return g_err.c_str(); }
const char *hpt_version(void) { return "hpt-mi355x 0.1 (gfx950)"; }

hpt_status hpt_create(int device, uint64_t budget, hpt_ctx **out) {
  if (!out) return fail(HPT_EINVAL, "out is null");
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
    return fail(HPT_ENODEV, "no such HIP device");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return fail(HPT_ENODEV, "device query failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(HPT_ENODEV, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
  if (hipSetDevice(device) != hipSuccess) return fail(HPT_ENODEV, "hipSetDevice failed");
  auto C = std::make_unique<hpt_ctx>();
  C->device = device;
  // device address of the allocation-free propagation's static scratch,
  // taken once per device with the device current
  if (hipError_t e = asm_noalloc_scratch(device, &C->na_scratch); e != hipSuccess)
    return fail(HPT_EDEVICE, std::string("scratch symbol lookup failed: ") + hipGetErrorString(e));
  size_t free_b = 0, total_b = 0;
  (void)hipMemGetInfo(&free_b, &total_b);
  C->budget = budget ? budget : (uint64_t)(0.9 * (double)free_b);
  // path capacity: a power of two, at most 2^26 (larger batches mean fewer
  // launches and fewer load-imbalanced launch tails), batch buffers (path state
  // and traversal stack spill) at most a quarter of the budget
  auto batch_bytes = [](uint32_t n) {
    return (uint64_t)n * kBytesPerPath + (uint64_t)kStackSpill * 4 * trace_grid(n) * trace_block();
  };
  uint32_t c = 1u << kSlotBits;  // a queue entry's slot word holds slots below 2^kSlotBits
  while (c > (1u << 16) && batch_bytes(c) > C->budget / 4) c /= 2;
  if (batch_bytes(c) > C->budget) return fail(HPT_EBUDGET, "budget too small for path state");
  C->capacity = c;
  if (hipStreamCreateWithFlags(&C->stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&C->acc, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&C->aux, hipStreamNonBlocking) != hipSuccess)
    return fail(HPT_EDEVICE, "stream creation failed");
  hpt_status s = alloc_batch(C.get());
  if (s != HPT_OK) {
    for (void *p : C->batch_bufs) (void)hipFree(p);
    return s;
  }
  hpt_ctx *raw = C.release();
  raw->worker = std::thread(scheduler, raw);
  *out = raw;
  return HPT_OK;
}

void hpt_destroy(hpt_ctx *C) {
  if (!C) return;
  {
    std::lock_guard<std::mutex> g(C->mu);
    C->stop = true;
    for (Job *J : C->running) J->cancel = true;
  }
  C->cv.notify_all();
  if (C->worker.joinable()) C->worker.join();
  (void)hipSetDevice(C->device);
  (void)hipStreamSynchronize(C->stream);
  (void)hipStreamSynchronize(C->acc);
  for (auto &kv : C->jobs) free_job_buffers(C, kv.second.get());
  for (auto &g : C->grfs) (void)hipFree(g->d);
  for (auto &kv : C->scenes) {
    for (void *p : kv.second->bufs) (void)hipFree(p);
    (void)hipFree(kv.second->dev);
    (void)hipFree(kv.second->cache);
  }
  for (void *p : C->batch_bufs) (void)hipFree(p);
  for (auto &L : C->slots) {
    if (L.h_units) (void)hipHostFree(L.h_units);
    if (L.h_cnt) (void)hipHostFree(L.h_cnt);
    if (L.h_work) (void)hipHostFree(L.h_work);
    for (hipEvent_t ev : {L.ev0, L.ev_rg, L.ev_shade, L.ev_done, L.ev_sh[0], L.ev_sh[1], L.ev_sh[2], L.ev_sh[3]})
      if (ev) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : L.pev)
      if (ev) (void)hipEventDestroy(ev);
  }
  (void)hipStreamDestroy(C->stream);
  (void)hipStreamDestroy(C->acc);
  (void)hipStreamDestroy(C->aux);
  delete C;
}

hpt_status hpt_ctx_stats_get(hpt_ctx *C, hpt_ctx_stats *out) {
  if (!C || !out) return fail(HPT_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(C->mu);
  out->budget_bytes = C->budget;
  out->used_bytes = C->used;
  out->batch_capacity_paths = C->capacity;
  out->batches = C->batches;
  out->jobs_done = C->jobs_done;
  out->jobs_queued = C->queue.size();
  out->jobs_running = C->running.size();
  return HPT_OK;
}

hpt_status hpt_scene_upload(hpt_ctx *C, const hpt_scene_desc *d, uint64_t *out) {
  if (!C || !d || !out) return fail(HPT_EINVAL, "null argument");
  if ((d->n_tri && (!d->tri || !d->tri_mat)) || (d->n_sph && (!d->sph || !d->sph_mat)))
    return fail(HPT_EINVAL, "missing primitive arrays");
  if (d->n_mat == 0 || !d->mat_type || !d->mat_rgb || !d->mat_rough || !d->mat_ior || !d->mat_emit || !d->env)
    return fail(HPT_EINVAL, "missing material arrays");
  if ((uint64_t)d->n_tri + d->n_sph >= (1ull << 27)) return fail(HPT_EINVAL, "too many primitives");
  for (uint32_t i = 0; i < d->n_mat; ++i) {
    if (d->mat_type[i] > HPT_PRINCIPLED) return fail(HPT_EINVAL, "unknown material type");
    if ((d->mat_type[i] == HPT_GGX || d->mat_type[i] == HPT_PRINCIPLED) &&
        !(d->mat_rough[i] > 0.f && d->mat_rough[i] <= 1.f))
      return fail(HPT_EINVAL, "GGX and principled roughness must be in (0, 1]");
    if (d->mat_type[i] == HPT_PRINCIPLED && d->mat_pbr)
      for (int k = 0; k < 4; ++k)
        if (!(d->mat_pbr[4 * i + k] >= 0.f && d->mat_pbr[4 * i + k] <= 1.f))
          return fail(HPT_EINVAL, "principled parameters must be in [0, 1]");
    if (d->mat_type[i] == HPT_DIELECTRIC && !(d->mat_ior[i] > 1.f && std::isfinite(d->mat_ior[i])))
      return fail(HPT_EINVAL, "dielectric index must be > 1");
    if (!finite3(d->mat_rgb + 3 * i) || !finite3(d->mat_emit + 3 * i)) return fail(HPT_EINVAL, "non-finite material");
  }
  if (!finite3(d->env)) return fail(HPT_EINVAL, "non-finite environment");
  if (d->n_pts > 4096 || (d->n_pts && !d->pts)) return fail(HPT_EINVAL, "point emitters: at most 4096, array required");
  for (uint32_t i = 0; i < d->n_pts; ++i) {
    const float *p = d->pts + 6 * (size_t)i;
    if (!finite3(p) || !finite3(p + 3) || p[3] < 0.f || p[4] < 0.f || p[5] < 0.f)
      return fail(HPT_EINVAL, "point emitter: non-finite position or negative amplitude");
  }
  for (uint32_t i = 0; i < d->n_tri; ++i) {
    if (d->tri_mat[i] >= d->n_mat) return fail(HPT_EINVAL, "triangle material index out of range");
    for (int k = 0; k < 3; ++k)
      if (!finite3(d->tri + 9 * (size_t)i + 3 * k)) return fail(HPT_EINVAL, "non-finite vertex");
  }
  for (uint32_t i = 0; i < d->n_sph; ++i) {
    if (d->sph_mat[i] >= d->n_mat) return fail(HPT_EINVAL, "sphere material index out of range");
    if (!finite3(d->sph + 4 * i) || !(d->sph[4 * i + 3] > 0.f) || !std::isfinite(d->sph[4 * i + 3]))
      return fail(HPT_EINVAL, "bad sphere");
  }
  // host BVH build without the lock
  auto S = std::make_unique<Scene>();
  BvhResult bvh;
  uint32_t n = d->n_tri + d->n_sph;
  if (n > 0 && !build_bvh(d->tri, d->n_tri, d->sph, d->n_sph, bvh))
    return fail(HPT_EINVAL, "BVH build failed (tree deeper than the traversal stack)");
  // bounds in FP64 from the float32 data (the radiance-cache grid uses them)
  for (int a = 0; a < 3; ++a) { S->lo[a] = INFINITY; S->hi[a] = -INFINITY; }
  for (uint32_t i = 0; i < d->n_sph; ++i)
    for (int a = 0; a < 3; ++a) {
      double c = d->sph[4 * i + a], r = d->sph[4 * i + 3];
      S->lo[a] = std::min(S->lo[a], c - r); S->hi[a] = std::max(S->hi[a], c + r);
    }
  for (size_t i = 0; i < 3 * (size_t)d->n_tri; ++i)
    for (int a = 0; a < 3; ++a) {
      double v = d->tri[3 * i + a];
      S->lo[a] = std::min(S->lo[a], v); S->hi[a] = std::max(S->hi[a], v);
    }
  if (n == 0)
    for (int a = 0; a < 3; ++a) { S->lo[a] = 0; S->hi[a] = 0; }
  std::vector<MaterialDev> mats(d->n_mat);
  for (uint32_t i = 0; i < d->n_mat; ++i) {
    MaterialDev &m = mats[i];
    m.type = d->mat_type[i];
    for (int c = 0; c < 3; ++c) { m.rgb[c] = d->mat_rgb[3 * i + c]; m.emit[c] = d->mat_emit[3 * i + c]; }
    m.rough = d->mat_rough[i]; m.ior = d->mat_ior[i];
    const float *pb = d->mat_pbr ? d->mat_pbr + 4 * i : nullptr;
    m.metallic = pb ? pb[0] : 0.f; m.specular = pb ? pb[1] : 0.5f;
    m.clearcoat = pb ? pb[2] : 0.f; m.clearcoat_gloss = pb ? pb[3] : 1.f;
    m.pad[0] = m.pad[1] = m.pad[2] = 0.f;
  }
  // one shading record per primitive in leaf order: FP64 plane of a triangle
  // (the coherent-prefix refinement and the hit normal) or the sphere itself
  std::vector<HitRec> hits(n);
  for (uint32_t i = 0; i < n; ++i) {
    uint32_t g;
    std::memcpy(&g, &bvh.prims[12 * (size_t)i + 3], 4);
    HitRec &r = hits[i];
    std::memset(&r, 0, sizeof(r));
    r.gid = (int32_t)g;
    if (g < d->n_sph) {
      for (int a = 0; a < 4; ++a) r.g[a] = d->sph[4 * (size_t)g + a];
      r.mat = d->sph_mat[g];
    } else {
      const float *v = d->tri + 9 * (size_t)(g - d->n_sph);
      double e1[3] = {(double)v[3] - v[0], (double)v[4] - v[1], (double)v[5] - v[2]};
      double e2[3] = {(double)v[6] - v[0], (double)v[7] - v[1], (double)v[8] - v[2]};
      double nx = e1[1] * e2[2] - e1[2] * e2[1], ny = e1[2] * e2[0] - e1[0] * e2[2],
             nz = e1[0] * e2[1] - e1[1] * e2[0];
      double len = std::sqrt(nx * nx + ny * ny + nz * nz);
      if (len > 0) { nx /= len; ny /= len; nz /= len; }
      r.g[0] = nx; r.g[1] = ny; r.g[2] = nz;
      r.g[3] = nx * v[0] + ny * v[1] + nz * v[2];
      r.mat = d->tri_mat[g - d->n_sph];
    }
  }
  // emitter triangles (next-event estimation): vertices, unit normal, area in FP64 from the FP32 input
  std::vector<float4> lights;
  std::vector<double> light_cdf;
  double light_area = 0.0;
  for (uint32_t i = 0; i < d->n_tri; ++i) {
    const uint32_t mi = d->tri_mat[i];
    if (d->mat_type[mi] != HPT_EMITTER) continue;
    const float *t = d->tri + 9 * (size_t)i;
    double e1[3], e2[3], cr[3];
    for (int k = 0; k < 3; ++k) { e1[k] = (double)t[3 + k] - t[k]; e2[k] = (double)t[6 + k] - t[k]; }
    cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
    cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
    cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
    const double a2 = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    if (!(a2 > 0.0)) continue;
    lights.push_back(make_float4(t[0], t[1], t[2], 0.f));
    lights.push_back(make_float4(t[3], t[4], t[5], 0.f));
    lights.push_back(make_float4(t[6], t[7], t[8], 0.f));
    float mbits;
    std::memcpy(&mbits, &mi, 4);
    lights.push_back(make_float4((float)(cr[0] / a2), (float)(cr[1] / a2), (float)(cr[2] / a2), mbits));
    light_area += 0.5 * a2;
    light_cdf.push_back(light_area);
  }
  std::lock_guard<std::mutex> g(C->mu);
  (void)hipSetDevice(C->device);
  std::vector<float4> pts(2 * (size_t)d->n_pts);
  for (uint32_t i = 0; i < d->n_pts; ++i) {
    const float *p = d->pts + 6 * (size_t)i;
    pts[2 * i] = make_float4(p[0], p[1], p[2], 0.f);
    pts[2 * i + 1] = make_float4(p[3], p[4], p[5], 0.f);
  }
  size_t need = bvh.nodes.size() * 4 + bvh.prims.size() * 4 + sizeof(HitRec) * hits.size() +
                sizeof(MaterialDev) * mats.size() + sizeof(SceneDev) + sizeof(float4) * lights.size() +
                sizeof(double) * light_cdf.size() + sizeof(float4) * pts.size();
  if (C->used + need > C->budget) evict_grfs(C, need);
  if (C->used + need > C->budget) return fail(HPT_EBUDGET, "scene does not fit the budget");
  auto put = [&](const void *src, size_t bytes, void **dst) {
    if (C->alloc(dst, bytes) != hipSuccess) return false;
    S->bufs.push_back(*dst);
    S->bytes += bytes;
    return bytes == 0 || hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
  };
  bool ok = true;
  void *p;
  SceneDev &h = S->host;
  std::memset(&h, 0, sizeof(h));
  if (n > 0) {
    ok &= put(bvh.nodes.data(), bvh.nodes.size() * 4, &p); h.nodes = (const float4 *)p;
    ok &= put(bvh.prims.data(), bvh.prims.size() * 4, &p); h.prims = (const float4 *)p;
    ok &= put(hits.data(), sizeof(HitRec) * hits.size(), &p); h.hits = (const HitRec *)p;
  }
  ok &= put(mats.data(), sizeof(MaterialDev) * mats.size(), &p); h.mats = (const MaterialDev *)p;
  if (!light_cdf.empty()) {
    ok &= put(lights.data(), sizeof(float4) * lights.size(), &p); h.lights = (const float4 *)p;
    ok &= put(light_cdf.data(), sizeof(double) * light_cdf.size(), &p); h.light_cdf = (const double *)p;
  }
  h.n_lights = (uint32_t)light_cdf.size();
  h.light_area = light_area;
  if (!pts.empty()) { ok &= put(pts.data(), sizeof(float4) * pts.size(), &p); h.pts = (const float4 *)p; }
  h.n_pts = d->n_pts;
  for (uint32_t i = 0; i < d->n_mat; ++i)
    if (d->mat_type[i] == HPT_PRINCIPLED) S->principled = true;
  h.n_sph = d->n_sph; h.n_tri = d->n_tri; h.n_mat = d->n_mat; h.n_nodes = n ? bvh.n_nodes : 0;
  for (int c = 0; c < 3; ++c) h.env[c] = d->env[c];
  ok &= C->alloc((void **)&S->dev, sizeof(SceneDev)) == hipSuccess;
  if (ok) S->bytes += sizeof(SceneDev);
  ok = ok && hipMemcpy(S->dev, &h, sizeof(SceneDev), hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    for (void *q : S->bufs) C->release(q, 0);
    C->used -= std::min<uint64_t>(C->used, S->bytes);
    if (S->dev) (void)hipFree(S->dev);
    return fail(HPT_ENOMEM, "scene upload failed");
  }
  S->id = C->next_id++;
  S->info.n_nodes = h.n_nodes;
  S->info.n_prims = n;
  S->info.max_depth = bvh.max_depth;
  S->info.device_bytes = S->bytes;
  S->info.build_ms = bvh.build_ms;
  for (int a = 0; a < 3; ++a) { S->info.bounds[a] = S->lo[a]; S->info.bounds[3 + a] = S->hi[a]; }
  *out = S->id;
  C->scenes[S->id] = std::move(S);
  return HPT_OK;
}

hpt_status hpt_scene_info_get(hpt_ctx *C, uint64_t scene, hpt_scene_info *out) {
  if (!C || !out) return fail(HPT_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(C->mu);
  Scene *S = find_scene(C, scene);
  if (!S) return fail(HPT_ENOTFOUND, "unknown scene");
  *out = S->info;
  return HPT_OK;
}

hpt_status hpt_scene_release(hpt_ctx *C, uint64_t scene) {
  if (!C) return fail(HPT_EINVAL, "null context");
  std::lock_guard<std::mutex> g(C->mu);
  Scene *S = find_scene(C, scene);
  if (!S) return fail(HPT_ENOTFOUND, "unknown scene");
  if (S->users > 0) return fail(HPT_EBUSY, "scene in use by a job");
  for (auto &kv : C->jobs)
    if (kv.second->scene == S) kv.second->scene = nullptr;
  for (void *p : S->bufs) (void)hipFree(p);
  (void)hipFree(S->dev);
  if (S->cache) (void)hipFree(S->cache);
  C->used -= std::min<uint64_t>(C->used, S->bytes + S->cache_bytes);
  C->scenes.erase(scene);
  return HPT_OK;
}

namespace {
hpt_status check_cache_desc(const hpt_cache_desc *cd, uint64_t &entries) {
  if (cd->res < 1 || cd->res > 256 || cd->bins < 1 || cd->bins > 64 || cd->spb < 1 || cd->spb > 4096 ||
      cd->max_bounces < 1 || cd->max_bounces > 31)
    return fail(HPT_EINVAL, "cache parameters out of range");
  entries = (uint64_t)cd->res * cd->res * cd->res * cd->bins * cd->bins;
  if (entries >= (1ull << 31) || cd->bins * cd->bins > 65536 || cd->spb > 65535)
    return fail(HPT_EINVAL, "cache too large");
  return HPT_OK;
}

// (Re)allocate the cache of S and set up its grid: the scene bounds inflated
// by 1e-3 of their largest extent, res^3 cells (lock held).
hpt_status cache_alloc(hpt_ctx *C, Scene *S, const hpt_cache_desc *cd, uint64_t entries) {
  size_t bytes = 3 * entries * sizeof(uint16_t);
  if (S->cache) { C->release(S->cache, S->cache_bytes); S->cache = nullptr; S->cache_bytes = 0; }
  if (C->used + bytes > C->budget) evict_grfs(C, bytes);
  if (C->used + bytes > C->budget) return fail(HPT_EBUDGET, "cache does not fit the budget");
  if (C->alloc((void **)&S->cache, bytes) != hipSuccess) return fail(HPT_ENOMEM, "cache allocation failed");
  S->cache_bytes = bytes;
  S->cache_desc = *cd;
  double ext = std::max({S->hi[0] - S->lo[0], S->hi[1] - S->lo[1], S->hi[2] - S->lo[2]});
  double pad = 1e-3 * ext;
  SceneDev &h = S->host;
  for (int a = 0; a < 3; ++a) {
    h.cache_lo_d[a] = S->lo[a] - pad;
    h.cache_hi_d[a] = S->hi[a] + pad;
    h.cache_lo[a] = (float)h.cache_lo_d[a];
    double w = h.cache_hi_d[a] - h.cache_lo_d[a];
    h.cache_scale[a] = (float)(w > 0 ? cd->res / w : 0.0);
  }
  h.cache = nullptr;  // set once the entries are in place
  h.cache_res = cd->res; h.cache_bins = cd->bins;
  return HPT_OK;
}
}  // namespace

hpt_status hpt_cache_import(hpt_ctx *C, uint64_t scene, const hpt_cache_desc *cd, const uint16_t *host, size_t n) {
  if (!C || !cd || !host) return fail(HPT_EINVAL, "null argument");
  uint64_t entries = 0;
  hpt_status st = check_cache_desc(cd, entries);
  if (st != HPT_OK) return st;
  if (n != 3 * entries) return fail(HPT_EINVAL, "size mismatch: n must be 3 res^3 bins^2");
  std::lock_guard<std::mutex> g(C->mu);
  Scene *S = find_scene(C, scene);
  if (!S) return fail(HPT_ENOTFOUND, "unknown scene");
  if (S->users > 0) return fail(HPT_EBUSY, "scene in use by a job");
  (void)hipSetDevice(C->device);
  st = cache_alloc(C, S, cd, entries);
  if (st != HPT_OK) return st;
  if (hipMemcpy(S->cache, host, S->cache_bytes, hipMemcpyHostToDevice) != hipSuccess)
    return fail(HPT_EDEVICE, "cache copy failed");
  S->host.cache = S->cache;
  if (hipMemcpy(S->dev, &S->host, sizeof(SceneDev), hipMemcpyHostToDevice) != hipSuccess)
    return fail(HPT_EDEVICE, "scene update failed");
  return HPT_OK;
}

hpt_status hpt_cache_build(hpt_ctx *C, uint64_t scene, const hpt_cache_desc *cd) {
  if (!C || !cd) return fail(HPT_EINVAL, "null argument");
  uint64_t entries = 0;
  hpt_status cst = check_cache_desc(cd, entries);
  if (cst != HPT_OK) return cst;
  uint64_t id;
  {
    std::unique_lock<std::mutex> lk(C->mu);
    Scene *S = find_scene(C, scene);
    if (!S) return fail(HPT_ENOTFOUND, "unknown scene");
    if (S->users > 0) return fail(HPT_EBUSY, "scene in use by a job");
    (void)hipSetDevice(C->device);
    cst = cache_alloc(C, S, cd, entries);
    if (cst != HPT_OK) return cst;
    SceneDev &h = S->host;  // h.cache stays null (unused) while the cache is being built
    if (hipMemcpy(S->dev, &h, sizeof(SceneDev), hipMemcpyHostToDevice) != hipSuccess)
      return fail(HPT_EDEVICE, "scene update failed");
    auto J = std::make_unique<Job>();
    J->id = id = C->next_id++;
    J->scene = S;
    J->cache_build = true;
    J->ext = S->principled;
    JobDev &jd = J->host;
    std::memset(&jd, 0, sizeof(jd));
    jd.max_bounces = cd->max_bounces;
    jd.seed = cd->seed;
    jd.scene = S->dev;
    jd.cache_out = S->cache;
    jd.cache_res = cd->res; jd.cache_bins = cd->bins; jd.cache_spb = cd->spb;
    jd.spp = 1;
    jd.T = 1;
    split_cache_units(J.get(), C->capacity);
    J->bytes = sizeof(JobDev);
    J->t_submit = Clock::now();
    S->users++;
    C->queue.push_back(J.get());
    C->jobs[id] = std::move(J);
  }
  C->cv.notify_all();
  std::unique_lock<std::mutex> lk(C->mu);
  Job *J = find_job(C, id);
  C->cv.wait(lk, [&] { return J->state != JS_QUEUED && J->state != JS_RUNNING; });
  hpt_status st = J->status;
  std::string err = J->err;
  Scene *S = find_scene(C, scene);
  free_job_buffers(C, J);
  C->jobs.erase(id);
  if (st != HPT_OK) return fail(st, err);
  if (S) {
    S->host.cache = S->cache;
    if (hipMemcpy(S->dev, &S->host, sizeof(SceneDev), hipMemcpyHostToDevice) != hipSuccess)
      return fail(HPT_EDEVICE, "scene update failed");
  }
  return HPT_OK;
}

hpt_status hpt_cache_export(hpt_ctx *C, uint64_t scene, uint16_t *host, size_t n) {
  if (!C || !host) return fail(HPT_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(C->mu);
  Scene *S = find_scene(C, scene);
  if (!S) return fail(HPT_ENOTFOUND, "unknown scene");
  if (!S->host.cache) return fail(HPT_EINVAL, "scene has no radiance cache");
  if (n * sizeof(uint16_t) != S->cache_bytes) return fail(HPT_EINVAL, "size mismatch");
  if (hipMemcpy(host, S->cache, S->cache_bytes, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(HPT_EDEVICE, "copy failed");
  return HPT_OK;
}

hpt_status hpt_trace_submit(hpt_ctx *C, uint64_t scene, const hpt_job_desc *d, void *d_field, void *hip_stream,
                            uint64_t *out) {
  if (!C || !d || !out) return fail(HPT_EINVAL, "null argument");
  if (d->width == 0 || d->height == 0 || d->width > 32768 || d->height > 32768)
    return fail(HPT_EINVAL, "bad SLM size");
  if (!(d->pitch > 0) || !std::isfinite(d->pitch)) return fail(HPT_EINVAL, "bad pitch");
  if (d->n_ch < 1 || d->n_ch > 3) return fail(HPT_EINVAL, "n_ch must be 1..3");
  if (d->T < 1 || d->T > (uint32_t)kMaxT) return fail(HPT_EINVAL, "T must be 1..64");
  if (d->spp < 1) return fail(HPT_EINVAL, "spp must be >= 1");
  if (d->max_bounces < 1 || d->max_bounces > 31) return fail(HPT_EINVAL, "max_bounces must be 1..31");
  if (d->phase_mode > HPT_PHASE_FP32) return fail(HPT_EINVAL, "bad phase mode");
  for (uint32_t c = 0; c < d->n_ch; ++c) {
    if (!(d->lambda[c] > 0) || !std::isfinite(d->lambda[c])) return fail(HPT_EINVAL, "bad wavelength");
    if (!(d->lambda[c] / (2 * d->pitch) < 1.0)) return fail(HPT_EINVAL, "lambda/(2 pitch) must be < 1");
    if (d->comp[c] > 2) return fail(HPT_EINVAL, "colour component must be 0..2");
  }
  if (d->grf_w < d->width || d->grf_h < d->height || d->grf_w > 4096 || d->grf_h > 4096)
    return fail(HPT_EINVAL, "random-field grid must cover the SLM and be <= 4096");
  uint32_t x0 = d->crop[0], y0 = d->crop[1], cw = d->crop[2], ch = d->crop[3];
  if (cw == 0 || ch == 0) { x0 = 0; y0 = 0; cw = d->width; ch = d->height; }
  if ((uint64_t)x0 + cw > d->width || (uint64_t)y0 + ch > d->height) return fail(HPT_EINVAL, "crop outside SLM");
  uint32_t sb = d->spp_begin, se = d->spp_end;
  if (sb == 0 && se == 0) se = d->spp;
  if (!(sb < se) || se > d->spp) return fail(HPT_EINVAL, "empty or invalid sample range");
  for (int k = 0; k < 12; ++k)
    if (!std::isfinite(d->holo_from_world[k])) return fail(HPT_EINVAL, "non-finite transform");
  double Ti[12];
  if (!affine_inverse(d->holo_from_world, Ti)) return fail(HPT_EINVAL, "singular transform");
  uint64_t n_paths = (uint64_t)d->n_ch * cw * ch * (se - sb);
  if ((d->debug & 3u) && n_paths > (1ull << 22)) return fail(HPT_EINVAL, "per-path debug output limited to 2^22 paths");
  std::unique_lock<std::mutex> lk(C->mu);
  Scene *S = find_scene(C, scene);
  if (!S) return fail(HPT_ENOTFOUND, "unknown scene");
  if (d->use_cache && !S->host.cache) return fail(HPT_EINVAL, "use_cache needs hpt_cache_build first");
  if (d->nee > 1) return fail(HPT_EINVAL, "nee must be 0 or 1");
  if (d->weight_mode > HPT_WEIGHT_PAPER_LITERAL) return fail(HPT_EINVAL, "unknown weight mode");
  auto J = std::make_unique<Job>();
  J->desc = *d;
  J->scene = S;
  J->ext = S->principled || d->nee != 0;
  JobDev &jd = J->host;
  std::memset(&jd, 0, sizeof(jd));
  jd.width = d->width; jd.height = d->height; jd.pitch = d->pitch;
  jd.crop_x0 = x0; jd.crop_y0 = y0; jd.crop_w = cw; jd.crop_h = ch;
  jd.n_ch = d->n_ch;
  for (uint32_t c = 0; c < d->n_ch; ++c) {
    jd.comp[c] = d->comp[c];
    jd.lambda[c] = d->lambda[c];
    jd.inv_lambda[c] = 1.0 / d->lambda[c];
    jd.s_cone[c] = d->lambda[c] / (2.0 * d->pitch);
    jd.lambda_f[c] = (float)jd.lambda[c];
    jd.inv_lambda_f[c] = (float)jd.inv_lambda[c];
    jd.s_cone_f[c] = (float)jd.s_cone[c];
  }
  jd.spp = d->spp; jd.max_bounces = d->max_bounces; jd.T = d->T; jd.phase_mode = d->phase_mode;
  jd.random_phase = d->random_phase ? 1 : 0;
  jd.use_cache = d->use_cache ? 1 : 0;
  jd.nee = d->nee ? 1 : 0;
  jd.weight_mode = d->weight_mode;
  jd.cache_depth = d->cache_depth;
  jd.debug = d->debug;
  jd.seed = d->seed;
  std::memcpy(jd.Tm, d->holo_from_world, sizeof(jd.Tm));
  std::memcpy(jd.Ti, Ti, sizeof(jd.Ti));
  static const double I[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};
  jd.identity_T = std::memcmp(I, d->holo_from_world, sizeof(I)) == 0 ? 1 : 0;
  jd.grf_w = d->grf_w; jd.grf_h = d->grf_h;
  jd.spp_lo = sb; jd.n_s = se - sb;
  jd.scene = S->dev;
  J->field_elems = (size_t)d->n_ch * d->T * cw * ch;
  J->own_field = d_field == nullptr;
  J->field = (float2 *)d_field;
  if (d->debug & 1u) J->n_rec = n_paths;
  if (d->debug & 2u) J->n_contrib = n_paths * d->T;
  if (d->debug & 4u) J->n_sig = (size_t)d->n_ch * cw * ch;
  J->bytes = (J->own_field ? J->field_elems * sizeof(float2) : 0) + J->n_rec * sizeof(hpt_path_record) +
             J->n_contrib * sizeof(float2) + J->n_sig * 8 + sizeof(JobDev);
  J->grf_bytes = grf_table_bytes(d->grf_w, d->grf_h, d->T) + grf_temp_bytes(d->grf_w, d->grf_h, d->T);
  // the fixed part (batch buffers, scenes, caches) never shrinks; refuse what can never fit
  uint64_t fixed = C->batch_bytes;
  for (auto &kv : C->scenes) fixed += kv.second->bytes + kv.second->cache_bytes;
  if (fixed + J->bytes + J->grf_bytes > C->budget) return fail(HPT_EBUDGET, "job can never fit the budget");
  if (hip_stream) {
    (void)hipSetDevice(C->device);
    if (hipEventCreateWithFlags(&J->ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(J->ready, (hipStream_t)hip_stream) != hipSuccess) {
      if (J->ready) (void)hipEventDestroy(J->ready);
      return fail(HPT_EDEVICE, "cannot record an event on the caller's stream");
    }
  }
  split_units(J.get(), C->capacity);
  J->id = C->next_id++;
  J->t_submit = Clock::now();
  S->users++;
  *out = J->id;
  C->queue.push_back(J.get());
  C->jobs[J->id] = std::move(J);
  lk.unlock();
  C->cv.notify_all();
  return HPT_OK;
}

hpt_status hpt_job_wait(hpt_ctx *C, uint64_t id, int64_t timeout_ms) {
  if (!C) return fail(HPT_EINVAL, "null context");
  std::unique_lock<std::mutex> lk(C->mu);
  Job *J = find_job(C, id);
  if (!J) return fail(HPT_ENOTFOUND, "unknown job");
  auto done = [&] { return J->state == JS_DONE || J->state == JS_FAILED || J->state == JS_CANCELED; };
  if (timeout_ms < 0) C->cv.wait(lk, done);
  else if (!C->cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), done))
    return fail(HPT_ETIMEOUT, "job not finished");
  if (J->status != HPT_OK) return fail(J->status, J->err);
  return HPT_OK;
}

hpt_status hpt_job_stats_get(hpt_ctx *C, uint64_t id, hpt_job_stats *out) {
  if (!C || !out) return fail(HPT_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(C->mu);
  Job *J = find_job(C, id);
  if (!J) return fail(HPT_ENOTFOUND, "unknown job");
  *out = J->stats;
  return HPT_OK;
}

static hpt_status copy_out(hpt_ctx *C, uint64_t id, int what, void *host, size_t n) {
  if (!C || !host) return fail(HPT_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(C->mu);
  Job *J = find_job(C, id);
  if (!J) return fail(HPT_ENOTFOUND, "unknown job");
  if (J->state != JS_DONE) return fail(J->state == JS_QUEUED || J->state == JS_RUNNING ? HPT_EBUSY : J->status,
                                       "job has not finished successfully");
  const void *src;
  size_t bytes;
  if (what == 0) { src = J->field; bytes = J->field_elems * sizeof(float2); if (n * 4 != bytes) return fail(HPT_EINVAL, "size mismatch"); }
  else if (what == 1) { src = J->rec; bytes = J->n_rec * sizeof(hpt_path_record); if (n * sizeof(hpt_path_record) != bytes) return fail(HPT_EINVAL, "size mismatch"); }
  else if (what == 2) { src = J->contrib; bytes = J->n_contrib * sizeof(float2); if (n * 4 != bytes) return fail(HPT_EINVAL, "size mismatch"); }
  else { src = J->sigsum; bytes = J->n_sig * 8; if (n * 8 != bytes) return fail(HPT_EINVAL, "size mismatch"); }
  if (!src) return fail(HPT_EINVAL, "the job has no such output (debug flags)");
  (void)hipSetDevice(C->device);
  if (hipMemcpy(host, src, bytes, hipMemcpyDeviceToHost) != hipSuccess) return fail(HPT_EDEVICE, "copy failed");
  return HPT_OK;
}

hpt_status hpt_field_read(hpt_ctx *C, uint64_t id, float *host, size_t n) { return copy_out(C, id, 0, host, n); }
hpt_status hpt_paths_read(hpt_ctx *C, uint64_t id, hpt_path_record *host, size_t n) {
  return copy_out(C, id, 1, host, n);
}
hpt_status hpt_contrib_read(hpt_ctx *C, uint64_t id, float *host, size_t n) { return copy_out(C, id, 2, host, n); }
hpt_status hpt_sigsum_read(hpt_ctx *C, uint64_t id, uint64_t *host, size_t n) {
  return copy_out(C, id, 3, host, n);
}

hpt_status hpt_field_device_ptr(hpt_ctx *C, uint64_t id, void **out) {
  if (!C || !out) return fail(HPT_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(C->mu);
  Job *J = find_job(C, id);
  if (!J) return fail(HPT_ENOTFOUND, "unknown job");
  if (!J->field) return fail(HPT_EBUSY, "field not allocated yet");
  *out = J->field;
  return HPT_OK;
}

hpt_status hpt_job_cancel(hpt_ctx *C, uint64_t id) {
  if (!C) return fail(HPT_EINVAL, "null context");
  {
    std::lock_guard<std::mutex> g(C->mu);
    Job *J = find_job(C, id);
    if (!J) return fail(HPT_ENOTFOUND, "unknown job");
    J->cancel = true;
  }
  C->cv.notify_all();
  return HPT_OK;
}

hpt_status hpt_job_release(hpt_ctx *C, uint64_t id) {
  if (!C) return fail(HPT_EINVAL, "null context");
  std::lock_guard<std::mutex> g(C->mu);
  Job *J = find_job(C, id);
  if (!J) return fail(HPT_ENOTFOUND, "unknown job");
  if (J->state == JS_QUEUED || J->state == JS_RUNNING) return fail(HPT_EBUSY, "job still active");
  (void)hipSetDevice(C->device);
  free_job_buffers(C, J);
  C->jobs.erase(id);
  return HPT_OK;
}

hpt_status hpt_debug_fail_batches(hpt_ctx *C, uint32_t n) {
  if (!C) return fail(HPT_EINVAL, "null context");
  {
    std::lock_guard<std::mutex> g(C->mu);
    C->fail_batches = n;
  }
  C->cv.notify_all();
  return HPT_OK;
}

hpt_status hpt_profile_set(hpt_ctx *C, uint32_t level) {
  if (!C || level > 2) return fail(HPT_EINVAL, "bad argument");
  std::lock_guard<std::mutex> g(C->mu);
  C->profile = level;
  return HPT_OK;
}

hpt_status hpt_profile_get(hpt_ctx *C, hpt_kernel_time *out, uint64_t *node_visits, uint64_t *prim_tests) {
  if (!C || !out) return fail(HPT_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(C->mu);
  for (int k = 0; k < HPT_K_KINDS; ++k) out[k] = C->ktime[k];
  if (node_visits) *node_visits = C->node_visits;
  if (prim_tests) *prim_tests = C->prim_tests;
  return HPT_OK;
}

hpt_status hpt_profile_reset(hpt_ctx *C) {
  if (!C) return fail(HPT_EINVAL, "null context");
  std::lock_guard<std::mutex> g(C->mu);
  for (int k = 0; k < HPT_K_KINDS; ++k) C->ktime[k] = hpt_kernel_time{};
  C->node_visits = C->prim_tests = 0;
  return HPT_OK;
}

hpt_status hpt_grf_read(hpt_ctx *C, uint32_t gw, uint32_t gh, uint32_t T, uint64_t seed, float *host, size_t n) {
  if (!C || !host) return fail(HPT_EINVAL, "null argument");
  if (gw < 1 || gh < 1 || gw > 4096 || gh > 4096 || T < 1 || T > (uint32_t)kMaxT)
    return fail(HPT_EINVAL, "bad table size");
  if (n != 2ull * gw * gh * T) return fail(HPT_EINVAL, "size mismatch");
  std::lock_guard<std::mutex> g(C->mu);
  (void)hipSetDevice(C->device);
  Grf *G = nullptr;
  hpt_status s = build_grf(C, gw, gh, T, seed, C->aux, &G);
  if (s != HPT_OK) return s;
  if (hipMemcpy(host, G->d, G->bytes, hipMemcpyDeviceToHost) != hipSuccess) return fail(HPT_EDEVICE, "copy failed");
  return HPT_OK;
}

}  // extern "C"

// Fields per launch of the FFT passes: their grids index fields in a
// dimension limited to 65535 blocks.
constexpr uint32_t kMaxFieldsPerLaunch = 65535;

namespace {
// Order the work about to be enqueued on `work` after everything enqueued on
// the caller's stream so far (no-op for a null caller stream).
hipError_t after_caller(hipStream_t work, void *caller) {
  if (!caller) return hipSuccess;
  hipEvent_t ev;
  hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e != hipSuccess) return e;
  e = hipEventRecord(ev, (hipStream_t)caller);
  if (e == hipSuccess) e = hipStreamWaitEvent(work, ev, 0);
  (void)hipEventDestroy(ev);  // released once the wait has been satisfied
  return e;
}

// Transfer-function constants of one propagation (na > 0: pupil cutoff NA / lambda).
AsmParams asm_params(uint32_t width, uint32_t height, double pitch, double lambda, double distance, uint32_t flags,
                     double na) {
  const uint32_t px = asm_padded(width), py = asm_padded(height);
  AsmParams P;
  P.dfx = 1.0 / (px * pitch);
  P.dfy = 1.0 / (py * pitch);
  P.lim_x = 1.0 / (lambda * std::sqrt(std::pow(2.0 * distance * P.dfx, 2) + 1.0));
  P.lim_y = 1.0 / (lambda * std::sqrt(std::pow(2.0 * distance * P.dfy, 2) + 1.0));
  P.inv_lam = 1.0 / lambda;
  P.inv_lam2 = P.inv_lam * P.inv_lam;
  P.z = distance;
  const double zr = distance / lambda;
  P.z_rev_frac = zr - std::floor(zr);
  P.pupil2 = na > 0.0 ? (na / lambda) * (na / lambda) : 0.0;
  P.band_limit = (flags & HPT_ASM_BAND_LIMIT) ? 1u : 0u;
  return P;
}
}  // namespace

extern "C" {

hpt_status hpt_asm_propagate(hpt_ctx *C, const void *d_in, void *d_out, uint32_t n_fields, uint32_t width,
                             uint32_t height, double pitch, double lambda, double distance, uint32_t flags,
                             void *hip_stream) {
  if (!C || !d_in || !d_out) return fail(HPT_EINVAL, "null argument");
  if (n_fields < 1 || width < 1 || height < 1 || width > 4096 || height > 4096)
    return fail(HPT_EINVAL, "field size out of range (1..4096 per axis, at least one field)");
  if (!(pitch > 0) || !std::isfinite(pitch) || !(lambda > 0) || !std::isfinite(lambda) || !std::isfinite(distance))
    return fail(HPT_EINVAL, "bad pitch, wavelength or distance");
  if (flags & ~HPT_ASM_BAND_LIMIT) return fail(HPT_EINVAL, "unknown flags");
  const uint32_t px = asm_padded(width), py = asm_padded(height);
  const AsmParams P = asm_params(width, height, pitch, lambda, distance, flags, 0.0);
  // scratch for a chunk of fields: two [h][Px] complex64 buffers per field
  const uint64_t per = 2ull * height * px * sizeof(float2);
  float2 *A = nullptr, *B = nullptr, *W = nullptr;
  const size_t tw_bytes = (size_t)(px + py) * sizeof(float2);  // twiddle tables
  uint32_t chunk = 0;
  {
    std::lock_guard<std::mutex> g(C->mu);
    (void)hipSetDevice(C->device);
    uint64_t free_b = C->budget > C->used ? C->budget - C->used : 0;
    if (free_b < per) evict_grfs(C, per);
    free_b = C->budget > C->used ? C->budget - C->used : 0;
    chunk = (uint32_t)std::min<uint64_t>({(uint64_t)n_fields, free_b / per, std::max<uint64_t>(1, (1ull << 30) / per),
                                           (uint64_t)kMaxFieldsPerLaunch});
    if (chunk == 0) return fail(HPT_EBUDGET, "propagation scratch does not fit the budget");
    const size_t half = (size_t)chunk * height * px * sizeof(float2);
    if (C->alloc((void **)&A, half) != hipSuccess) return fail(HPT_ENOMEM, "scratch allocation failed");
    if (C->alloc((void **)&B, half) != hipSuccess) {
      C->release(A, half);
      return fail(HPT_ENOMEM, "scratch allocation failed");
    }
    if (C->alloc((void **)&W, tw_bytes) != hipSuccess) {
      C->release(A, half);
      C->release(B, half);
      return fail(HPT_ENOMEM, "scratch allocation failed");
    }
  }
  hipError_t e = after_caller(C->aux, hip_stream);
  if (e == hipSuccess) e = launch_asm_twiddles(W, width, height, C->aux);
  const size_t field = (size_t)width * height;
  for (uint32_t f0 = 0; f0 < n_fields && e == hipSuccess; f0 += chunk) {
    uint32_t nf = std::min(chunk, n_fields - f0);
    e = launch_asm((const float2 *)d_in + f0 * field, (float2 *)d_out + f0 * field, A, B, W, nf, width, height,
                   P, C->aux);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(C->aux);
  else (void)hipStreamSynchronize(C->aux);  // launches already queued still use the scratch
  {
    std::lock_guard<std::mutex> g(C->mu);
    const size_t half = (size_t)chunk * height * px * sizeof(float2);
    C->release(A, half);
    C->release(B, half);
    C->release(W, tw_bytes);
  }
  if (e != hipSuccess) return fail(HPT_EDEVICE, std::string("propagation failed: ") + hipGetErrorString(e));
  return HPT_OK;
}

hpt_status hpt_asm_propagate_noalloc(hpt_ctx *C, const void *d_in, void *d_out, uint32_t n_fields, uint32_t width,
                                     uint32_t height, double pitch, double lambda, double distance, uint32_t flags,
                                     void *hip_stream) {
  if (!C || !d_in || !d_out) return fail(HPT_EINVAL, "null argument");
  if (n_fields < 1 || width < 1 || height < 1 || width > 4096 || height > 4096)
    return fail(HPT_EINVAL, "field size out of range (1..4096 per axis, at least one field)");
  if (!(pitch > 0) || !std::isfinite(pitch) || !(lambda > 0) || !std::isfinite(lambda) || !std::isfinite(distance))
    return fail(HPT_EINVAL, "bad pitch, wavelength or distance");
  if (flags & ~HPT_ASM_BAND_LIMIT) return fail(HPT_EINVAL, "unknown flags");
  const uint32_t px = asm_padded(width), py = asm_padded(height);
  auto up = [](size_t n) { return (n + 31) / 32 * 32; };   // 256-byte boundaries
  const size_t tw = up((size_t)px + py), per = up((size_t)height * px);
  if (tw + 2 * per > kNoAllocScratchElems)
    return fail(HPT_EINVAL, "field too large for the static scratch: 2 height P_x + P_x + P_y complex64 must fit "
                            "9437184 (P: padded sizes)");
  const uint32_t chunk = (uint32_t)std::min<size_t>({(size_t)n_fields, (kNoAllocScratchElems - tw) / (2 * per),
                                                     (size_t)kMaxFieldsPerLaunch});
  const AsmParams P = asm_params(width, height, pitch, lambda, distance, flags, 0.0);
  // scratch: twiddle tables, then the two work buffers of a chunk of fields
  float2 *W = C->na_scratch, *A = W + tw, *B = A + (size_t)chunk * height * px;
  hipStream_t st = hip_stream ? (hipStream_t)hip_stream : C->aux;
  (void)hipSetDevice(C->device);
  hipError_t e = launch_asm_twiddles(W, width, height, st);
  const size_t field = (size_t)width * height;
  for (uint32_t f0 = 0; f0 < n_fields && e == hipSuccess; f0 += chunk) {
    const uint32_t nf = std::min(chunk, n_fields - f0);
    e = launch_asm((const float2 *)d_in + f0 * field, (float2 *)d_out + f0 * field, A, B, W, nf, width, height, P,
                   st);
  }
  if (e == hipSuccess && !hip_stream) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(HPT_EDEVICE, std::string("propagation failed: ") + hipGetErrorString(e));
  return HPT_OK;
}

hpt_status hpt_encode_phase(hpt_ctx *C, const void *d_fields, uint32_t n_fields, uint32_t width, uint32_t height,
                            double pitch, double lambda, double distance, uint32_t iterations, double lr,
                            uint32_t flags, void *d_phase, double *loss_out, void *hip_stream) {
  if (!C || !d_fields || !d_phase) return fail(HPT_EINVAL, "null argument");
  if (n_fields < 1 || width < 1 || height < 1 || width > 4096 || height > 4096)
    return fail(HPT_EINVAL, "field size out of range (1..4096 per axis, at least one field)");
  if (!(pitch > 0) || !std::isfinite(pitch) || !(lambda > 0) || !std::isfinite(lambda) || !std::isfinite(distance))
    return fail(HPT_EINVAL, "bad pitch, wavelength or distance");
  if (iterations > 100000 || !(lr > 0) || !std::isfinite(lr)) return fail(HPT_EINVAL, "bad iteration count or step");
  if (flags & ~(HPT_ASM_BAND_LIMIT | HPT_ENCODE_WARM_START)) return fail(HPT_EINVAL, "unknown flags");
  const uint32_t px = asm_padded(width), py = asm_padded(height);
  const uint32_t bl = flags & HPT_ASM_BAND_LIMIT;
  const AsmParams Pf = asm_params(width, height, pitch, lambda, distance, bl, 0.0);
  const AsmParams Pb = asm_params(width, height, pitch, lambda, -distance, bl, 0.0);
  const uint32_t hw = width * height;
  const uint32_t nb = enc_dot_blocks(hw);
  // per field: target V, phasor a, work field R (complex64), Adam moments m, v
  // (float), two ASM buffers [h][Px], dot partials, |V|^2, scale
  const uint64_t per = 32ull * hw + 16ull * height * px + 24ull * nb + 8 + 16;
  const size_t tw_bytes = (size_t)(px + py) * sizeof(float2);
  const size_t rel_bytes = (size_t)n_fields * sizeof(double);
  std::vector<std::pair<void **, size_t>> bufs;
  float2 *V = nullptr, *a = nullptr, *R = nullptr, *A = nullptr, *B = nullptr, *W = nullptr;
  float *m = nullptr, *v = nullptr;
  double *part = nullptr, *vv = nullptr, *rel = nullptr;
  double2 *sc = nullptr;
  uint32_t chunk = 0;
  {
    std::lock_guard<std::mutex> g(C->mu);
    (void)hipSetDevice(C->device);
    const uint64_t fixed = tw_bytes + rel_bytes;
    uint64_t free_b = C->budget > C->used ? C->budget - C->used : 0;
    if (free_b < per + fixed) evict_grfs(C, per + fixed);
    free_b = C->budget > C->used ? C->budget - C->used : 0;
    free_b = free_b > fixed ? free_b - fixed : 0;
    chunk = (uint32_t)std::min<uint64_t>({(uint64_t)n_fields, free_b / per, std::max<uint64_t>(1, (1ull << 30) / per),
                                           (uint64_t)kMaxFieldsPerLaunch});
    if (chunk == 0) return fail(HPT_EBUDGET, "encoding scratch does not fit the budget");
    const size_t f = (size_t)chunk * hw, ap = (size_t)chunk * height * px;
    bufs = {{(void **)&V, 8 * f}, {(void **)&a, 8 * f}, {(void **)&R, 8 * f}, {(void **)&m, 4 * f},
            {(void **)&v, 4 * f}, {(void **)&A, 8 * ap}, {(void **)&B, 8 * ap},
            {(void **)&part, (size_t)chunk * nb * 3 * sizeof(double)}, {(void **)&vv, chunk * sizeof(double)},
            {(void **)&sc, chunk * sizeof(double2)}, {(void **)&rel, rel_bytes}, {(void **)&W, tw_bytes}};
    bool ok = true;
    for (auto &b : bufs) ok = ok && C->alloc(b.first, b.second) == hipSuccess;
    if (!ok) {
      for (auto &b : bufs)
        if (*b.first) C->release(*b.first, b.second);
      return fail(HPT_ENOMEM, "scratch allocation failed");
    }
  }
  hipStream_t st = C->aux;
  hipError_t e = after_caller(st, hip_stream);
  if (e == hipSuccess) e = launch_asm_twiddles(W, width, height, st);
  const bool warm = (flags & HPT_ENCODE_WARM_START) != 0;
  for (uint32_t f0 = 0; f0 < n_fields && e == hipSuccess; f0 += chunk) {
    const uint32_t nf = std::min(chunk, n_fields - f0);
    const size_t n = (size_t)nf * hw;
    const float2 *U = (const float2 *)d_fields + (size_t)f0 * hw;
    float *phi = (float *)d_phase + (size_t)f0 * hw;
    e = launch_asm(U, V, A, B, W, nf, width, height, Pf, st);
    if (e == hipSuccess) e = launch_enc_norm(V, part, vv, nf, hw, st);
    if (e == hipSuccess) e = launch_enc_init(U, phi, a, n, warm, st);
    if (e == hipSuccess) e = hipMemsetAsync(m, 0, 4 * n, st);
    if (e == hipSuccess) e = hipMemsetAsync(v, 0, 4 * n, st);
    for (uint32_t k = 1; k <= iterations && e == hipSuccess; ++k) {
      e = launch_asm(a, R, A, B, W, nf, width, height, Pf, st);
      if (e == hipSuccess) e = launch_enc_scale(R, V, part, vv, sc, rel + f0, nf, hw, st);
      if (e == hipSuccess) e = launch_enc_residual(R, V, sc, nf, hw, st);
      if (e == hipSuccess) e = launch_asm(R, R, A, B, W, nf, width, height, Pb, st);
      const float bc1 = (float)(1.0 - std::pow(0.9, (double)k)), bc2 = (float)(1.0 - std::pow(0.999, (double)k));
      if (e == hipSuccess) e = launch_enc_adam(phi, m, v, a, R, n, (float)lr, bc1, bc2, st);
    }
    if (e == hipSuccess) e = launch_asm(a, R, A, B, W, nf, width, height, Pf, st);
    if (e == hipSuccess) e = launch_enc_scale(R, V, part, vv, sc, rel + f0, nf, hw, st);
  }
  std::vector<double> rel_h(n_fields, 0.0);
  if (e == hipSuccess) e = hipMemcpyAsync(rel_h.data(), rel, rel_bytes, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  else (void)hipStreamSynchronize(st);  // launches already queued still use the scratch
  {
    std::lock_guard<std::mutex> g(C->mu);
    for (auto &b : bufs) C->release(*b.first, b.second);
  }
  if (e != hipSuccess) return fail(HPT_EDEVICE, std::string("encoding failed: ") + hipGetErrorString(e));
  if (loss_out) std::copy(rel_h.begin(), rel_h.end(), loss_out);
  return HPT_OK;
}

hpt_status hpt_reconstruct(hpt_ctx *C, const void *d_fields, uint32_t n_ch, uint32_t T, uint32_t width,
                           uint32_t height, double pitch, const double *lambdas, uint32_t n_planes,
                           const double *distances, double na, uint32_t flags, void *d_out, void *hip_stream) {
  if (!C || !d_fields || !d_out || !lambdas || !distances) return fail(HPT_EINVAL, "null argument");
  if (n_ch < 1 || T < 1 || n_planes < 1 || n_planes > 64)
    return fail(HPT_EINVAL, "need n_ch >= 1, T >= 1 and 1..64 planes");
  if (width < 1 || height < 1 || width > 4096 || height > 4096)
    return fail(HPT_EINVAL, "field size out of range (1..4096 per axis)");
  if (!(pitch > 0) || !std::isfinite(pitch) || !std::isfinite(na)) return fail(HPT_EINVAL, "bad pitch or aperture");
  for (uint32_t c = 0; c < n_ch; ++c)
    if (!(lambdas[c] > 0) || !std::isfinite(lambdas[c])) return fail(HPT_EINVAL, "bad wavelength");
  for (uint32_t p = 0; p < n_planes; ++p)
    if (!std::isfinite(distances[p])) return fail(HPT_EINVAL, "bad distance");
  if (flags & ~HPT_ASM_BAND_LIMIT) return fail(HPT_EINVAL, "unknown flags");
  const uint32_t px = asm_padded(width), py = asm_padded(height);
  // scratch per frame of a chunk: row spectra (kept over the planes) and two work buffers
  const uint64_t per = 3ull * height * px * sizeof(float2);
  const size_t tw_bytes = (size_t)(px + py) * sizeof(float2);
  float2 *A = nullptr, *B = nullptr, *B0 = nullptr, *W = nullptr;
  uint32_t chunk = 0;
  size_t third = 0;
  {
    std::lock_guard<std::mutex> g(C->mu);
    (void)hipSetDevice(C->device);
    uint64_t free_b = C->budget > C->used ? C->budget - C->used : 0;
    if (free_b < per + tw_bytes) evict_grfs(C, per + tw_bytes);
    free_b = C->budget > C->used ? C->budget - C->used : 0;
    free_b = free_b > tw_bytes ? free_b - tw_bytes : 0;
    chunk = (uint32_t)std::min<uint64_t>({(uint64_t)T, free_b / per, std::max<uint64_t>(1, (1ull << 30) / per),
                                           (uint64_t)kMaxFieldsPerLaunch});
    if (chunk == 0) return fail(HPT_EBUDGET, "reconstruction scratch does not fit the budget");
    third = (size_t)chunk * height * px * sizeof(float2);
    bool ok = C->alloc((void **)&A, third) == hipSuccess;
    ok = ok && C->alloc((void **)&B, third) == hipSuccess;
    ok = ok && C->alloc((void **)&B0, third) == hipSuccess;
    ok = ok && C->alloc((void **)&W, tw_bytes) == hipSuccess;
    if (!ok) {
      if (A) C->release(A, third);
      if (B) C->release(B, third);
      if (B0) C->release(B0, third);
      if (W) C->release(W, tw_bytes);
      return fail(HPT_ENOMEM, "scratch allocation failed");
    }
  }
  hipError_t e = after_caller(C->aux, hip_stream);
  if (e == hipSuccess) e = launch_asm_twiddles(W, width, height, C->aux);
  const size_t field = (size_t)width * height;
  const float weight = 1.0f / (float)T;
  for (uint32_t c = 0; c < n_ch && e == hipSuccess; ++c) {
    for (uint32_t t0 = 0; t0 < T && e == hipSuccess; t0 += chunk) {
      const uint32_t nf = std::min(chunk, T - t0);
      e = launch_asm_spectra((const float2 *)d_fields + ((size_t)c * T + t0) * field, A, B0, W, nf, width, height,
                             C->aux);
      for (uint32_t p = 0; p < n_planes && e == hipSuccess; ++p) {
        const AsmParams P = asm_params(width, height, pitch, lambdas[c], distances[p], flags, na);
        float *I = (float *)d_out + ((size_t)c * n_planes + p) * field;
        e = launch_asm_intensity(B0, B, A, W, nf, width, height, P, I, weight, t0 > 0, C->aux);
      }
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(C->aux);
  else (void)hipStreamSynchronize(C->aux);  // launches already queued still use the scratch
  {
    std::lock_guard<std::mutex> g(C->mu);
    C->release(A, third);
    C->release(B, third);
    C->release(B0, third);
    C->release(W, tw_bytes);
  }
  if (e != hipSuccess) return fail(HPT_EDEVICE, std::string("reconstruction failed: ") + hipGetErrorString(e));
  return HPT_OK;
}

}  // extern "C"
