// Continuous-batching serving engine of libltrk.
//
// Tracking jobs of different sizes, schemes and precisions are admitted into
// slots while others run. Admission is by footprint: every job's state and
// moment rows live in one device arena (allocated once at create) managed by
// a first-fit free list; a job that does not fit now gets LTRK_EAGAIN and is
// retried by the caller after retirements free space. A step is one tiled
// kernel launch over all active jobs (each advancing by min(k, turns left)
// with its own scheme and precision) plus one finalize launch writing each
// job's moment rows. Two steps may be in flight; host tables for a step are
// staged in pinned double buffers.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace ltrk {
namespace {

// 8 particles per lane: one mixed launch runs FP64 and FP32 + Kahan tiles of
// every scheme, and at 16 the FP32 + Kahan Ruth4 tile alone takes 256 VGPRs
// (its single-bunch kernel ran 35% slower at 16 than at 8); single-bunch and
// batched FP64 calls use 16 where it pays.
constexpr int kEnginePpl = 8;
constexpr int kEngineBlock = 256;
constexpr int kDepth = 2;  // steps in flight

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// First-fit allocator over [0, size) of the arena, 256-byte granules.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    size_ = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t free_bytes() const {
    size_t s = 0;
    for (auto& kv : free_) s += kv.second;
    return s;
  }
  size_t largest() const {
    size_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }
  size_t size() const { return size_; }

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0;
};

struct Slot {
  bool used = false;
  bool cancelled = false;
  int64_t n = 0, turns = 0, done_turns = 0;
  int integrator = 0, dtype = 0;
  size_t off = 0, bytes = 0;
  void* z = nullptr;
  void* dp = nullptr;
  void* zc = nullptr;
  void* dc = nullptr;
  ltrk_moments* mom = nullptr;
  double* centre = nullptr;  // centre of the job's moment sums (k_centre at admission)
  Coeffs c;
  int64_t waves = 0;
  hipEvent_t last = nullptr;  // recorded after the slot's latest enqueued work
};

// State, moment rows and the centre of the moment sums, each 256-B aligned.
int64_t footprint(int64_t n, int64_t turns) {
  return static_cast<int64_t>(round_up(static_cast<size_t>(n) * 16, 256) +
                              round_up(static_cast<size_t>(turns) * sizeof(ltrk_moments), 256) +
                              kCentreDoubles * sizeof(double));
}

int validate_job(const ltrk_job* j) {
  if (!j) return fail(LTRK_EINVAL, "job is NULL");
  if (j->n < 1) return fail(LTRK_EINVAL, "job n must be >= 1");
  if (j->turns < 1 || j->turns > INT32_MAX) return fail(LTRK_EINVAL, "job turns out of range");
  if (!valid_integrator(j->integrator)) return fail(LTRK_EINVAL, "unknown integrator");
  if (!valid_dtype(j->dtype)) return fail(LTRK_EINVAL, "unknown dtype");
  int rc = validate_ring(&j->ring);
  if (rc) return rc;
  if (!j->z0 || !j->dp0) return fail(LTRK_EINVAL, "job initial state is NULL");
  if (j->dtype == LTRK_F32C && (!j->z0_comp || !j->dp0_comp))
    return fail(LTRK_EINVAL, "F32C job needs compensation arrays");
  return LTRK_OK;
}

}  // namespace
}  // namespace ltrk

using namespace ltrk;

struct ltrk_engine {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t copy = nullptr;  // step-table uploads, ahead of the steps that read them
  char* arena_base = nullptr;
  Arena arena;
  std::vector<Slot> slots;
  double* partials = nullptr;
  size_t partial_bytes = 0;
  // per-step tables, double buffered
  size_t cap_b = 0, cap_t = 0;
  BunchDev* h_b[kDepth] = {nullptr, nullptr};
  TileDev* h_t[kDepth] = {nullptr, nullptr};
  FinalizeDev* h_f[kDepth] = {nullptr, nullptr};
  BunchDev* d_b[kDepth] = {nullptr, nullptr};
  TileDev* d_t[kDepth] = {nullptr, nullptr};
  FinalizeDev* d_f[kDepth] = {nullptr, nullptr};
  hipEvent_t buf_ev[kDepth] = {nullptr, nullptr};
  hipEvent_t copy_ev[kDepth] = {nullptr, nullptr};
  bool buf_used[kDepth] = {false, false};
  int cur = 0;
  int64_t steps = 0;
  int64_t particle_turns = 0;
};

namespace {

int with_device(ltrk_engine* e) {
  hipError_t er = hipSetDevice(e->device);
  return er == hipSuccess ? LTRK_OK : fail_hip(er, "hipSetDevice");
}

void free_tables(ltrk_engine* e) {
  for (int i = 0; i < kDepth; ++i) {
    if (e->h_b[i]) hipHostFree(e->h_b[i]);
    if (e->h_t[i]) hipHostFree(e->h_t[i]);
    if (e->h_f[i]) hipHostFree(e->h_f[i]);
    if (e->d_b[i]) hipFree(e->d_b[i]);
    if (e->d_t[i]) hipFree(e->d_t[i]);
    if (e->d_f[i]) hipFree(e->d_f[i]);
    e->h_b[i] = nullptr;
    e->h_t[i] = nullptr;
    e->h_f[i] = nullptr;
    e->d_b[i] = nullptr;
    e->d_t[i] = nullptr;
    e->d_f[i] = nullptr;
  }
}

// Grow table capacity (engine idle: callers synchronise first).
int ensure_tables(ltrk_engine* e, size_t nb, size_t nt) {
  if (nb <= e->cap_b && nt <= e->cap_t && e->h_b[0]) return LTRK_OK;
  hipError_t er = hipStreamSynchronize(e->stream);
  if (er == hipSuccess && e->copy) er = hipStreamSynchronize(e->copy);
  if (er != hipSuccess) return fail_hip(er, "engine synchronise");
  free_tables(e);
  const size_t cb = std::max<size_t>(nb, e->slots.size());
  const size_t ct = std::max<size_t>(nt, 1024);
  for (int i = 0; i < kDepth; ++i) {
    if (hipHostMalloc(reinterpret_cast<void**>(&e->h_b[i]), cb * sizeof(BunchDev)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&e->h_t[i]), ct * sizeof(TileDev)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&e->h_f[i]), cb * sizeof(FinalizeDev)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&e->d_b[i]), cb * sizeof(BunchDev)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&e->d_t[i]), ct * sizeof(TileDev)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&e->d_f[i]), cb * sizeof(FinalizeDev)) != hipSuccess) {
      (void)hipGetLastError();
      free_tables(e);
      e->cap_b = e->cap_t = 0;
      return fail(LTRK_ENOMEM, "engine step tables");
    }
    e->buf_used[i] = false;
  }
  e->cap_b = cb;
  e->cap_t = ct;
  return LTRK_OK;
}

Slot* slot_at(ltrk_engine* e, int slot) {
  if (!e || slot < 0 || slot >= static_cast<int>(e->slots.size())) return nullptr;
  Slot* s = &e->slots[slot];
  return s->used ? s : nullptr;
}

int engine_step(ltrk_engine* e, int k, hipStream_t user, int64_t* advanced) {
  if (advanced) *advanced = 0;
  if (k < 1 || k > 4096) return fail(LTRK_EINVAL, "k must be in [1, 4096]");
  int rc = with_device(e);
  if (rc) return rc;
  std::vector<int> act;
  int64_t cols_total = 0, max_groups = 1;
  for (int i = 0; i < static_cast<int>(e->slots.size()); ++i) {
    const Slot& s = e->slots[i];
    if (s.used && !s.cancelled && s.done_turns < s.turns) {
      act.push_back(i);
      cols_total += scratch_cols(s.waves);
      max_groups = std::max(max_groups, finalize_groups(s.waves));
    }
  }
  if (act.empty()) return LTRK_OK;
  // Heaviest tiles first (the launch's blocks are dispatched in tile order,
  // so the cheap ones fill in behind and the launch ends on short blocks):
  // jobs by per-particle-turn cost, a scheme's flops, F32C about 1.4 times
  // FP64 (FP32/FP64 conversions and Kahan additions; measured 1.25-1.45 over
  // the schemes); a job's tiles stay together. The results do not depend on
  // the order.
  auto unit_cost = [&](int i) {
    const Slot& s = e->slots[i];
    static const double flops[4] = {30.0, 32.0, 76.0, 112.0};
    const double f = s.integrator >= 0 && s.integrator < 4 ? flops[s.integrator] : 32.0;
    return f * (s.dtype == LTRK_F32C ? 1.4 : 1.0);
  };
  std::stable_sort(act.begin(), act.end(),
                   [&](int a, int b) { return unit_cost(a) > unit_cost(b); });
  // turns this step: bounded by the partial-sum scratch
  int64_t kcap = static_cast<int64_t>(e->partial_bytes / (sizeof(double) * 5)) /
                 std::max<int64_t>(cols_total, 1);
  if (kcap < 1) return fail(LTRK_ENOMEM, "engine partial scratch too small for active jobs");
  const int64_t kk = std::min<int64_t>(k, kcap);
  size_t ntiles = 0;
  const int wpb = kEngineBlock / kWave;
  for (int i : act) ntiles += static_cast<size_t>((e->slots[i].waves + wpb - 1) / wpb);
  if ((rc = ensure_tables(e, act.size(), ntiles))) return rc;

  hipError_t er;
  if (user) {
    hipEvent_t dep = nullptr;
    if (hipEventCreateWithFlags(&dep, hipEventDisableTiming) == hipSuccess) {
      hipEventRecord(dep, user);
      hipStreamWaitEvent(e->stream, dep, 0);
      hipEventDestroy(dep);
    }
  }
  const int b = e->cur;
  if (e->buf_used[b]) {
    er = hipEventSynchronize(e->buf_ev[b]);
    if (er != hipSuccess) return fail_hip(er, "engine step wait");
  }
  BunchDev* hb = e->h_b[b];
  TileDev* ht = e->h_t[b];
  FinalizeDev* hf = e->h_f[b];
  size_t t = 0, off = 0;
  int32_t max_rows = 0;
  int64_t pt = 0;
  for (size_t j = 0; j < act.size(); ++j) {
    Slot& s = e->slots[act[j]];
    const int64_t rows = std::min<int64_t>(kk, s.turns - s.done_turns);
    BunchDev& d = hb[j];
    std::memset(&d, 0, sizeof(d));
    d.z = s.z;
    d.dp = s.dp;
    d.z_comp = s.zc;
    d.dp_comp = s.dc;
    d.n = s.n;
    d.waves = s.waves;
    d.partials = e->partials + off;
    d.centre = s.centre;
    d.c = s.c;
    d.integrator = s.integrator;
    d.dtype = s.dtype;
    d.turns = static_cast<int32_t>(rows);
    d.active = 1;
    FinalizeDev& f = hf[j];
    std::memset(&f, 0, sizeof(f));
    f.partials = d.partials;
    f.stage = d.partials + rows * 5 * s.waves;
    f.waves = s.waves;
    f.groups = finalize_groups(s.waves);
    f.n = s.n;
    f.out = s.mom + s.done_turns;
    f.centre = s.centre;
    f.rows = static_cast<int32_t>(rows);
    off += static_cast<size_t>(rows) * 5 * scratch_cols(s.waves);
    max_rows = std::max<int32_t>(max_rows, static_cast<int32_t>(rows));
    for (int64_t w0 = 0; w0 < s.waves; w0 += wpb) ht[t++] = TileDev{static_cast<int32_t>(j), static_cast<int32_t>(w0)};
    pt += s.n * rows;
  }
  const int nb = static_cast<int>(act.size());
  // The uploads run on the copy stream while the previous steps compute (the
  // buffers were last read by the step two back, which buf_ev[b] waited for)
  if ((er = hipMemcpyAsync(e->d_b[b], hb, nb * sizeof(BunchDev), hipMemcpyHostToDevice, e->copy)) != hipSuccess ||
      (er = hipMemcpyAsync(e->d_t[b], ht, t * sizeof(TileDev), hipMemcpyHostToDevice, e->copy)) != hipSuccess ||
      (er = hipMemcpyAsync(e->d_f[b], hf, nb * sizeof(FinalizeDev), hipMemcpyHostToDevice, e->copy)) != hipSuccess ||
      (er = hipEventRecord(e->copy_ev[b], e->copy)) != hipSuccess ||
      (er = hipStreamWaitEvent(e->stream, e->copy_ev[b], 0)) != hipSuccess)
    return fail_hip(er, "engine table upload");
  void* tok = nullptr;
  timing_begin(e->stream, kTimeTrack, &tok);
  er = launch_track_mixed(e->d_b[b], e->d_t[b], static_cast<int64_t>(t), kEnginePpl, kEngineBlock, e->stream);
  timing_end(e->stream, tok);
  if (er != hipSuccess) return fail_hip(er, "engine track launch");
  timing_begin(e->stream, kTimeFinalize, &tok);
  er = launch_finalize_multi(e->d_f[b], nb, max_rows, 0, max_groups, e->stream);
  timing_end(e->stream, tok);
  if (er != hipSuccess) return fail_hip(er, "engine finalize launch");
  hipEventRecord(e->buf_ev[b], e->stream);
  e->buf_used[b] = true;
  e->cur = (b + 1) % kDepth;
  for (int i : act) {
    Slot& s = e->slots[i];
    s.done_turns += std::min<int64_t>(kk, s.turns - s.done_turns);
    hipEventRecord(s.last, e->stream);
  }
  if (user) {
    hipEvent_t dep = nullptr;
    if (hipEventCreateWithFlags(&dep, hipEventDisableTiming) == hipSuccess) {
      hipEventRecord(dep, e->stream);
      hipStreamWaitEvent(user, dep, 0);
      hipEventDestroy(dep);
    }
  }
  e->steps++;
  e->particle_turns += pt;
  if (advanced) *advanced = pt;
  return LTRK_OK;
}

void engine_free(ltrk_engine* e) {
  if (!e) return;
  hipSetDevice(e->device);
  if (e->stream) hipStreamSynchronize(e->stream);
  if (e->copy) hipStreamSynchronize(e->copy);
  free_tables(e);
  for (Slot& s : e->slots)
    if (s.last) hipEventDestroy(s.last);
  for (int i = 0; i < kDepth; ++i) {
    if (e->buf_ev[i]) hipEventDestroy(e->buf_ev[i]);
    if (e->copy_ev[i]) hipEventDestroy(e->copy_ev[i]);
  }
  if (e->partials) hipFree(e->partials);
  if (e->arena_base) hipFree(e->arena_base);
  if (e->stream) hipStreamDestroy(e->stream);
  if (e->copy) hipStreamDestroy(e->copy);
  delete e;
}

}  // namespace

#define ENGINE_GUARD(body)                                   \
  try {                                                      \
    clear_error();                                           \
    body                                                     \
  } catch (const std::bad_alloc&) {                          \
    return fail(LTRK_ENOMEM, "host allocation failed");      \
  } catch (...) {                                            \
    return fail(LTRK_EDEVICE, "unexpected internal error");  \
  }

extern "C" {

int ltrk_engine_create(int device, int64_t hbm_budget_bytes, int max_slots, ltrk_engine** out) {
  ENGINE_GUARD({
    if (!out) return fail(LTRK_EINVAL, "out is NULL");
    *out = nullptr;
    if (hbm_budget_bytes < 4096) return fail(LTRK_EINVAL, "budget must be >= 4096 bytes");
    if (max_slots < 1 || max_slots > 65535) return fail(LTRK_EINVAL, "max_slots out of range");
    int ndev = 0;
    hipError_t er = hipGetDeviceCount(&ndev);
    if (er != hipSuccess) return fail_hip(er, "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(LTRK_EINVAL, "no device %d", device);
    ltrk_engine* e = new ltrk_engine;
    e->device = device;
    int rc = LTRK_OK;
    if ((er = hipSetDevice(device)) != hipSuccess ||
        (er = hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking)) != hipSuccess ||
        (er = hipStreamCreateWithFlags(&e->copy, hipStreamNonBlocking)) != hipSuccess) {
      rc = fail_hip(er, "engine stream");
    }
    const size_t arena = round_up(static_cast<size_t>(hbm_budget_bytes), 256);
    if (rc == LTRK_OK && hipMalloc(reinterpret_cast<void**>(&e->arena_base), arena) != hipSuccess) {
      (void)hipGetLastError();
      rc = fail(LTRK_ENOMEM, "engine arena of %zu bytes", arena);
    }
    if (rc == LTRK_OK) {
      // 1 GiB (of 288 GB): a step advances every active job by min(k, what
      // the scratch holds) turns, so a larger scratch means fewer, longer
      // steps (measured at 300 requests: 256 MiB 6.6e11, 1 GiB 7.0e11
      // particle-turns/s, the GPU busy 94% and 98% of the run)
      const char* env = std::getenv("LTRK_ENGINE_PARTIALS_MB");
      long mb = env ? std::atol(env) : 1024;
      if (mb < 1) mb = 1;
      e->partial_bytes = static_cast<size_t>(mb) << 20;
      if (hipMalloc(reinterpret_cast<void**>(&e->partials), e->partial_bytes) != hipSuccess) {
        (void)hipGetLastError();
        rc = fail(LTRK_ENOMEM, "engine partial scratch");
      }
    }
    if (rc == LTRK_OK) {
      e->arena.reset(arena);
      e->slots.resize(static_cast<size_t>(max_slots));
      for (Slot& s : e->slots)
        if (hipEventCreateWithFlags(&s.last, hipEventDisableTiming) != hipSuccess) rc = fail(LTRK_EDEVICE, "engine events");
      for (int i = 0; i < kDepth && rc == LTRK_OK; ++i)
        if (hipEventCreateWithFlags(&e->buf_ev[i], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&e->copy_ev[i], hipEventDisableTiming) != hipSuccess)
          rc = fail(LTRK_EDEVICE, "engine events");
    }
    if (rc != LTRK_OK) {
      engine_free(e);
      return rc;
    }
    *out = e;
    return LTRK_OK;
  })
}

int ltrk_engine_footprint(const ltrk_job* job, int64_t* bytes) {
  ENGINE_GUARD({
    if (!job || !bytes) return fail(LTRK_EINVAL, "NULL argument");
    if (job->n < 0 || job->turns < 0) return fail(LTRK_EINVAL, "negative size");
    *bytes = footprint(job->n, job->turns);
    return LTRK_OK;
  })
}

int ltrk_engine_admit(ltrk_engine* e, const ltrk_job* job, int* slot) {
  ENGINE_GUARD({
    if (!e || !slot) return fail(LTRK_EINVAL, "NULL argument");
    *slot = -1;
    int rc = validate_job(job);
    if (rc) return rc;
    const size_t need = static_cast<size_t>(footprint(job->n, job->turns));
    if (need > e->arena.size()) return fail(LTRK_EINVAL, "job footprint %zu exceeds the arena", need);
    int free_slot = -1;
    for (int i = 0; i < static_cast<int>(e->slots.size()); ++i)
      if (!e->slots[i].used) {
        free_slot = i;
        break;
      }
    if (free_slot < 0) return fail(LTRK_EAGAIN, "no free slot");
    // A step needs one row of moment partials per active job in the partial
    // scratch (it then advances them by as many turns as the scratch holds),
    // so the jobs that are still running must fit in it together.
    const int64_t cap_cols = static_cast<int64_t>(e->partial_bytes / (5 * sizeof(double)));
    const int64_t cols = scratch_cols(waves_for(job->n, kEnginePpl));
    if (cols > cap_cols)
      return fail(LTRK_EINVAL, "job needs %lld moment-partial columns, the engine holds %lld "
                  "(LTRK_ENGINE_PARTIALS_MB)", (long long)cols, (long long)cap_cols);
    int64_t cols_running = 0;
    for (const Slot& o : e->slots)
      if (o.used && !o.cancelled && o.done_turns < o.turns) cols_running += scratch_cols(o.waves);
    if (cols_running + cols > cap_cols)
      return fail(LTRK_EAGAIN, "moment-partial scratch taken by running jobs");
    size_t off = 0;
    if (!e->arena.alloc(need, &off)) return fail(LTRK_EAGAIN, "arena has no free block of %zu bytes", need);
    if ((rc = with_device(e))) {
      e->arena.release(off, need);
      return rc;
    }
    Slot& s = e->slots[free_slot];
    s.used = true;
    s.cancelled = false;
    s.n = job->n;
    s.turns = job->turns;
    s.done_turns = 0;
    s.integrator = job->integrator;
    s.dtype = job->dtype;
    s.off = off;
    s.bytes = need;
    s.waves = waves_for(job->n, kEnginePpl);
    make_coeffs(job->ring, job->integrator, &s.c);
    char* base = e->arena_base + off;
    const size_t n = static_cast<size_t>(job->n);
    const size_t elem = job->dtype == LTRK_F64 ? 8 : 4;
    s.z = base;
    s.dp = base + n * elem;
    s.zc = job->dtype == LTRK_F32C ? base + 2 * n * elem : nullptr;
    s.dc = job->dtype == LTRK_F32C ? base + 3 * n * elem : nullptr;
    s.mom = reinterpret_cast<ltrk_moments*>(base + round_up(n * 16, 256));
    s.centre = reinterpret_cast<double*>(
        base + round_up(n * 16, 256) +
        round_up(static_cast<size_t>(job->turns) * sizeof(ltrk_moments), 256));
    // Synchronous copies: the caller's host arrays are free to go once admit
    // returns. The arena block is idle (its previous job was retired after
    // its last step completed), so no ordering with the engine stream is needed.
    hipError_t er;
    if ((er = hipMemcpy(s.z, job->z0, n * elem, hipMemcpyHostToDevice)) != hipSuccess ||
        (er = hipMemcpy(s.dp, job->dp0, n * elem, hipMemcpyHostToDevice)) != hipSuccess ||
        (job->dtype == LTRK_F32C &&
         ((er = hipMemcpy(s.zc, job->z0_comp, n * elem, hipMemcpyHostToDevice)) != hipSuccess ||
          (er = hipMemcpy(s.dc, job->dp0_comp, n * elem, hipMemcpyHostToDevice)) != hipSuccess))) {
      s.used = false;
      e->arena.release(off, need);
      return fail_hip(er, "job upload");
    }
    // the centre of the job's moment sums, from its initial state, as a
    // standalone call computes it (the same kernel and sample)
    if ((er = launch_centre(CentreDev{s.z, s.dp, s.zc, s.dc, s.n, s.dtype, s.centre},
                            e->stream)) != hipSuccess) {
      s.used = false;
      e->arena.release(off, need);
      return fail_hip(er, "job centre");
    }
    hipEventRecord(s.last, e->stream);
    *slot = free_slot;
    return LTRK_OK;
  })
}

int ltrk_engine_step(ltrk_engine* e, int k, void* stream, int64_t* advanced) {
  ENGINE_GUARD({
    if (!e) return fail(LTRK_EINVAL, "engine is NULL");
    return engine_step(e, k, static_cast<hipStream_t>(stream), advanced);
  })
}

int ltrk_engine_poll(ltrk_engine* e, int slot, int* done) {
  ENGINE_GUARD({
    Slot* s = slot_at(e, slot);
    if (!s || !done) return fail(LTRK_EINVAL, "invalid slot");
    *done = 0;
    if (s->done_turns < s->turns && !s->cancelled) return LTRK_OK;
    hipError_t er = hipEventQuery(s->last);
    if (er == hipSuccess) {
      *done = 1;
      return LTRK_OK;
    }
    if (er == hipErrorNotReady) {
      (void)hipGetLastError();
      return LTRK_OK;
    }
    return fail_hip(er, "engine poll");
  })
}

int ltrk_engine_result(ltrk_engine* e, int slot, void* z, void* dp, void* z_comp, void* dp_comp,
                       ltrk_moments* moments) {
  ENGINE_GUARD({
    Slot* s = slot_at(e, slot);
    if (!s) return fail(LTRK_EINVAL, "invalid slot");
    int rc = with_device(e);
    if (rc) return rc;
    const size_t n = static_cast<size_t>(s->n);
    const size_t elem = s->dtype == LTRK_F64 ? 8 : 4;
    hipError_t er = hipEventSynchronize(s->last);
    if (er != hipSuccess) return fail_hip(er, "engine result wait");
    if ((z && (er = hipMemcpy(z, s->z, n * elem, hipMemcpyDeviceToHost)) != hipSuccess) ||
        (dp && (er = hipMemcpy(dp, s->dp, n * elem, hipMemcpyDeviceToHost)) != hipSuccess) ||
        (s->dtype == LTRK_F32C && z_comp &&
         (er = hipMemcpy(z_comp, s->zc, n * elem, hipMemcpyDeviceToHost)) != hipSuccess) ||
        (s->dtype == LTRK_F32C && dp_comp &&
         (er = hipMemcpy(dp_comp, s->dc, n * elem, hipMemcpyDeviceToHost)) != hipSuccess) ||
        (moments && (er = hipMemcpy(moments, s->mom, static_cast<size_t>(s->done_turns) * sizeof(ltrk_moments),
                                    hipMemcpyDeviceToHost)) != hipSuccess))
      return fail_hip(er, "engine result copy");
    return LTRK_OK;
  })
}

int ltrk_engine_retire(ltrk_engine* e, int slot) {
  ENGINE_GUARD({
    Slot* s = slot_at(e, slot);
    if (!s) return fail(LTRK_EINVAL, "invalid slot");
    int rc = with_device(e);
    if (rc) return rc;
    hipError_t er = hipEventSynchronize(s->last);  // its arena block may still be in use
    if (er != hipSuccess) return fail_hip(er, "engine retire wait");
    e->arena.release(s->off, s->bytes);
    s->used = false;
    s->cancelled = false;
    return LTRK_OK;
  })
}

int ltrk_engine_cancel(ltrk_engine* e, int slot) {
  ENGINE_GUARD({
    Slot* s = slot_at(e, slot);
    if (!s) return fail(LTRK_EINVAL, "invalid slot");
    s->cancelled = true;
    return LTRK_OK;
  })
}

int ltrk_engine_stats_get(ltrk_engine* e, ltrk_engine_stats* out) {
  ENGINE_GUARD({
    if (!e || !out) return fail(LTRK_EINVAL, "NULL argument");
    int act = 0;
    for (const Slot& s : e->slots) act += s.used ? 1 : 0;
    out->active_slots = act;
    out->max_slots = static_cast<int32_t>(e->slots.size());
    out->arena_bytes = static_cast<int64_t>(e->arena.size());
    out->arena_free_bytes = static_cast<int64_t>(e->arena.free_bytes());
    out->largest_free_block = static_cast<int64_t>(e->arena.largest());
    out->steps = e->steps;
    out->particle_turns = e->particle_turns;
    return LTRK_OK;
  })
}

int ltrk_engine_destroy(ltrk_engine* e) {
  ENGINE_GUARD({
    engine_free(e);
    return LTRK_OK;
  })
}

}  // extern "C"
