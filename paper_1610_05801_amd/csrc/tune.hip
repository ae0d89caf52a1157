// Launch plans for libltrk: a process-wide forced plan, a tuning cache filled
// by the project's own autotuner (times candidate plans on scratch particles
// with HIP events), and a built-in default.
//
// A plan is (K turns per launch, block size, particles per lane P, graph
// replay). P changes the order of the moment sums (lane-local over P
// particles), so results are bit-identical across plans with the same P and
// agree to rounding across different P.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"
#include "kernels.h"

extern "C" int ltrk_track_f64(double*, double*, int64_t, int64_t, const ltrk_ring*, int,
                              ltrk_moments*, void*);
extern "C" int ltrk_track_f32c(float*, float*, float*, float*, int64_t, int64_t,
                               const ltrk_ring*, int, ltrk_moments*, void*);
extern "C" int ltrk_track_batched(const ltrk_bunch*, int, int64_t, int, int, void*);

namespace ltrk {

namespace {

using TuneKey = std::tuple<std::string, int, int, int, int>;  // arch, integ, dtype, log2 n, batched

std::mutex g_plan_mu;
bool g_forced = false;
ltrk_plan g_forced_plan{128, 256, 4, 1};
std::map<TuneKey, ltrk_plan> g_tuned;

bool plan_valid(const ltrk_plan& p) {
  const bool k_ok = p.turns_per_launch >= 1 && p.turns_per_launch <= 65536;
  const bool b_ok = p.block == 64 || p.block == 128 || p.block == 256;
  const bool p_ok = p.ppl == 1 || p.ppl == 2 || p.ppl == 4 || p.ppl == 8 || p.ppl == 16;
  return k_ok && b_ok && p_ok && (p.use_graph == 0 || p.use_graph == 1);
}

// Architecture name of the current device (cached per device: the property
// query costs more than the rest of a call's host work).
std::string device_arch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown";
  }
  static std::mutex mu;
  static std::map<int, std::string> cache;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown";
  }
  std::string a(prop.gcnArchName);
  const size_t colon = a.find(':');
  a = colon == std::string::npos ? a : a.substr(0, colon);
  cache[dev] = a;
  return a;
}

int log2_bucket(int64_t n) {
  int b = 0;
  while (n > 1) {
    n >>= 1;
    ++b;
  }
  return b;
}

}  // namespace

// Wave slots of the single-bunch kernels on the device (256 CUs x 4 SIMDs x
// 2 waves) and the relative cost of a particle at 16 per lane against 8.
constexpr int64_t kWaveSlots = 2048;
constexpr double kCostPerSlot16 = 0.93;

ltrk_plan default_plan(int integrator, int dtype, int64_t n, bool /*batched*/) {
  ltrk_plan p;
  // 1024 turns per launch: 1.2-1.6% over 512 at 1e6 particles (fewer launch
  // boundaries), while a launch's moment partials (80 MB at 1e6 particles)
  // still fit the 256 MB last-level cache; 5000 or more turns were slower.
  p.turns_per_launch = 1024;
  p.block = 256;
  p.use_graph = 1;
  // More particles per lane give more independent FP64 chains per lane and
  // spread the per-turn moment reduction over more particles; use them while
  // the wave tiles still cover the 1024 SIMDs about 1.5 times (measured at
  // 1e6 particles: P = 8 beats P = 4 by ~15%).
  if (waves_for(n, 8) >= 1536)
    p.ppl = 8;
  else if (waves_for(n, 4) >= 2048)
    p.ppl = 4;
  else if (waves_for(n, 2) >= 2048)
    p.ppl = 2;
  else
    p.ppl = 1;
  // 16 particles per lane (a batched call counts the waves of all its
  // bunches) halve the per-particle share of the moment reduction and of the
  // partials, and still run two waves per SIMD; a lane's particles cost ~7%
  // less than at 8 (FP64: 1.57e12 against 1.49e12 at 1e7 particles, 1.59e12
  // against 1.46e12 at 4e7; F32C leap-frog 1.066e12 against 1.003e12 at 1e7).
  // The kernels hold two waves per SIMD (the LDS rows, and ~230 VGPRs at 16
  // for FP64, 250 for F32C Euler-Cromer and leap-frog), so waves run in rounds
  // of kWaveSlots and a launch lasts ceil(waves / kWaveSlots) rounds of P
  // particles each: 16 is taken where that costs less (2e6, 4e6 and from 6e6
  // particles on; not at 1e6, where it would leave one wave per SIMD: 1.25e12
  // against 1.43e12, nor at 3e6 or 5e6, where the last round would be a small
  // one). Not for F32C Ruth4 and RK4: the single-bunch Ruth4 kernel needs more
  // than 256 registers at 16 (one wave per SIMD; measured 35% slower at 1e7),
  // and RK4 gains nothing (+0.5% at 1e7, within noise; Euler-Cromer +5.5%).
  const bool sixteen = dtype == LTRK_F64 || integrator == LTRK_EULER_CROMER ||
                       integrator == LTRK_LEAPFROG;
  if (sixteen && p.ppl == 8) {
    auto rounds = [&](int ppl) { return (waves_for(n, ppl) + kWaveSlots - 1) / kWaveSlots; };
    if (static_cast<double>(rounds(16)) * 16.0 * kCostPerSlot16 <
        static_cast<double>(rounds(8)) * 8.0)
      p.ppl = 16;
  }
  if (waves_for(n, p.ppl) < 1024) p.block = 64;
  return p;
}

ltrk_plan choose_plan(int integrator, int dtype, int64_t n, bool batched, bool* is_default) {
  std::lock_guard<std::mutex> g(g_plan_mu);
  if (is_default) *is_default = false;
  if (g_forced) return g_forced_plan;
  auto it = g_tuned.find(TuneKey(device_arch(), integrator, dtype, log2_bucket(n), batched));
  if (it != g_tuned.end()) return it->second;
  if (is_default) *is_default = true;
  return default_plan(integrator, dtype, n, batched);
}

// A launch writes one row of moment partials per turn, which the finalize
// reads after the launch; the default plan keeps a launch's rows within
// 192 MiB, so they are still in the 256 MB last-level cache then. Measured
// (leap-frog, 8 particles per lane): 1e6 particles (78 KB per row) best at
// 1024-2048 turns, 4e6 (312 KB) at 512, 1e7 (781 KB) at 256 (+3.7% over
// 1024); the 6-D map at 1e6 (469 KB) at 256 (+7% over 1024). Largest power
// of two within the budget, at least 64, at most the plan's value.
int64_t default_turns_for_partials(int64_t turns_per_launch, int64_t bytes_per_row) {
  const int64_t budget = int64_t(192) << 20;
  int64_t k = 64;
  while (2 * k <= turns_per_launch && 2 * k * bytes_per_row <= budget) k *= 2;
  return std::min<int64_t>(turns_per_launch, std::max<int64_t>(k, 64));
}

namespace {

// Time one single-bunch call with plan p; returns milliseconds or < 0.
double time_call(int integrator, int dtype, int64_t n, int64_t turns, void* const* arrays,
                 ltrk_moments* mom, hipStream_t s, const ltrk_ring& ring, const ltrk_plan& p,
                 int* rc_out) {
  {
    std::lock_guard<std::mutex> g(g_plan_mu);
    g_forced = true;
    g_forced_plan = p;
  }
  auto call = [&]() {
    if (dtype == LTRK_F64)
      return ltrk_track_f64(static_cast<double*>(arrays[0]), static_cast<double*>(arrays[1]), n,
                            turns, &ring, integrator, mom, s);
    return ltrk_track_f32c(static_cast<float*>(arrays[0]), static_cast<float*>(arrays[1]),
                           static_cast<float*>(arrays[2]), static_cast<float*>(arrays[3]), n,
                           turns, &ring, integrator, mom, s);
  };
  double best = -1.0;
  int rc = call();  // warm-up (and graph capture)
  hipEvent_t a = nullptr, b = nullptr;
  if (rc == LTRK_OK && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess) {
    for (int rep = 0; rep < 2 && rc == LTRK_OK; ++rep) {
      hipEventRecord(a, s);
      rc = call();
      hipEventRecord(b, s);
      if (hipEventSynchronize(b) != hipSuccess) {
        rc = fail(LTRK_EDEVICE, "autotune: event synchronisation failed");
        break;
      }
      float ms = 0.0f;
      hipEventElapsedTime(&ms, a, b);
      if (rc == LTRK_OK && (best < 0.0 || ms < best)) best = ms;
    }
  }
  if (a) hipEventDestroy(a);
  if (b) hipEventDestroy(b);
  *rc_out = rc;
  return rc == LTRK_OK ? best : -1.0;
}

int autotune(int integrator, int dtype, int64_t n, hipStream_t s, ltrk_plan* best_out) {
  if (!valid_integrator(integrator)) return fail(LTRK_EINVAL, "unknown integrator %d", integrator);
  if (!valid_dtype(dtype)) return fail(LTRK_EINVAL, "unknown dtype %d", dtype);
  if (n < 1 || n > (int64_t(1) << 34)) return fail(LTRK_EINVAL, "n out of range for tuning");
  // Work per probe call ~2^29 particle-turns (a few ms at full rate).
  int64_t turns = (int64_t(1) << 29) / n;
  turns = turns < 64 ? 64 : (turns > 4096 ? 4096 : turns);
  const size_t elem = dtype == LTRK_F64 ? 8 : 4;
  const int narr = dtype == LTRK_F64 ? 2 : 4;
  void* arrays[4] = {nullptr, nullptr, nullptr, nullptr};
  ltrk_moments* mom = nullptr;
  int rc = LTRK_OK;
  for (int i = 0; i < narr && rc == LTRK_OK; ++i)
    if (hipMalloc(&arrays[i], static_cast<size_t>(n) * elem) != hipSuccess)
      rc = fail(LTRK_ENOMEM, "autotune state");
  if (rc == LTRK_OK &&
      hipMalloc(reinterpret_cast<void**>(&mom), static_cast<size_t>(4096) * sizeof(ltrk_moments)) !=
          hipSuccess)
    rc = fail(LTRK_ENOMEM, "autotune moments");
  if (rc == LTRK_OK) {
    if (dtype == LTRK_F64) {
      hipError_t e = launch_fill_probe(static_cast<double*>(arrays[0]),
                                       static_cast<double*>(arrays[1]), n, s);
      if (e != hipSuccess) rc = fail_hip(e, "autotune fill");
    } else {
      for (int i = 0; i < 4; ++i) hipMemsetAsync(arrays[i], 0, static_cast<size_t>(n) * elem, s);
    }
  }
  // Ring of the plain workload: 6911 m, h 4620, 2 MV, 26 GeV/c protons.
  const ltrk_ring ring{6911.0, 4620.0, 2.0e6, 26.0e9, 0.938e9, 22.77, 1.0};
  bool saved_forced;
  ltrk_plan saved_plan;
  {
    std::lock_guard<std::mutex> g(g_plan_mu);
    saved_forced = g_forced;
    saved_plan = g_forced_plan;
  }
  // Turns per launch, block and particles per lane searched jointly; every
  // probe call runs at least two launches of its plan.
  ltrk_plan best{128, 256, 4, 1};
  double best_rate = -1.0;
  const int ppls[5] = {1, 2, 4, 8, 16};
  const int n_ppls = 5;
  const int blocks[3] = {64, 128, 256};
  const int ks[6] = {32, 128, 256, 512, 1024, 2048};
  for (int ki = 0; ki < 6 && rc == LTRK_OK; ++ki) {
    const int64_t t = std::min<int64_t>(4096, std::max<int64_t>(turns, 2 * ks[ki]));
    for (int pi = 0; pi < n_ppls && rc == LTRK_OK; ++pi) {
      for (int bi = 0; bi < 3 && rc == LTRK_OK; ++bi) {
        const ltrk_plan p{ks[ki], blocks[bi], ppls[pi], 1};
        const double ms = time_call(integrator, dtype, n, t, arrays, mom, s, ring, p, &rc);
        if (ms > 0.0) {
          const double rate = static_cast<double>(n) * t / ms;
          if (rate > best_rate) {
            best_rate = rate;
            best = p;
          }
        }
      }
    }
  }
  {
    std::lock_guard<std::mutex> g(g_plan_mu);
    g_forced = saved_forced;
    g_forced_plan = saved_plan;
  }
  hipStreamSynchronize(s);
  for (void* p : arrays)
    if (p) hipFree(p);
  if (mom) hipFree(mom);
  if (rc != LTRK_OK) return rc;
  {
    std::lock_guard<std::mutex> g(g_plan_mu);
    g_tuned[TuneKey(device_arch(), integrator, dtype, log2_bucket(n), 0)] = best;
  }
  if (best_out) *best_out = best;
  return LTRK_OK;
}

// Milliseconds of one batched call of `turns` turns over `table` with plan p
// (best of two after a warm-up call that builds its launch graph), or < 0.
double time_batched(const std::vector<ltrk_bunch>& table, int64_t turns, int integrator,
                    int dtype, hipStream_t s, const ltrk_plan& p, int* rc_out) {
  {
    std::lock_guard<std::mutex> g(g_plan_mu);
    g_forced = true;
    g_forced_plan = p;
  }
  auto call = [&]() {
    return ltrk_track_batched(table.data(), static_cast<int>(table.size()), turns, integrator,
                              dtype, s);
  };
  double best = -1.0;
  int rc = call();
  hipEvent_t a = nullptr, b = nullptr;
  if (rc == LTRK_OK && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess) {
    for (int rep = 0; rep < 2 && rc == LTRK_OK; ++rep) {
      hipEventRecord(a, s);
      rc = call();
      hipEventRecord(b, s);
      if (hipEventSynchronize(b) != hipSuccess) {
        rc = fail(LTRK_EDEVICE, "autotune: event synchronisation failed");
        break;
      }
      float ms = 0.0f;
      hipEventElapsedTime(&ms, a, b);
      if (rc == LTRK_OK && (best < 0.0 || ms < best)) best = ms;
    }
  }
  if (a) hipEventDestroy(a);
  if (b) hipEventDestroy(b);
  *rc_out = rc;
  return rc == LTRK_OK ? best : -1.0;
}

// Tune the batched launch on probe bunches of the caller's sizes and rings
// (with moments where the caller's bunch has them): turns per launch, block
// and particles per lane searched jointly.
int autotune_batched(const ltrk_bunch* bunches, int nb, int integrator, int dtype, hipStream_t s,
                     ltrk_plan* best_out) {
  if (!valid_integrator(integrator)) return fail(LTRK_EINVAL, "unknown integrator %d", integrator);
  if (!valid_dtype(dtype)) return fail(LTRK_EINVAL, "unknown dtype %d", dtype);
  if (nb < 1 || nb > 65535 || !bunches) return fail(LTRK_EINVAL, "invalid bunch table");
  int64_t total = 0;
  int n_mom = 0;
  for (int i = 0; i < nb; ++i) {
    if (bunches[i].n < 0) return fail(LTRK_EINVAL, "bunch %d: n < 0", i);
    int rc = validate_ring(&bunches[i].ring);
    if (rc) return fail(rc, "bunch %d: invalid ring", i);
    total += bunches[i].n;
    n_mom += bunches[i].moments && bunches[i].n > 0 ? 1 : 0;
  }
  if (total < 1 || total > (int64_t(1) << 34))
    return fail(LTRK_EINVAL, "total particles out of range for tuning");
  // ~2^31 particle-turns per probe call, at least two launches of the plan
  const int64_t base_turns = std::max<int64_t>(64, std::min<int64_t>(4096, (int64_t(1) << 31) / total));
  const size_t elem = dtype == LTRK_F64 ? 8 : 4;
  const int narr = dtype == LTRK_F64 ? 2 : 4;
  const size_t state_bytes = static_cast<size_t>(total) * elem * narr;
  const size_t mom_bytes = static_cast<size_t>(n_mom) * 4096 * sizeof(ltrk_moments);
  char* buf = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&buf), state_bytes + mom_bytes + 256) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LTRK_ENOMEM, "autotune probe bunches");
  }
  std::vector<ltrk_bunch> table(nb);
  int rc = LTRK_OK;
  size_t off = 0;
  int mi = 0;
  char* mom_base = buf + ((state_bytes + 255) & ~size_t(255));
  for (int i = 0; i < nb && rc == LTRK_OK; ++i) {
    ltrk_bunch& t = table[i];
    std::memset(&t, 0, sizeof(t));
    const size_t bytes = static_cast<size_t>(bunches[i].n) * elem;
    void* arr[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int k = 0; k < narr; ++k) {
      arr[k] = bunches[i].n > 0 ? buf + off : nullptr;
      off += bytes;
    }
    t.z = arr[0];
    t.dp = arr[1];
    t.z_comp = arr[2];
    t.dp_comp = arr[3];
    t.n = bunches[i].n;
    t.ring = bunches[i].ring;
    if (bunches[i].moments && bunches[i].n > 0)
      t.moments = reinterpret_cast<ltrk_moments*>(mom_base) + static_cast<size_t>(mi++) * 4096;
    if (t.n > 0) {
      hipError_t e = hipSuccess;
      if (dtype == LTRK_F64)
        e = launch_fill_probe(static_cast<double*>(t.z), static_cast<double*>(t.dp), t.n, s);
      else
        for (int k = 0; k < 4 && e == hipSuccess; ++k) e = hipMemsetAsync(arr[k], 0, bytes, s);
      if (e != hipSuccess) rc = fail_hip(e, "autotune fill");
    }
  }
  bool saved_forced;
  ltrk_plan saved_plan;
  {
    std::lock_guard<std::mutex> g(g_plan_mu);
    saved_forced = g_forced;
    saved_plan = g_forced_plan;
  }
  ltrk_plan best{256, 256, 8, 1};
  double best_rate = -1.0;
  const int ppls[4] = {2, 4, 8, 16};
  const int n_ppls = 4;
  const int blocks[3] = {64, 128, 256};
  const int ks[4] = {128, 256, 512, 1024};
  for (int ki = 0; ki < 4 && rc == LTRK_OK; ++ki) {
    const int64_t turns = std::min<int64_t>(4096, std::max<int64_t>(base_turns, 2 * ks[ki]));
    for (int pi = 0; pi < n_ppls && rc == LTRK_OK; ++pi) {
      for (int bi = 0; bi < 3 && rc == LTRK_OK; ++bi) {
        const ltrk_plan p{ks[ki], blocks[bi], ppls[pi], 1};
        const double ms = time_batched(table, turns, integrator, dtype, s, p, &rc);
        if (ms > 0.0) {
          const double rate = static_cast<double>(total) * turns / ms;
          if (rate > best_rate) {
            best_rate = rate;
            best = p;
          }
        }
      }
    }
  }
  {
    std::lock_guard<std::mutex> g(g_plan_mu);
    g_forced = saved_forced;
    g_forced_plan = saved_plan;
  }
  hipStreamSynchronize(s);
  hipFree(buf);
  if (rc != LTRK_OK) return rc;
  {
    std::lock_guard<std::mutex> g(g_plan_mu);
    g_tuned[TuneKey(device_arch(), integrator, dtype, log2_bucket(total), 1)] = best;
  }
  if (best_out) *best_out = best;
  return LTRK_OK;
}

}  // namespace
}  // namespace ltrk

using namespace ltrk;

extern "C" {

int ltrk_set_plan(const ltrk_plan* plan) {
  clear_error();
  std::lock_guard<std::mutex> g(g_plan_mu);
  if (!plan) {
    g_forced = false;
    return LTRK_OK;
  }
  if (!plan_valid(*plan))
    return fail(LTRK_EINVAL, "invalid plan (K %d, block %d, ppl %d, graph %d)",
                plan->turns_per_launch, plan->block, plan->ppl, plan->use_graph);
  g_forced = true;
  g_forced_plan = *plan;
  return LTRK_OK;
}

int ltrk_get_plan(int integrator, int dtype, int64_t n, ltrk_plan* out) {
  clear_error();
  if (!out) return fail(LTRK_EINVAL, "out is NULL");
  if (!valid_integrator(integrator) || !valid_dtype(dtype) || n < 0)
    return fail(LTRK_EINVAL, "invalid integrator, dtype or n");
  *out = choose_plan(integrator, dtype, n, false);
  return LTRK_OK;
}

int ltrk_get_plan_batched(int integrator, int dtype, int64_t total_n, ltrk_plan* out) {
  clear_error();
  if (!out) return fail(LTRK_EINVAL, "out is NULL");
  if (!valid_integrator(integrator) || !valid_dtype(dtype) || total_n < 0)
    return fail(LTRK_EINVAL, "invalid integrator, dtype or n");
  *out = choose_plan(integrator, dtype, total_n, true);
  return LTRK_OK;
}

int ltrk_autotune(int integrator, int dtype, int64_t n, void* stream, ltrk_plan* best) {
  try {
    clear_error();
    return autotune(integrator, dtype, n, static_cast<hipStream_t>(stream), best);
  } catch (...) {
    return fail(LTRK_EDEVICE, "unexpected internal error in autotune");
  }
}

int ltrk_autotune_batched(const ltrk_bunch* bunches, int nb, int integrator, int dtype,
                          void* stream, ltrk_plan* best) {
  try {
    clear_error();
    return autotune_batched(bunches, nb, integrator, dtype, static_cast<hipStream_t>(stream),
                            best);
  } catch (...) {
    return fail(LTRK_EDEVICE, "unexpected internal error in autotune");
  }
}

int ltrk_tune_cache_save(const char* path) {
  clear_error();
  if (!path) return fail(LTRK_EINVAL, "path is NULL");
  std::lock_guard<std::mutex> g(g_plan_mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(LTRK_EINVAL, "cannot open %s", path);
  std::fprintf(f, "# arch integrator dtype log2n batched K block ppl graph\n");
  for (const auto& kv : g_tuned) {
    const auto& k = kv.first;
    const ltrk_plan& p = kv.second;
    std::fprintf(f, "%s %d %d %d %d %d %d %d %d\n", std::get<0>(k).c_str(), std::get<1>(k),
                 std::get<2>(k), std::get<3>(k), std::get<4>(k), p.turns_per_launch, p.block, p.ppl,
                 p.use_graph);
  }
  std::fclose(f);
  return LTRK_OK;
}

int ltrk_tune_cache_load(const char* path) {
  clear_error();
  if (!path) return fail(LTRK_EINVAL, "path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(LTRK_EINVAL, "cannot open %s", path);
  // Lines that do not parse as a valid entry are skipped.
  char line[256];
  std::lock_guard<std::mutex> g(g_plan_mu);
  while (std::fgets(line, sizeof(line), f)) {
    if (line[0] == '#') continue;
    char arch[64];
    int integ, dtype, bucket, batched;
    ltrk_plan p;
    if (std::sscanf(line, "%63s %d %d %d %d %d %d %d %d", arch, &integ, &dtype, &bucket, &batched,
                    &p.turns_per_launch, &p.block, &p.ppl, &p.use_graph) == 9 &&
        plan_valid(p) && valid_integrator(integ) && valid_dtype(dtype)) {
      g_tuned[TuneKey(arch, integ, dtype, bucket, batched)] = p;
    }
  }
  std::fclose(f);
  return LTRK_OK;
}

}  // extern "C"
