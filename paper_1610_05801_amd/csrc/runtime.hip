// Host runtime and C ABI of libltrk: argument validation, ring constants,
// per-stream scratch for moment partials, launch sequences (eager, timed or
// replayed from a cached hipGraph) and the single-bunch / batched tracking
// entry points declared in include/ltrk.h.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <list>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "sinpi_coeffs.h"

namespace ltrk {

// ---------------------------------------------------------------------------
// Errors

namespace {
thread_local int t_err_code = 0;
thread_local char t_err_msg[512] = "";
}  // namespace

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(t_err_msg, sizeof(t_err_msg), fmt, ap);
  va_end(ap);
  t_err_code = code;
  return code;
}

int fail_hip(hipError_t e, const char* what) {
  return fail(LTRK_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() {
  t_err_code = 0;
  t_err_msg[0] = '\0';
}

// ---------------------------------------------------------------------------
// Ring constants

bool valid_integrator(int i) { return i >= LTRK_EULER_CROMER && i <= LTRK_RK4; }
bool valid_dtype(int d) { return d == LTRK_F64 || d == LTRK_F32C; }

int validate_ring(const ltrk_ring* r) {
  if (!r) return fail(LTRK_EINVAL, "ring is NULL");
  const double v[7] = {r->circumference_m, r->harmonic, r->voltage_V, r->p0c_eV,
                       r->mass_eV,         r->gamma_t,  r->charge_e};
  for (double x : v)
    if (!std::isfinite(x)) return fail(LTRK_EINVAL, "ring parameter is not finite");
  if (!(r->circumference_m > 0.0)) return fail(LTRK_EINVAL, "circumference must be > 0");
  if (!(r->harmonic > 0.0) || std::floor(r->harmonic) != r->harmonic)
    return fail(LTRK_EINVAL, "harmonic must be a positive integer");
  if (!(r->p0c_eV > 0.0)) return fail(LTRK_EINVAL, "p0c must be > 0");
  if (!(r->mass_eV >= 0.0)) return fail(LTRK_EINVAL, "mass must be >= 0");
  if (!(r->gamma_t > 0.0)) return fail(LTRK_EINVAL, "gamma_t must be > 0");
  return LTRK_OK;
}

void derive(const ltrk_ring& r, ltrk_derived* o) {
  // Lorentz factors from the momentum in units of the rest energy.
  if (r.mass_eV == 0.0) {
    o->gamma = INFINITY;
    o->beta = 1.0;
  } else {
    const double bg = r.p0c_eV / r.mass_eV;
    o->gamma = std::sqrt(1.0 + bg * bg);
    o->beta = bg / o->gamma;
  }
  o->eta = 1.0 / (r.gamma_t * r.gamma_t) - 1.0 / (o->gamma * o->gamma);
  o->kick_amplitude = r.charge_e * r.voltage_V / (o->beta * r.p0c_eV);
  o->wavenumber = 2.0 * M_PI * r.harmonic / r.circumference_m;
  o->slip_length = o->eta * r.circumference_m;
  const double A = o->kick_amplitude, k = o->wavenumber, D = o->slip_length;
  const double w2 = A * k * D;
  if (w2 > 0.0) {
    o->omega_s = std::sqrt(w2);
    o->q_s = o->omega_s / (2.0 * M_PI);
    o->q_leapfrog = o->omega_s < 2.0 ? std::asin(0.5 * o->omega_s) / M_PI : NAN;
    o->bucket_height = 2.0 * std::sqrt(A / (k * D));
  } else {
    o->omega_s = o->q_s = o->q_leapfrog = o->bucket_height = NAN;
  }
  o->bucket_half_length = 0.5 * r.circumference_m / r.harmonic;
  o->h_separatrix = -2.0 * A / k;
}

void make_coeffs(const ltrk_ring& r, int integrator, Coeffs* c) {
  ltrk_derived d;
  derive(r, &d);
  const double A = d.kick_amplitude, D = d.slip_length;
  std::memset(c, 0, sizeof(*c));
  c->half_rev_per_m = 2.0 * r.harmonic / r.circumference_m;
  c->neg_D = -D;
  double kw[2] = {A, 0.0};  // kick weights x A
  double drift_sum = 1.0, kick_sum = 1.0;  // summed absolute drift and kick weights
  switch (integrator) {
    case LTRK_EULER_CROMER:
      c->nd[0] = -D;
      break;
    case LTRK_LEAPFROG:
      c->nd[0] = -(0.5 * D);
      break;
    case LTRK_RUTH4: {
      // Forest-Ruth: drifts th/2, (1-th)/2, (1-th)/2, th/2; kicks th, 1-2th, th.
      const double th = 1.0 / (2.0 - std::cbrt(2.0));
      c->nd[0] = -((0.5 * th) * D);
      c->nd[1] = -((0.5 * (1.0 - th)) * D);
      kw[0] = th * A;
      kw[1] = (1.0 - 2.0 * th) * A;
      drift_sum = th + (th - 1.0);
      kick_sum = 2.0 * th + (2.0 * th - 1.0);
      break;
    }
    default:  // RK4: the force A sin(k z); a step moves delta by at most |A| and
              // z (stages included) by at most |D| (|delta| + |A|)
      break;
  }
  c->z_exact = kExactRange / c->half_rev_per_m;
  c->reach_d = drift_sum * std::fabs(D);
  c->reach_k = kick_sum * std::fabs(A);
  static_assert(kSinTerms == kSinPiTerms, "polynomial length");
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < kSinTerms; ++j) c->kq[i][j] = kw[i] * kSinPiCoeff[j];
  for (int i = 0; i < 2; ++i) {
    c->nd_f[i][0] = static_cast<float>(c->nd[i]);
    c->nd_f[i][1] = static_cast<float>(c->nd[i] - static_cast<double>(c->nd_f[i][0]));
    const double a = kw[i] * M_PI;
    c->ka_f[i][0] = static_cast<float>(a);
    c->ka_f[i][1] = static_cast<float>(a - static_cast<double>(c->ka_f[i][0]));
  }
}

int validate_rf2(const ltrk_rf2* r) {
  if (!r) return fail(LTRK_EINVAL, "rf2 is NULL");
  int rc = validate_ring(&r->ring);
  if (rc) return rc;
  const double v[6] = {r->phi1_rad, r->harmonic2, r->voltage2_V, r->phi2_rad, r->eta1, r->eta2};
  for (double x : v)
    if (!std::isfinite(x)) return fail(LTRK_EINVAL, "rf2 parameter is not finite");
  if (r->voltage2_V != 0.0 && (!(r->harmonic2 > 0.0) || std::floor(r->harmonic2) != r->harmonic2))
    return fail(LTRK_EINVAL, "harmonic2 must be a positive integer");
  return LTRK_OK;
}

void make_coeffs_rf2(const ltrk_rf2& r, int integrator, CoeffsRf2* c) {
  ltrk_derived d;
  derive(r.ring, &d);
  const double C = r.ring.circumference_m;
  const double eta[3] = {d.eta, r.eta1, r.eta2};
  const double A[2] = {d.kick_amplitude,
                       r.ring.charge_e * r.voltage2_V / (d.beta * r.ring.p0c_eV)};
  std::memset(c, 0, sizeof(*c));
  c->s[0] = 2.0 * r.ring.harmonic / C;
  c->s[1] = 2.0 * r.harmonic2 / C;
  c->u0[0] = r.phi1_rad / M_PI;
  c->u0[1] = r.phi2_rad / M_PI;
  c->harmonics = r.voltage2_V != 0.0 ? 2 : 1;
  double wd[2] = {1.0, 0.0}, wk[2] = {1.0, 0.0};  // drift and kick weights (turns)
  switch (integrator) {
    case LTRK_LEAPFROG:
      wd[0] = 0.5;
      break;
    case LTRK_RUTH4: {
      const double th = 1.0 / (2.0 - std::cbrt(2.0));
      wd[0] = 0.5 * th;
      wd[1] = 0.5 * (1.0 - th);
      wk[0] = th;
      wk[1] = 1.0 - 2.0 * th;
      break;
    }
    default:  // Euler-Cromer and RK4 (slip and force of weight 1)
      break;
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) c->nd[i][j] = -((wd[i] * C) * eta[j]);
  for (int i = 0; i < 2; ++i)
    for (int h = 0; h < 2; ++h)
      for (int j = 0; j < kSinTerms; ++j) c->kq[i][h][j] = (wk[i] * A[h]) * kSinPiCoeff[j];
}

// ---------------------------------------------------------------------------
// RF programme: per-turn records of folded coefficients

int validate_program(const ltrk_rf2* rf, const ltrk_rf_turn* prog, int64_t turns,
                     int integrator, bool* accel, int* harmonics) {
  int rc = validate_rf2(rf);
  if (rc) return rc;
  if (turns > 0 && !prog) return fail(LTRK_EINVAL, "program is NULL");
  const double h2 = rf->harmonic2;
  const bool h2_ok = h2 > 0.0 && std::floor(h2) == h2;
  bool acc = false;
  int harm = 1;
  double before = rf->ring.p0c_eV;
  for (int64_t t = 0; t < turns; ++t) {
    const ltrk_rf_turn& e = prog[t];
    const double v[5] = {e.voltage_V, e.phi1_rad, e.voltage2_V, e.phi2_rad, e.p0c_eV};
    for (double x : v)
      if (!std::isfinite(x))
        return fail(LTRK_EINVAL, "programme entry %lld is not finite", (long long)t);
    if (!(e.p0c_eV > 0.0))
      return fail(LTRK_EINVAL, "programme entry %lld: p0c must be > 0", (long long)t);
    if (e.voltage2_V != 0.0) {
      if (!h2_ok)
        return fail(LTRK_EINVAL, "programme entry %lld has voltage2 but harmonic2 is not a "
                    "positive integer", (long long)t);
      harm = 2;
    }
    if (e.p0c_eV != before) acc = true;
    before = e.p0c_eV;
  }
  if (acc && integrator == LTRK_RK4)
    return fail(LTRK_EUNSUPPORTED, "RK4 needs a constant reference momentum");
  *accel = acc;
  *harmonics = harm;
  return LTRK_OK;
}

// Fill `turns` records of prog_layout(integrator) for the programme. Turn t
// moves the reference from p_a to p_b; kick j of weight wk_j ends at the
// reference p_a + W_j (p_b - p_a) (W_j: kick weights summed up to j, the last
// one exactly p_b), and drift j runs at the reference current before it. The
// constants use derive() on the ring at that momentum, so a constant
// programme gives the coefficients of make_coeffs_rf2 bit for bit.
void fill_program(const ltrk_rf2& rf, const ltrk_rf_turn* prog, int64_t turns, int integrator,
                  double* out) {
  const ProgLayout L = prog_layout(integrator);
  const double th = 1.0 / (2.0 - std::cbrt(2.0));
  double wd[4] = {1.0, 0.0, 0.0, 0.0}, wk[3] = {1.0, 0.0, 0.0}, W[3] = {1.0, 0.0, 0.0};
  int dref[4] = {0, 0, 0, 0};  // reference index (0 = p_a, j+1 = after kick j) of drift j
  if (integrator == LTRK_LEAPFROG) {
    wd[0] = wd[1] = 0.5;
    dref[1] = 1;
  } else if (integrator == LTRK_RUTH4) {
    wd[0] = wd[3] = 0.5 * th;
    wd[1] = wd[2] = 0.5 * (1.0 - th);
    wk[0] = wk[2] = th;
    wk[1] = 1.0 - 2.0 * th;
    W[0] = th;
    W[1] = 1.0 - th;
    W[2] = 1.0;
    dref[1] = 1;
    dref[2] = 2;
    dref[3] = 3;
  }
  const double C = rf.ring.circumference_m;
  const double q = rf.ring.charge_e;
  ltrk_ring r = rf.ring;
  ltrk_derived d;
  double memo_p = NAN, memo_eta = 0.0, memo_beta = 0.0;
  auto at = [&](double p) {  // (eta0, beta) at reference momentum p
    if (p != memo_p) {
      r.p0c_eV = p;
      derive(r, &d);
      memo_p = p;
      memo_eta = d.eta;
      memo_beta = d.beta;
    }
  };
  double p_a = rf.ring.p0c_eV;
  for (int64_t t = 0; t < turns; ++t) {
    const ltrk_rf_turn& e = prog[t];
    const double p_b = e.p0c_eV;
    double pr[4];
    pr[0] = p_a;
    for (int j = 0; j < L.kicks; ++j) pr[j + 1] = j + 1 == L.kicks ? p_b : p_a + W[j] * (p_b - p_a);
    at(p_a);
    const double beta_a = memo_beta;
    double* o = out + t * L.stride;
    std::memset(o, 0, sizeof(double) * L.stride);
    o[L.u0 + 0] = e.phi1_rad / M_PI;
    o[L.u0 + 1] = e.phi2_rad / M_PI;
    for (int j = 0; j < L.drifts; ++j) {
      at(pr[dref[j]]);
      o[L.nd + j] = -((wd[j] * C) * memo_eta);
    }
    const double V[2] = {e.voltage_V, e.voltage2_V};
    for (int j = 0; j < L.kicks; ++j) {
      const double p = pr[j], pn = pr[j + 1];
      o[L.ref + 2 * j] = p / pn;
      o[L.ref + 2 * j + 1] = (p - pn) / pn;
      for (int h = 0; h < 2; ++h) {
        const double A = q * V[h] / (beta_a * pn);
        for (int k = 0; k < kSinTerms; ++k)
          o[L.kq + (2 * j + h) * kSinTerms + k] = (wk[j] * A) * kSinPiCoeff[k];
      }
    }
    p_a = p_b;
  }
}

// ---------------------------------------------------------------------------
// Wake kick: validation and the wake at the lags between slice centres

int validate_wake(const ltrk_wake* w) {
  if (!w) return fail(LTRK_EINVAL, "wake is NULL");
  const double v[6] = {w->shunt, w->freq_hz, w->quality, w->intensity, w->z_lo, w->z_hi};
  for (double x : v)
    if (!std::isfinite(x)) return fail(LTRK_EINVAL, "wake parameter is not finite");
  if (w->model != LTRK_WAKE_RESONATOR && w->model != LTRK_WAKE_CONSTANT)
    return fail(LTRK_EINVAL, "unknown wake model %d", w->model);
  if (w->n_slices < 1 || w->n_slices > kWakeMaxSlices)
    return fail(LTRK_EINVAL, "n_slices must be in [1, %d]", kWakeMaxSlices);
  if (!(w->z_hi > w->z_lo)) return fail(LTRK_EINVAL, "z_hi must be > z_lo");
  if (!(w->intensity >= 0.0)) return fail(LTRK_EINVAL, "intensity must be >= 0");
  if (w->model == LTRK_WAKE_RESONATOR && (!(w->freq_hz > 0.0) || !(w->quality > 0.5)))
    return fail(LTRK_EINVAL, "resonator needs freq_hz > 0 and quality > 1/2");
  return LTRK_OK;
}

// Blocks of the wake turn kernel (grid-stride over wave tiles): each adds its
// slice histogram into the global counts once per turn, so fewer blocks mean
// fewer contended adds and more tiles per block. LTRK_WAKE_BLOCKS overrides
// the default (1 .. kWakeMaxBlocks).
// Grid of the wake turn kernel for a bunch that needs `needed` blocks of wave
// tiles, when the device holds `resident` blocks at once: all of them for a
// bunch of at most one round of blocks, else whole rounds, at most
// kWakeMaxBlocks blocks (the waves then walk the remaining tiles). Measured
// (1000 turns, moments every turn): at 1e7 particles 4096 blocks (4 rounds)
// 1.65e11 particle-turns/s against 1.58e11 with 1024 and 1.60e11 with one
// block per 4 tiles (4883); at 1e8, 8192 blocks 1.74e11 against 1.69e11 with
// 4096 and 1.60e11 with 1024. Every block adds its histogram into the global
// slice counts with integer atomics, so the grid is capped. LTRK_WAKE_BLOCKS
// (1..kWakeMaxBlocks) fixes the number of blocks instead.
int64_t wake_grid(int64_t needed, int64_t resident) {
  static const long forced = [] {
    const char* e = std::getenv("LTRK_WAKE_BLOCKS");
    const long v = e ? std::atol(e) : 0;
    return v > 0 ? std::min<long>(v, kWakeMaxBlocks) : 0L;
  }();
  if (forced) return std::min<int64_t>(needed, forced);
  if (resident <= 0) resident = kWakeMinBlocks;
  if (needed <= resident) return needed;
  const int64_t cap = std::max<int64_t>(kWakeMaxBlocks / resident, 1) * resident;
  return std::min<int64_t>((needed / resident) * resident, std::min<int64_t>(cap, kWakeMaxBlocks));
}

// W at tau = m dz / (beta c), m < n_slices (W(0): half the limit).
void make_wake_table(const ltrk_wake& w, double beta, double* tab) {
  const double c_light = 299792458.0;
  const double dz = (w.z_hi - w.z_lo) / static_cast<double>(w.n_slices);
  const double tau1 = dz / (beta * c_light);
  if (w.model == LTRK_WAKE_CONSTANT) {
    for (int m = 0; m < w.n_slices; ++m) tab[m] = m == 0 ? 0.5 * w.shunt : w.shunt;
    return;
  }
  const double omega_r = 2.0 * M_PI * w.freq_hz;
  const double alpha = omega_r / (2.0 * w.quality);
  const double omega_bar = std::sqrt(omega_r * omega_r - alpha * alpha);
  tab[0] = alpha * w.shunt;
  for (int m = 1; m < w.n_slices; ++m) {
    const double tau = static_cast<double>(m) * tau1;
    tab[m] = 2.0 * alpha * w.shunt * std::exp(-alpha * tau) *
             (std::cos(omega_bar * tau) - alpha / omega_bar * std::sin(omega_bar * tau));
  }
}

// ---------------------------------------------------------------------------
// 6-D map: Twiss parameters of the transverse planes

int validate_twiss(const ltrk_twiss* t) {
  if (!t) return fail(LTRK_EINVAL, "twiss is NULL");
  const double v[8] = {t->q_x, t->qp_x, t->alpha_x, t->beta_x,
                       t->q_y, t->qp_y, t->alpha_y, t->beta_y};
  for (double x : v)
    if (!std::isfinite(x)) return fail(LTRK_EINVAL, "twiss parameter is not finite");
  if (!(t->beta_x > 0.0) || !(t->beta_y > 0.0)) return fail(LTRK_EINVAL, "beta must be > 0");
  return LTRK_OK;
}

// Phase in half revolutions u = 2 frac(Q) + 2 Q' delta (the integer part of
// the tune is dropped exactly: the rotation depends on Q modulo 1).
void make_plane(double q, double qp, double alpha, double beta, PlaneDev* p) {
  p->u0 = 2.0 * (q - std::floor(q));
  p->u1 = 2.0 * qp;
  p->alpha = alpha;
  p->beta = beta;
  p->neg_gamma = -((1.0 + alpha * alpha) / beta);
}

// Doubles per (row, moment) of moment scratch for a bunch of W wave tiles:
// the per-wave sums plus, for two-stage finalizes, the group sums.
int64_t scratch_cols(int64_t W) {
  const int64_t G = finalize_groups(W);
  return W + (G > 1 ? G : 0);
}

int64_t waves_for(int64_t n, int ppl) {
  const int64_t per = static_cast<int64_t>(kWave) * ppl;
  return (n + per - 1) / per;
}

int current_device(int* dev) {
  hipError_t e = hipGetDevice(dev);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  return LTRK_OK;
}

int check_device_range(const void* p, size_t bytes, const char* name) {
  if (!p) return fail(LTRK_EINVAL, "%s is NULL", name);
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(LTRK_EINVAL, "%s (%p) is not device memory (%s)", name, p, hipGetErrorString(e));
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return fail(LTRK_EINVAL, "%s (%p) is not device memory (memory type %d)", name, p,
                static_cast<int>(attr.type));
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  e = hipMemGetAddressRange(&base, &size, const_cast<void*>(p));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(LTRK_EINVAL, "%s: cannot determine its allocation", name);
  }
  const char* b = static_cast<const char*>(base);
  const char* q = static_cast<const char*>(p);
  if (q < b || static_cast<size_t>(q - b) + bytes > size)
    return fail(LTRK_EINVAL, "%s: allocation holds %zu bytes past it, %zu needed", name,
                size - static_cast<size_t>(q - b), bytes);
  return LTRK_OK;
}

// ---------------------------------------------------------------------------
// Timing (ltrk_timing_enable)

namespace {
struct TimedLaunch {
  int kind;
  hipEvent_t a, b;
  bool owns_a;  // false when a is the previous segment's b (a timed graph's chain)
  int count;    // launches between a and b
};
std::mutex g_time_mu;
bool g_time_on = false;
std::vector<TimedLaunch> g_timed;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t pooled_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

bool timing_on() {
  std::lock_guard<std::mutex> g(g_time_mu);
  return g_time_on;
}

void timing_begin(hipStream_t s, int kind, void** token) {
  *token = nullptr;
  std::lock_guard<std::mutex> g(g_time_mu);
  if (!g_time_on) return;
  TimedLaunch t{kind, pooled_event(), pooled_event(), true, 1};
  if (!t.a || !t.b) {
    if (t.a) g_event_pool.push_back(t.a);
    if (t.b) g_event_pool.push_back(t.b);
    return;
  }
  hipEventRecord(t.a, s);
  g_timed.push_back(t);
  *token = reinterpret_cast<void*>(g_timed.size());
}

void timing_end(hipStream_t s, void* token) {
  if (!token) return;
  std::lock_guard<std::mutex> g(g_time_mu);
  const size_t i = reinterpret_cast<size_t>(token) - 1;
  if (i < g_timed.size()) hipEventRecord(g_timed[i].b, s);
}

// Events for a timed graph replay: segment i (counts[i] launches of kind
// kinds[i]) runs between ev[i] and ev[i + 1]. False (and no events) when
// timing is off or events run out.
bool timing_chain(const std::vector<int>& kinds, const std::vector<int>& counts,
                  std::vector<hipEvent_t>* ev) {
  std::lock_guard<std::mutex> g(g_time_mu);
  ev->clear();
  if (!g_time_on) return false;
  for (size_t i = 0; i <= kinds.size(); ++i) {
    hipEvent_t e = pooled_event();
    if (!e) {
      for (hipEvent_t x : *ev) g_event_pool.push_back(x);
      ev->clear();
      return false;
    }
    ev->push_back(e);
  }
  for (size_t i = 0; i < kinds.size(); ++i)
    g_timed.push_back(TimedLaunch{kinds[i], (*ev)[i], (*ev)[i + 1], i == 0, counts[i]});
  return true;
}

// ---------------------------------------------------------------------------
// Launch sequences

namespace {

struct Launch {
  int kind;  // kTimeTrack / kTimeFinalize
  std::function<hipError_t(hipStream_t)> fn;
};

hipError_t run_eager(const std::vector<Launch>& seq, hipStream_t s) {
  for (const Launch& l : seq) {
    void* tok = nullptr;
    timing_begin(s, l.kind, &tok);
    hipError_t e = l.fn(s);
    timing_end(s, tok);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  std::vector<void*> owned;  // device tables that the graph's kernels read
  // Timed graphs (built while ltrk_timing is on): the sequence in segments of
  // consecutive launches of one kind (counts[i] launches of kind kinds[i]),
  // an event-record node before the first segment and one after each
  // (ev_nodes.size() == kinds.size() + 1); every replay sets fresh events
  // into them, so the times come from the replayed graph itself. Events only
  // between segments: an event-record node costs a few microseconds of
  // launch cadence, so a segment's average per launch includes the short
  // gaps between its launches and nothing else.
  std::vector<hipGraphNode_t> ev_nodes;
  std::vector<int> kinds, counts;
  hipEvent_t placeholder = nullptr;
  hipGraph_t graph = nullptr;  // a timed graph's nodes stay valid only with it
};

// Replay a cached graph; a timed one first gets a fresh event per node (the
// placeholder when timing is off or out of events, so that events handed back
// to the pool are never recorded again by an old replay).
hipError_t launch_graph(GraphEntry& ge, hipStream_t s) {
  if (!ge.ev_nodes.empty()) {
    std::vector<hipEvent_t> ev;
    const bool timed = timing_chain(ge.kinds, ge.counts, &ev);
    for (size_t i = 0; i < ge.ev_nodes.size(); ++i) {
      hipError_t e = hipGraphExecEventRecordNodeSetEvent(ge.exec, ge.ev_nodes[i],
                                                         timed ? ev[i] : ge.placeholder);
      if (e != hipSuccess) return e;
    }
  }
  return hipGraphLaunch(ge.exec, s);
}

// Build a timed graph for `seq`: each segment of consecutive launches of one
// kind captured on s into a child graph, the segments chained through
// event-record nodes.
hipError_t build_timed_graph(const std::vector<Launch>& seq, hipStream_t s, GraphEntry* ge,
                             hipGraph_t* out) {
  *out = nullptr;
  hipError_t e = hipEventCreate(&ge->placeholder);
  if (e != hipSuccess) {
    ge->placeholder = nullptr;
    return e;
  }
  hipGraph_t g = nullptr;
  if ((e = hipGraphCreate(&g, 0)) != hipSuccess) return e;
  hipGraphNode_t prev = nullptr;
  if ((e = hipGraphAddEventRecordNode(&prev, g, nullptr, 0, ge->placeholder)) != hipSuccess) {
    hipGraphDestroy(g);
    return e;
  }
  ge->ev_nodes.push_back(prev);
  for (size_t i = 0; i < seq.size();) {
    size_t j = i;
    while (j < seq.size() && seq[j].kind == seq[i].kind) ++j;
    hipGraph_t child = nullptr;
    if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess) break;
    hipError_t le = hipSuccess;
    for (size_t k = i; k < j && le == hipSuccess; ++k) le = seq[k].fn(s);
    e = hipStreamEndCapture(s, &child);
    if (le != hipSuccess || e != hipSuccess || !child) {
      if (child) hipGraphDestroy(child);
      if (e == hipSuccess) e = le != hipSuccess ? le : hipErrorUnknown;
      break;
    }
    hipGraphNode_t cn = nullptr, en = nullptr;
    e = hipGraphAddChildGraphNode(&cn, g, &prev, 1, child);
    hipGraphDestroy(child);
    if (e != hipSuccess) break;
    if ((e = hipGraphAddEventRecordNode(&en, g, &cn, 1, ge->placeholder)) != hipSuccess) break;
    ge->ev_nodes.push_back(en);
    ge->kinds.push_back(seq[i].kind);
    ge->counts.push_back(static_cast<int>(j - i));
    prev = en;
    i = j;
  }
  if (e != hipSuccess) {
    hipGraphDestroy(g);
    return e;
  }
  *out = g;
  return hipSuccess;
}

bool stream_capturing(hipStream_t s) {
  if (!s) return false;
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return st != hipStreamCaptureStatusNone;
}

struct Scratch {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// Per-stream staged tables (programme records, wake table): device copy,
// pinned staging, and an event recorded after the last copy out of the
// staging buffer.
struct ProgBuf {
  void* dev = nullptr;
  size_t dev_bytes = 0;
  double* host = nullptr;
  size_t host_bytes = 0;
  hipEvent_t copied = nullptr;
};

struct DeviceCtx {
  std::mutex mu;
  std::unordered_map<hipStream_t, Scratch> scratch;
  std::vector<void*> retired;  // grown-out scratch buffers, freed at shutdown
  std::unordered_map<hipStream_t, ProgBuf> progs;
  std::list<std::pair<std::string, GraphEntry>> graphs;  // most recent first
  size_t max_graphs = 32;
};

std::mutex g_ctx_mu;
std::unordered_map<int, std::unique_ptr<DeviceCtx>> g_ctx;

DeviceCtx& ctx_for(int dev) {
  std::lock_guard<std::mutex> g(g_ctx_mu);
  auto& p = g_ctx[dev];
  if (!p) p.reset(new DeviceCtx);
  return *p;
}

// Cap of one call's moment-partial scratch, LTRK_SCRATCH_MB (MiB, at least
// 16; default 192), read at every call: runs that need more rows are
// finalized in chunks. The default keeps a chunk's partials within the 256 MB
// last-level cache, where the finalize reads them back (measured +1.4% at
// 1e6 particles over a 1 GiB cap, whose single chunk of 10^4 rows the
// finalize had to read from HBM; equal at 1e7).
size_t scratch_cap_bytes() {
  const char* e = std::getenv("LTRK_SCRATCH_MB");
  long mb = e ? std::atol(e) : 192;
  if (mb < 16) mb = 16;
  return static_cast<size_t>(mb) << 20;
}

void destroy_entry(GraphEntry& ge) {
  if (ge.exec) hipGraphExecDestroy(ge.exec);
  for (void* p : ge.owned) hipFree(p);
  if (ge.placeholder) hipEventDestroy(ge.placeholder);
  if (ge.graph) hipGraphDestroy(ge.graph);
  ge.graph = nullptr;
  ge.exec = nullptr;
  ge.owned.clear();
  ge.ev_nodes.clear();
  ge.kinds.clear();
  ge.counts.clear();
  ge.placeholder = nullptr;
}

// Cache key of a graph: timed and untimed graphs of one sequence differ.
std::string graph_key(const std::string& key) {
  return key + (timing_on() ? 'T' : 'U');
}

// Drop every cached graph (device must be idle w.r.t. them).
void clear_graphs(DeviceCtx& c) {
  for (auto& kv : c.graphs) destroy_entry(kv.second);
  c.graphs.clear();
}

// Scratch of at least `bytes` for stream s (grown, never shrunk). A grown-out
// buffer is kept until shutdown rather than freed: graphs that a caller
// captured from earlier calls on the stream still name it (cached graphs of
// the library key on the scratch address, so they keep using it too). Growth
// at least doubles the buffer, so the kept buffers add up to less than the
// current one. Under stream capture the scratch cannot grow (EUNSUPPORTED).
int ensure_scratch(DeviceCtx& c, hipStream_t s, size_t bytes, void** out) {
  Scratch& sc = c.scratch[s];
  if (sc.bytes >= bytes && sc.ptr) {
    *out = sc.ptr;
    return LTRK_OK;
  }
  if (stream_capturing(s))
    return fail(LTRK_EUNSUPPORTED,
                "the call needs %zu bytes of scratch on a capturing stream that has %zu; run it "
                "once uncaptured first",
                bytes, sc.bytes);
  size_t want = std::max(bytes, static_cast<size_t>(1) << 20);
  if (sc.ptr) want = std::max(want, 2 * sc.bytes);
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess && want > bytes) {  // the doubling alone may not fit
    (void)hipGetLastError();
    want = std::max(bytes, static_cast<size_t>(1) << 20);
    e = hipMalloc(&p, want);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(LTRK_ENOMEM, "scratch allocation of %zu bytes failed", want);
  }
  if (sc.ptr) c.retired.push_back(sc.ptr);
  sc.ptr = p;
  sc.bytes = want;
  *out = sc.ptr;
  return LTRK_OK;
}

// Staging and device buffers of at least `bytes` for stream s. Returns once
// the staging buffer is free (its previous copy has run); the device buffer
// is overwritten in stream order by send_program.
int stage_program(DeviceCtx& c, hipStream_t s, size_t bytes, double** host, void** dev) {
  ProgBuf& pb = c.progs[s];
  hipError_t e;
  if (!pb.copied) {
    if ((e = hipEventCreateWithFlags(&pb.copied, hipEventDisableTiming)) != hipSuccess) {
      pb.copied = nullptr;
      return fail_hip(e, "programme event");
    }
  } else if ((e = hipEventSynchronize(pb.copied)) != hipSuccess) {
    return fail_hip(e, "wait for the previous programme copy");
  }
  const size_t want = std::max(bytes, static_cast<size_t>(1) << 16);
  if (pb.host_bytes < bytes) {
    if (pb.host) hipHostFree(pb.host);
    pb.host = nullptr;
    pb.host_bytes = 0;
    if ((e = hipHostMalloc(reinterpret_cast<void**>(&pb.host), want, hipHostMallocDefault)) !=
        hipSuccess) {
      (void)hipGetLastError();
      pb.host = nullptr;
      return fail(LTRK_ENOMEM, "pinned programme staging of %zu bytes failed", want);
    }
    pb.host_bytes = want;
  }
  if (pb.dev_bytes < bytes) {
    if ((e = hipDeviceSynchronize()) != hipSuccess)
      return fail_hip(e, "hipDeviceSynchronize before programme buffer growth");
    clear_graphs(c);  // cached graphs may name the old buffer
    if (pb.dev) hipFree(pb.dev);
    pb.dev = nullptr;
    pb.dev_bytes = 0;
    if ((e = hipMalloc(&pb.dev, want)) != hipSuccess) {
      (void)hipGetLastError();
      pb.dev = nullptr;
      return fail(LTRK_ENOMEM, "programme buffer of %zu bytes failed", want);
    }
    pb.dev_bytes = want;
  }
  *host = pb.host;
  *dev = pb.dev;
  return LTRK_OK;
}

int send_program(DeviceCtx& c, hipStream_t s, size_t bytes) {
  ProgBuf& pb = c.progs[s];
  hipError_t e = hipMemcpyAsync(pb.dev, pb.host, bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return fail_hip(e, "programme upload");
  if ((e = hipEventRecord(pb.copied, s)) != hipSuccess) return fail_hip(e, "programme event");
  return LTRK_OK;
}


// Run `seq` on s: from the graph cache under `key` when allowed, else eagerly.
// `owned` device tables are kept alive with the cached graph (or freed after
// an eager run once the stream is done with them).
int execute(DeviceCtx& c, const std::string& key_in, std::vector<Launch>& seq, hipStream_t s,
            bool use_graph, GraphEntry** made = nullptr) {
  if (made) *made = nullptr;
  const bool graph = use_graph && s != nullptr && !stream_capturing(s);
  if (!graph) {
    hipError_t e = run_eager(seq, s);
    if (e != hipSuccess) return fail_hip(e, "kernel launch");
    return LTRK_OK;
  }
  const std::string key = graph_key(key_in);
  const bool timed = key.back() == 'T';
  for (auto it = c.graphs.begin(); it != c.graphs.end(); ++it) {
    if (it->first == key) {
      c.graphs.splice(c.graphs.begin(), c.graphs, it);
      hipError_t e = launch_graph(it->second, s);
      if (e != hipSuccess) return fail_hip(e, "hipGraphLaunch");
      return LTRK_OK;
    }
  }
  GraphEntry ge;
  hipGraph_t g = nullptr;
  hipError_t e;
  if (timed) {
    e = build_timed_graph(seq, s, &ge, &g);
    if (e != hipSuccess) {
      destroy_entry(ge);
      return fail_hip(e, "timed graph capture");
    }
  } else {
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      e = run_eager(seq, s);
      return e == hipSuccess ? LTRK_OK : fail_hip(e, "kernel launch");
    }
    hipError_t le = run_eager(seq, s);
    e = hipStreamEndCapture(s, &g);
    if (le != hipSuccess || e != hipSuccess || !g) {
      if (g) hipGraphDestroy(g);
      return fail_hip(le != hipSuccess ? le : e, "graph capture");
    }
  }
  e = hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0);
  if (timed)
    ge.graph = g;  // its event-record node handles are set on every replay
  else
    hipGraphDestroy(g);
  if (e != hipSuccess) {
    ge.exec = nullptr;
    destroy_entry(ge);
    return fail_hip(e, "hipGraphInstantiate");
  }
  if (c.graphs.size() >= c.max_graphs) {
    hipDeviceSynchronize();
    destroy_entry(c.graphs.back().second);
    c.graphs.pop_back();
  }
  c.graphs.emplace_front(key, std::move(ge));
  if (made) *made = &c.graphs.front().second;
  e = launch_graph(c.graphs.front().second, s);
  if (e != hipSuccess) return fail_hip(e, "hipGraphLaunch");
  return LTRK_OK;
}

// Launches of one call above which the call runs eagerly, its sequence
// launched in pieces of this length as it is generated (LTRK_MAX_GRAPH_LAUNCHES,
// at least 16, read at every call; default 32768): a graph of that many nodes
// takes long to build and saves nothing on launches of a millisecond, and a
// long sequence is never held whole in host memory.
size_t max_graph_launches() {
  const char* e = std::getenv("LTRK_MAX_GRAPH_LAUNCHES");
  long v = e ? std::atol(e) : 32768;
  if (v < 16) v = 16;
  return static_cast<size_t>(v);
}

// Launches of a run of `turns` turns in chunks of `rows` (the moment finalize
// cadence), `per` turns per launch, plus `extra` launches after each chunk.
int64_t count_launches(int64_t turns, int64_t rows, int64_t per, int64_t extra) {
  auto in = [&](int64_t len) { return (len + per - 1) / per + extra; };
  return (turns / rows) * in(rows) + (turns % rows ? in(turns % rows) : 0);
}

// A call's launch sequence: collected for execute(), or, when `expected`
// exceeds max_graph_launches(), launched eagerly in pieces as it is pushed.
class LaunchSeq {
 public:
  LaunchSeq(int64_t expected, hipStream_t s)
      : piece_(max_graph_launches()), eager_(expected > static_cast<int64_t>(piece_)), s_(s) {}
  bool eager() const { return eager_; }
  std::vector<Launch>& seq() { return seq_; }
  void push(Launch l) {
    seq_.push_back(std::move(l));
    if (eager_ && seq_.size() >= piece_) flush();
  }
  // Launch what is pending (eager mode); the first launch error, if any.
  hipError_t flush() {
    if (err_ == hipSuccess && !seq_.empty()) err_ = run_eager(seq_, s_);
    seq_.clear();
    return err_;
  }

 private:
  size_t piece_;
  bool eager_;
  hipStream_t s_;
  hipError_t err_ = hipSuccess;
  std::vector<Launch> seq_;
};

// Run a collected or streamed sequence to its end.
int finish(DeviceCtx& c, const std::string& key, LaunchSeq& ls, hipStream_t s, bool use_graph,
           GraphEntry** made = nullptr) {
  if (made) *made = nullptr;
  if (ls.eager()) {
    hipError_t e = ls.flush();
    return e == hipSuccess ? LTRK_OK : fail_hip(e, "kernel launch");
  }
  return execute(c, key, ls.seq(), s, use_graph, made);
}

template <typename T>
void key_add(std::string& k, const T& v) {
  k.append(reinterpret_cast<const char*>(&v), sizeof(T));
}

// Rows (turns) of partial sums per finalize chunk for `waves_total` waves,
// a multiple of K unless the whole run is shorter.
int64_t chunk_rows(int64_t turns, int64_t K, int64_t cols_total, bool two_stage,
                   size_t cap_bytes) {
  const int64_t per_row = cols_total * 5 * static_cast<int64_t>(sizeof(double));
  int64_t cap = static_cast<int64_t>(cap_bytes) / std::max<int64_t>(per_row, 1);
  if (two_stage && cap > 65535) cap = 65535;  // grid rows of the group-sum stage
  if (cap >= turns) return turns;
  if (cap >= K) return (cap / K) * K;
  return cap;  // may be < K (the caller then shortens launches)
}

int64_t chunk_rows(int64_t turns, int64_t K, int64_t cols_total, bool two_stage) {
  return chunk_rows(turns, K, cols_total, two_stage, scratch_cap_bytes());
}

}  // namespace

// ---------------------------------------------------------------------------
// Single-bunch tracking

static int track_single(void* z, void* dp, void* zc, void* dc, int64_t n, int64_t turns,
                        const ltrk_ring* ring, int integrator, int dtype, ltrk_moments* mom,
                        hipStream_t s, const ltrk_rf2* ext = nullptr,
                        const ltrk_rf_turn* program = nullptr, bool use_program = false) {
  bool accel = false;
  int harmonics = 1;
  int rc = use_program ? validate_program(ext, program, turns, integrator, &accel, &harmonics)
           : ext       ? validate_rf2(ext)
                       : validate_ring(ring);
  if (rc) return rc;
  if (ext) ring = &ext->ring;
  if (!valid_integrator(integrator)) return fail(LTRK_EINVAL, "unknown integrator %d", integrator);
  if (n < 0) return fail(LTRK_EINVAL, "n must be >= 0");
  if (turns < 0) return fail(LTRK_EINVAL, "turns must be >= 0");
  if (turns > INT32_MAX) return fail(LTRK_EINVAL, "turns must be < 2^31");
  if (turns == 0) return LTRK_OK;
  if (use_program && stream_capturing(s))
    return fail(LTRK_EUNSUPPORTED, "the programme upload cannot be captured into a graph");
  if (mom && (rc = check_device_range(mom, static_cast<size_t>(turns) * sizeof(ltrk_moments),
                                      "moments")))
    return rc;
  if (n == 0) {
    if (!mom) return LTRK_OK;
    hipError_t e = launch_fill_nan(mom, turns, s);
    return e == hipSuccess ? LTRK_OK : fail_hip(e, "fill moments");
  }
  const size_t elem = dtype == LTRK_F64 ? sizeof(double) : sizeof(float);
  const size_t bytes = static_cast<size_t>(n) * elem;
  if ((rc = check_device_range(z, bytes, "z"))) return rc;
  if ((rc = check_device_range(dp, bytes, "dp"))) return rc;
  if (dtype == LTRK_F32C) {
    if ((rc = check_device_range(zc, bytes, "z_comp"))) return rc;
    if ((rc = check_device_range(dc, bytes, "dp_comp"))) return rc;
  }
  int dev = 0;
  if ((rc = current_device(&dev))) return rc;
  bool default_plan = false;
  ltrk_plan plan = choose_plan(integrator, dtype, n, false, &default_plan);
  // extended kernels: 4 or 8 particles per lane (16 is compiled for the
  // single-harmonic kernels only)
  if (ext) plan.ppl = std::min(std::max(plan.ppl, 4), 8);
  if (mom && default_plan)
    plan.turns_per_launch = static_cast<int32_t>(default_turns_for_partials(
        plan.turns_per_launch,
        5 * waves_for(n, plan.ppl) * static_cast<int64_t>(sizeof(double))));

  BunchDev b;
  std::memset(&b, 0, sizeof(b));
  b.z = z;
  b.dp = dp;
  b.z_comp = zc;
  b.dp_comp = dc;
  b.n = n;
  b.waves = waves_for(n, plan.ppl);
  b.integrator = integrator;
  b.dtype = dtype;
  b.active = 1;
  make_coeffs(*ring, integrator, &b.c);
  CoeffsRf2 ce;
  std::memset(&ce, 0, sizeof(ce));
  if (ext) make_coeffs_rf2(*ext, integrator, &ce);
  if (use_program) ce.harmonics = harmonics;

  DeviceCtx& c = ctx_for(dev);
  std::lock_guard<std::mutex> lock(c.mu);
  int64_t K = plan.turns_per_launch;
  int64_t rows = turns;
  void* scratch = nullptr;
  const int64_t groups = finalize_groups(b.waves);
  double* centre = nullptr;
  if (mom) {
    rows = chunk_rows(turns, K, scratch_cols(b.waves), groups > 1);
    if (rows < 1) return fail(LTRK_ENOMEM, "scratch cap too small for %lld waves", (long long)b.waves);
    K = std::min<int64_t>(K, rows);
    const size_t part = static_cast<size_t>(rows) * 5 * scratch_cols(b.waves);
    if ((rc = ensure_scratch(c, s, (part + kCentreDoubles) * sizeof(double), &scratch)))
      return rc;
    centre = static_cast<double*>(scratch) + part;
    b.centre = centre;
  }

  void* prog_dev = nullptr;
  if (use_program) {
    const size_t stride = static_cast<size_t>(prog_layout(integrator).stride);
    const size_t bytes = static_cast<size_t>(turns) * stride * sizeof(double);
    double* host = nullptr;
    if ((rc = stage_program(c, s, bytes, &host, &prog_dev))) return rc;
    fill_program(*ext, program, turns, integrator, host);
    if ((rc = send_program(c, s, bytes))) return rc;
  }

  std::string key;
  key_add(key, use_program ? 4 : ext ? 3 : 1);
  key_add(key, b);
  if (ext) key_add(key, ce);
  if (use_program) {
    key_add(key, prog_dev);
    key_add(key, accel);
  }
  key_add(key, plan);
  key_add(key, turns);
  key_add(key, mom);
  key_add(key, scratch);

  LaunchSeq seq(count_launches(turns, rows, K, mom ? 1 : 0) + (mom ? 1 : 0), s);
  if (mom) {
    const CentreDev cd{z, dp, zc, dc, n, dtype, centre};
    seq.push({kTimeFinalize, [cd](hipStream_t st) { return launch_centre(cd, st); }});
  }
  for (int64_t c0 = 0; c0 < turns; c0 += rows) {
    const int64_t len = std::min(rows, turns - c0);
    for (int64_t j = 0; j < len; j += K) {
      BunchDev bl = b;
      bl.turns = static_cast<int32_t>(std::min(K, len - j));
      bl.partials = static_cast<double*>(scratch);
      const int32_t row0 = static_cast<int32_t>(j);
      const int ppl = plan.ppl, block = plan.block;
      const int32_t turn0 = static_cast<int32_t>(c0 + j);
      if (use_program)
        seq.push({kTimeTrack, [bl, ce, prog_dev, turn0, row0, ppl, block, accel](
                                       hipStream_t st) {
                         return launch_track_prog(bl, ce, static_cast<const double*>(prog_dev),
                                                  turn0, row0, ppl, block, accel, st);
                       }});
      else if (ext)
        seq.push({kTimeTrack, [bl, ce, row0, ppl, block](hipStream_t st) {
                         return launch_track_rf2(bl, ce, row0, ppl, block, st);
                       }});
      else
        seq.push({kTimeTrack, [bl, row0, ppl, block](hipStream_t st) {
                         return launch_track_single(bl, row0, ppl, block, st);
                       }});
    }
    if (mom) {
      FinalizeDev f;
      std::memset(&f, 0, sizeof(f));
      f.partials = static_cast<const double*>(scratch);
      f.stage = static_cast<double*>(scratch) + rows * 5 * b.waves;
      f.waves = b.waves;
      f.groups = groups;
      f.n = n;
      f.out = mom + c0;
      f.centre = centre;
      f.rows = static_cast<int32_t>(len);
      seq.push({kTimeFinalize, [f](hipStream_t st) { return launch_finalize_single(f, st); }});
    }
  }
  return finish(c, key, seq, s, plan.use_graph != 0);
}

// ---------------------------------------------------------------------------
// Tracking without allocation (ltrk_track_f64_noalloc)

namespace noalloc {

// The moment-partial scratch of the allocation-free entry point: one array on
// every device the library runs on, for the life of the process. In host code
// the name `scratch` stands for a host-side stand-in, not device memory: host
// code uses only the device address that hipGetSymbolAddress returned for
// the device (device_scratch), for kernel arguments as for anything else.
constexpr size_t kBytes = LTRK_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) double scratch[kBytes / sizeof(double)];

constexpr int kMaxDevices = 64;

namespace {
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
}  // namespace

// Set-up, once per device (dev is current): the device address of `scratch`,
// and the plan lookup's first use on the device (it caches the device's
// architecture name), so that later calls allocate nothing on the host either.
static int device_scratch(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return fail(LTRK_EINVAL, "device %d: the allocation-free path serves devices 0 to %d", dev,
                kMaxDevices - 1);
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail_hip(e != hipSuccess ? e : hipErrorInvalidSymbol,
                      "hipGetSymbolAddress of the allocation-free scratch");
    }
    (void)choose_plan(LTRK_LEAPFROG, LTRK_F64, 1, false);
    g_ptr[dev] = p;
  }
  *out = static_cast<double*>(g_ptr[dev]);
  return LTRK_OK;
}

}  // namespace noalloc

// ltrk_track_f64 with the moment partials in noalloc::scratch: the same plan
// (hence the same results, bit for bit), launched directly on the stream in
// chunks of turns whose partials fit the array; no graph (instantiating one
// allocates), no launch timing, no hipMalloc or hipFree, no host containers.
static int track_f64_noalloc(double* z, double* dp, int64_t n, int64_t turns,
                             const ltrk_ring* ring, int integrator, ltrk_moments* mom,
                             hipStream_t s) {
  int rc = validate_ring(ring);
  if (rc) return rc;
  if (!valid_integrator(integrator)) return fail(LTRK_EINVAL, "unknown integrator %d", integrator);
  if (n < 0) return fail(LTRK_EINVAL, "n must be >= 0");
  if (turns < 0) return fail(LTRK_EINVAL, "turns must be >= 0");
  if (turns > INT32_MAX) return fail(LTRK_EINVAL, "turns must be < 2^31");
  if (turns == 0) return LTRK_OK;
  if (mom && (rc = check_device_range(mom, static_cast<size_t>(turns) * sizeof(ltrk_moments),
                                      "moments")))
    return rc;
  int dev = 0;
  if ((rc = current_device(&dev))) return rc;
  double* base = nullptr;
  if ((rc = noalloc::device_scratch(dev, &base))) return rc;
  if (n == 0) {
    if (!mom) return LTRK_OK;
    hipError_t e = launch_fill_nan(mom, turns, s);
    return e == hipSuccess ? LTRK_OK : fail_hip(e, "fill moments");
  }
  const size_t bytes = static_cast<size_t>(n) * sizeof(double);
  if ((rc = check_device_range(z, bytes, "z"))) return rc;
  if ((rc = check_device_range(dp, bytes, "dp"))) return rc;
  bool default_plan = false;
  const ltrk_plan plan = choose_plan(integrator, LTRK_F64, n, false, &default_plan);
  BunchDev b;
  std::memset(&b, 0, sizeof(b));
  b.z = z;
  b.dp = dp;
  b.n = n;
  b.waves = waves_for(n, plan.ppl);
  b.integrator = integrator;
  b.dtype = LTRK_F64;
  b.active = 1;
  make_coeffs(*ring, integrator, &b.c);
  int64_t K = plan.turns_per_launch;
  if (mom && default_plan)
    K = default_turns_for_partials(K, 5 * b.waves * static_cast<int64_t>(sizeof(double)));
  int64_t rows = turns;
  const int64_t groups = finalize_groups(b.waves);
  // the last kCentreDoubles of the array hold the centre of the moment sums
  double* centre = base + (noalloc::kBytes / sizeof(double) - kCentreDoubles);
  if (mom) {
    const int64_t row_bytes = 5 * scratch_cols(b.waves) * static_cast<int64_t>(sizeof(double));
    rows = chunk_rows(turns, K, scratch_cols(b.waves), groups > 1,
                      noalloc::kBytes - kCentreDoubles * sizeof(double));
    if (rows < 1)
      return fail(LTRK_EINVAL,
                  "%lld particles need %lld bytes of moment partials per turn; the "
                  "allocation-free scratch holds %zu (pass moments = NULL, or use "
                  "ltrk_track_f64)",
                  static_cast<long long>(n), static_cast<long long>(row_bytes), noalloc::kBytes);
    K = std::min<int64_t>(K, rows);
    b.centre = centre;
    hipError_t e = launch_centre(CentreDev{z, dp, nullptr, nullptr, n, LTRK_F64, centre}, s);
    if (e != hipSuccess) return fail_hip(e, "centre launch");
  }
  for (int64_t c0 = 0; c0 < turns; c0 += rows) {
    const int64_t len = std::min(rows, turns - c0);
    for (int64_t j = 0; j < len; j += K) {
      BunchDev bl = b;
      bl.turns = static_cast<int32_t>(std::min(K, len - j));
      bl.partials = mom ? base : nullptr;
      hipError_t e = launch_track_single(bl, static_cast<int32_t>(j), plan.ppl, plan.block, s);
      if (e != hipSuccess) return fail_hip(e, "kernel launch");
    }
    if (mom) {
      FinalizeDev f;
      std::memset(&f, 0, sizeof(f));
      f.partials = base;
      f.stage = base + rows * 5 * b.waves;
      f.waves = b.waves;
      f.groups = groups;
      f.n = n;
      f.out = mom + c0;
      f.centre = centre;
      f.rows = static_cast<int32_t>(len);
      hipError_t e = launch_finalize_single(f, s);
      if (e != hipSuccess) return fail_hip(e, "finalize launch");
    }
  }
  return LTRK_OK;
}

// ---------------------------------------------------------------------------
// 6-D tracking

static int track_6d(double* const* arr, int64_t n, int64_t turns, const ltrk_rf2* rf,
                    const ltrk_twiss* tw, int integrator, ltrk_moments* mom, hipStream_t s) {
  int rc = validate_rf2(rf);
  if (rc) return rc;
  if ((rc = validate_twiss(tw))) return rc;
  if (!valid_integrator(integrator)) return fail(LTRK_EINVAL, "unknown integrator %d", integrator);
  if (n < 0) return fail(LTRK_EINVAL, "n must be >= 0");
  if (turns < 0) return fail(LTRK_EINVAL, "turns must be >= 0");
  if (turns > INT32_MAX / 3) return fail(LTRK_EINVAL, "turns must be < 2^31 / 3");
  if (turns == 0) return LTRK_OK;
  if (mom && (rc = check_device_range(mom, static_cast<size_t>(turns) * 3 * sizeof(ltrk_moments),
                                      "moments")))
    return rc;
  if (n == 0) {
    if (!mom) return LTRK_OK;
    hipError_t e = launch_fill_nan(mom, 3 * turns, s);
    return e == hipSuccess ? LTRK_OK : fail_hip(e, "fill moments");
  }
  static const char* names[6] = {"z", "dp", "x", "xp", "y", "yp"};
  for (int k = 0; k < 6; ++k)
    if ((rc = check_device_range(arr[k], static_cast<size_t>(n) * sizeof(double), names[k])))
      return rc;
  int dev = 0;
  if ((rc = current_device(&dev))) return rc;
  bool default_plan = false;
  ltrk_plan plan = choose_plan(integrator, LTRK_F64, n, false, &default_plan);
  // six FP64 coordinates per particle: 4 or 8 particles per lane (8 takes
  // ~177 VGPRs and still two waves per SIMD; at 1e6 particles, on one MI355X, it
  // ran leap-frog 2.42e11 against 2.24e11 with 4 and Ruth4 1.64e11 against
  // 1.51e11, both at 256 turns per launch). The default plan takes at most
  // 256 turns per launch here (with 8 per lane: leap-frog 2.43e11 at 512,
  // Ruth4 1.58e11 at 512 against 1.64e11 at 256).
  const int ppl = std::min(std::max(plan.ppl, 4), 8);
  if (mom && default_plan)
    plan.turns_per_launch = static_cast<int32_t>(std::min<int64_t>(
        256, default_turns_for_partials(
                 plan.turns_per_launch,
                 15 * waves_for(n, ppl) * static_cast<int64_t>(sizeof(double)))));

  Bunch6Dev b;
  std::memset(&b, 0, sizeof(b));
  b.z = arr[0];
  b.dp = arr[1];
  b.x = arr[2];
  b.xp = arr[3];
  b.y = arr[4];
  b.yp = arr[5];
  b.n = n;
  b.waves = waves_for(n, ppl);
  b.integrator = integrator;
  Coeffs6d c6;
  std::memset(&c6, 0, sizeof(c6));
  make_coeffs_rf2(*rf, integrator, &c6.rf);
  make_plane(tw->q_x, tw->qp_x, tw->alpha_x, tw->beta_x, &c6.plane[0]);
  make_plane(tw->q_y, tw->qp_y, tw->alpha_y, tw->beta_y, &c6.plane[1]);

  DeviceCtx& c = ctx_for(dev);
  std::lock_guard<std::mutex> lock(c.mu);
  int64_t K = plan.turns_per_launch;
  int64_t rows = turns;
  void* scratch = nullptr;
  const int64_t groups = finalize_groups(b.waves);
  const int64_t cols = 3 * scratch_cols(b.waves);  // 3 planes of 5 sums per row
  double* centre = nullptr;
  if (mom) {
    rows = chunk_rows(turns, K, cols, groups > 1);
    if (rows < 1) return fail(LTRK_ENOMEM, "scratch cap too small for %lld waves", (long long)b.waves);
    K = std::min<int64_t>(K, rows);
    const size_t part = static_cast<size_t>(rows) * 5 * cols;
    if ((rc = ensure_scratch(c, s, (part + kCentreDoubles) * sizeof(double), &scratch)))
      return rc;
    centre = static_cast<double*>(scratch) + part;
    b.centre = centre;
  }

  std::string key;
  key_add(key, 6);
  key_add(key, b);
  key_add(key, c6);
  key_add(key, plan);
  key_add(key, ppl);
  key_add(key, turns);
  key_add(key, mom);
  key_add(key, scratch);

  LaunchSeq seq(count_launches(turns, rows, K, mom ? 3 : 0) + (mom ? 1 : 0), s);
  if (mom) {
    const CentreDev cd{arr[0], arr[1], nullptr, nullptr, n, LTRK_F64, centre};
    seq.push({kTimeFinalize, [cd](hipStream_t st) { return launch_centre(cd, st); }});
  }
  for (int64_t c0 = 0; c0 < turns; c0 += rows) {
    const int64_t len = std::min(rows, turns - c0);
    for (int64_t j = 0; j < len; j += K) {
      Bunch6Dev bl = b;
      bl.turns = static_cast<int32_t>(std::min(K, len - j));
      bl.partials = static_cast<double*>(scratch);
      const int32_t row0 = static_cast<int32_t>(j);
      const int block = plan.block;
      seq.push({kTimeTrack, [bl, c6, row0, ppl, block](hipStream_t st) {
                       return launch_track_6d(bl, c6, row0, ppl, block, st);
                     }});
    }
    if (mom) {
      double* base = static_cast<double*>(scratch);
      for (int p = 0; p < 3; ++p) {
        FinalizeDev f;
        std::memset(&f, 0, sizeof(f));
        f.partials = base + p * 5 * b.waves;
        f.stage = base + rows * 15 * b.waves + p * rows * 5 * groups;
        f.waves = b.waves;
        f.groups = groups;
        f.n = n;
        f.out = mom + c0 * 3 + p;
        f.centre = p == 0 ? centre : nullptr;
        f.rows = static_cast<int32_t>(len);
        f.planes = 3;
        seq.push({kTimeFinalize, [f](hipStream_t st) { return launch_finalize_single(f, st); }});
      }
    }
  }
  return finish(c, key, seq, s, plan.use_graph != 0);
}

// ---------------------------------------------------------------------------
// Tracking with a wake kick after every turn

static int track_wake(double* z, double* dp, int64_t n, int64_t turns, const ltrk_rf2* rf,
                      const ltrk_wake* wk, int integrator, ltrk_moments* mom, hipStream_t s) {
  int rc = validate_rf2(rf);
  if (rc) return rc;
  if ((rc = validate_wake(wk))) return rc;
  if (!valid_integrator(integrator)) return fail(LTRK_EINVAL, "unknown integrator %d", integrator);
  if (n < 0) return fail(LTRK_EINVAL, "n must be >= 0");
  if (turns < 0) return fail(LTRK_EINVAL, "turns must be >= 0");
  if (turns >= INT32_MAX) return fail(LTRK_EINVAL, "turns must be < 2^31 - 1");
  if (turns == 0) return LTRK_OK;
  if (stream_capturing(s))
    return fail(LTRK_EUNSUPPORTED, "the wake table upload cannot be captured into a graph");
  if (mom && (rc = check_device_range(mom, static_cast<size_t>(turns) * sizeof(ltrk_moments),
                                      "moments")))
    return rc;
  if (n == 0) {
    if (!mom) return LTRK_OK;
    hipError_t e = launch_fill_nan(mom, turns, s);
    return e == hipSuccess ? LTRK_OK : fail_hip(e, "fill moments");
  }
  const size_t bytes = static_cast<size_t>(n) * sizeof(double);
  if ((rc = check_device_range(z, bytes, "z"))) return rc;
  if ((rc = check_device_range(dp, bytes, "dp"))) return rc;
  int dev = 0;
  if ((rc = current_device(&dev))) return rc;
  ltrk_plan plan = choose_plan(integrator, LTRK_F64, n, false);
  const int ppl = std::min(std::max(plan.ppl, 4), 8);  // the wake kernels: 4 or 8
  const int block = plan.block;
  const int wpb = block / kWave;

  BunchDev b;
  std::memset(&b, 0, sizeof(b));
  b.z = z;
  b.dp = dp;
  b.n = n;
  b.waves = waves_for(n, ppl);
  b.integrator = integrator;
  b.dtype = LTRK_F64;
  b.active = 1;
  CoeffsRf2 ce;
  make_coeffs_rf2(*rf, integrator, &ce);
  ltrk_derived d;
  derive(rf->ring, &d);

  const int grid = static_cast<int>(
      wake_grid((b.waves + wpb - 1) / wpb,
                wake_resident_blocks(integrator, ce.harmonics, ppl, block, wk->n_slices)));
  const int64_t gwaves = static_cast<int64_t>(grid) * wpb;  // moment columns
  const int ns = wk->n_slices;
  const int64_t groups = finalize_groups(gwaves);
  const int64_t cols = scratch_cols(gwaves);

  DeviceCtx& c = ctx_for(dev);
  std::lock_guard<std::mutex> lock(c.mu);
  int64_t rows = turns;
  if (mom) {
    rows = chunk_rows(turns, 1, cols, groups > 1);
    if (rows < 1) return fail(LTRK_ENOMEM, "scratch cap too small for %lld waves", (long long)gwaves);
  }
  const size_t part_bytes = mom ? static_cast<size_t>(rows) * 5 * cols * sizeof(double) : 0;
  // Scratch: the potential, the two parities' count buffers (turns
  // alternate), the centre and the moment partials, each starting on its own
  // 64 KiB. The count buffers take every block's atomic adds; next to the
  // potential or the partials they made every other turn up to 1.7x slower at
  // 1e7 particles with 4096 or more blocks, depending on where the partials
  // ended.
  const size_t hist_half = static_cast<size_t>(kWakeCountCopies) * kWakeCountStride(ns) *
                           sizeof(uint32_t);
  const size_t pot_bytes = static_cast<size_t>(ns) * sizeof(double);
  auto span = [](size_t x) { return (x + 65535) & ~static_cast<size_t>(65535); };
  const size_t off_p0 = span(pot_bytes);
  const size_t off_p1 = off_p0 + span(hist_half);
  const size_t off_cen = off_p1 + span(hist_half);
  const size_t off_part = off_cen + span(kCentreDoubles * sizeof(double));
  void* scratch = nullptr;
  if ((rc = ensure_scratch(c, s, off_part + part_bytes, &scratch))) return rc;
  char* base = static_cast<char*>(scratch);
  double* centre = mom ? reinterpret_cast<double*>(base + off_cen) : nullptr;

  double* host = nullptr;
  void* wtab = nullptr;
  if ((rc = stage_program(c, s, pot_bytes, &host, &wtab))) return rc;
  make_wake_table(*wk, d.beta, host);
  if ((rc = send_program(c, s, pot_bytes))) return rc;

  const double e_charge = 1.602176634e-19;
  const double q_mp = rf->ring.charge_e * e_charge * wk->intensity / static_cast<double>(n);
  WakeDev w;
  std::memset(&w, 0, sizeof(w));
  w.z_lo = wk->z_lo;
  w.dz = (wk->z_hi - wk->z_lo) / static_cast<double>(ns);
  w.per_dz = static_cast<double>(ns) / (wk->z_hi - wk->z_lo);
  w.kappa = rf->ring.charge_e * q_mp / (d.beta * rf->ring.p0c_eV);
  w.wtab = static_cast<const double*>(wtab);
  w.counts = reinterpret_cast<uint32_t*>(base + off_p0);
  w.clear = reinterpret_cast<uint32_t*>(base + off_p1);
  w.pot = reinterpret_cast<double*>(base);
  w.n_slices = ns;
  b.partials = mom ? reinterpret_cast<double*>(base + off_part) : nullptr;
  b.centre = centre;

  std::string key;
  key_add(key, 7);
  key_add(key, b);
  key_add(key, ce);
  key_add(key, w);
  key_add(key, plan);
  key_add(key, ppl);
  key_add(key, turns);
  key_add(key, mom);

  // A(t) kicks with turn t-1's potential and writes moment row t-1; row r
  // lives at r - c0 in the chunk [c0, c0 + rows) finalized once complete.
  // 2 turns + 2 launches, and a finalize after each chunk of rows.
  LaunchSeq seq(2 * turns + 2 + (mom ? (turns + rows - 1) / rows + 1 : 0), s);
  if (mom) {
    const CentreDev cd{z, dp, nullptr, nullptr, n, LTRK_F64, centre};
    seq.push({kTimeFinalize, [cd](hipStream_t st) { return launch_centre(cd, st); }});
  }
  // Turn launch i bins into the counts of parity i % 2; potential i reads them
  // and zeroes the other parity's, which launch i + 1 then bins into.
  auto parity_of = [&](int64_t i) {
    WakeDev wi = w;
    if (i % 2) std::swap(wi.counts, wi.clear);
    return wi;
  };
  int64_t launch_i = 0;
  auto turn_launch = [&](int phase, int64_t row) {
    const int32_t local = static_cast<int32_t>(row < 0 ? 0 : row % rows);
    const WakeDev wi = parity_of(launch_i);
    seq.push({kTimeTrack, [b, ce, wi, phase, local, block, grid, ppl](hipStream_t st) {
                     return launch_wake_turn(b, ce, wi, phase, local, ppl, block, grid, st);
                   }});
    if (mom && row >= 0 && (row % rows == rows - 1 || row == turns - 1)) {
      const int64_t c0 = row - row % rows;
      FinalizeDev f;
      std::memset(&f, 0, sizeof(f));
      f.partials = b.partials;
      f.stage = b.partials + rows * 5 * gwaves;
      f.waves = gwaves;
      f.groups = groups;
      f.n = n;
      f.out = mom + c0;
      f.centre = centre;
      f.rows = static_cast<int32_t>(row - c0 + 1);
      seq.push({kTimeFinalize, [f](hipStream_t st) { return launch_finalize_single(f, st); }});
    }
  };
  auto potential = [&]() {
    const WakeDev wi = parity_of(launch_i);
    seq.push({kTimeFinalize, [wi](hipStream_t st) { return launch_wake_potential(wi, st); }});
    ++launch_i;
  };
  seq.push({kTimeFinalize, [w](hipStream_t st) { return launch_wake_zero(w, st); }});
  turn_launch(0, -1);
  for (int64_t t = 1; t < turns; ++t) {
    potential();
    turn_launch(1, t - 1);
  }
  potential();
  turn_launch(2, turns - 1);
  return finish(c, key, seq, s, plan.use_graph != 0);
}

static int moments_single(const void* z, const void* dp, const void* zc, const void* dc,
                          int64_t n, int dtype, ltrk_moments* out, hipStream_t s) {
  int rc;
  if (n < 0) return fail(LTRK_EINVAL, "n must be >= 0");
  if ((rc = check_device_range(out, sizeof(ltrk_moments), "out"))) return rc;
  if (n == 0) {
    hipError_t e = launch_fill_nan(out, 1, s);
    return e == hipSuccess ? LTRK_OK : fail_hip(e, "fill moments");
  }
  const size_t bytes = static_cast<size_t>(n) * (dtype == LTRK_F64 ? 8 : 4);
  if ((rc = check_device_range(z, bytes, "z"))) return rc;
  if ((rc = check_device_range(dp, bytes, "dp"))) return rc;
  if (dtype == LTRK_F32C) {
    if ((rc = check_device_range(zc, bytes, "z_comp"))) return rc;
    if ((rc = check_device_range(dc, bytes, "dp_comp"))) return rc;
  }
  int dev = 0;
  if ((rc = current_device(&dev))) return rc;
  const int ppl = 4, block = 256;
  BunchDev b;
  std::memset(&b, 0, sizeof(b));
  b.z = const_cast<void*>(z);
  b.dp = const_cast<void*>(dp);
  b.z_comp = const_cast<void*>(zc);
  b.dp_comp = const_cast<void*>(dc);
  b.n = n;
  b.waves = waves_for(n, ppl);
  b.integrator = kMeasureOnly;
  b.dtype = dtype;
  b.turns = 1;
  b.active = 1;
  DeviceCtx& c = ctx_for(dev);
  std::lock_guard<std::mutex> lock(c.mu);
  void* scratch = nullptr;
  const size_t part = static_cast<size_t>(5) * scratch_cols(b.waves);
  if ((rc = ensure_scratch(c, s, (part + kCentreDoubles) * sizeof(double), &scratch)))
    return rc;
  b.partials = static_cast<double*>(scratch);
  double* centre = b.partials + part;
  b.centre = centre;
  hipError_t e = launch_centre(CentreDev{z, dp, zc, dc, n, dtype, centre}, s);
  if (e != hipSuccess) return fail_hip(e, "moments centre");
  e = launch_track_single(b, 0, ppl, block, s);
  if (e != hipSuccess) return fail_hip(e, "moments launch");
  FinalizeDev f;
  std::memset(&f, 0, sizeof(f));
  f.partials = b.partials;
  f.stage = b.partials + 5 * b.waves;
  f.waves = b.waves;
  f.groups = finalize_groups(b.waves);
  f.n = n;
  f.out = out;
  f.centre = centre;
  f.rows = 1;
  e = launch_finalize_single(f, s);
  return e == hipSuccess ? LTRK_OK : fail_hip(e, "moments finalize");
}

// ---------------------------------------------------------------------------
// Batched tracking

static int track_batched(const ltrk_bunch* bunches, int nb, int64_t turns, int integrator,
                         int dtype, hipStream_t s) {
  int rc;
  if (nb < 0 || (nb > 0 && !bunches)) return fail(LTRK_EINVAL, "invalid bunch table");
  if (!valid_integrator(integrator)) return fail(LTRK_EINVAL, "unknown integrator %d", integrator);
  if (!valid_dtype(dtype)) return fail(LTRK_EINVAL, "unknown dtype %d", dtype);
  if (turns < 0) return fail(LTRK_EINVAL, "turns must be >= 0");
  if (turns > INT32_MAX) return fail(LTRK_EINVAL, "turns must be < 2^31");
  if (nb > 65535) return fail(LTRK_EINVAL, "at most 65535 bunches per call");
  const size_t elem = dtype == LTRK_F64 ? 8 : 4;
  int64_t total_n = 0;
  for (int i = 0; i < nb; ++i) {
    const ltrk_bunch& b = bunches[i];
    if (b.n < 0) return fail(LTRK_EINVAL, "bunch %d: n < 0", i);
    if ((rc = validate_ring(&b.ring))) return fail(rc, "bunch %d: invalid ring", i);
    if (turns > 0 && b.moments &&
        (rc = check_device_range(b.moments, static_cast<size_t>(turns) * sizeof(ltrk_moments),
                                 "bunch moments")))
      return rc;
    if (b.n > 0 && turns > 0) {
      const size_t bytes = static_cast<size_t>(b.n) * elem;
      if ((rc = check_device_range(b.z, bytes, "bunch z"))) return rc;
      if ((rc = check_device_range(b.dp, bytes, "bunch dp"))) return rc;
      if (dtype == LTRK_F32C) {
        if ((rc = check_device_range(b.z_comp, bytes, "bunch z_comp"))) return rc;
        if ((rc = check_device_range(b.dp_comp, bytes, "bunch dp_comp"))) return rc;
      }
    }
    total_n += b.n;
  }
  if (turns == 0 || nb == 0) return LTRK_OK;
  if (stream_capturing(s))
    return fail(LTRK_EUNSUPPORTED,
                "a batched call cannot be captured: it uploads its bunch and tile tables");
  for (int i = 0; i < nb; ++i) {
    if (bunches[i].n == 0 && bunches[i].moments) {
      hipError_t e = launch_fill_nan(bunches[i].moments, turns, s);
      if (e != hipSuccess) return fail_hip(e, "fill moments");
    }
  }
  if (total_n == 0) return LTRK_OK;
  int dev = 0;
  if ((rc = current_device(&dev))) return rc;
  ltrk_plan plan = choose_plan(integrator, dtype, total_n, true);
  const int wpb = plan.block / kWave;

  std::vector<BunchDev> bd(nb);
  std::vector<TileDev> tiles;
  int64_t waves_mom = 0;  // scratch columns of bunches that want moments
  bool any_mom = false, two_stage = false;
  int64_t max_groups = 1;
  for (int i = 0; i < nb; ++i) {
    const ltrk_bunch& in = bunches[i];
    BunchDev& b = bd[i];
    std::memset(&b, 0, sizeof(b));
    b.z = in.z;
    b.dp = in.dp;
    b.z_comp = in.z_comp;
    b.dp_comp = in.dp_comp;
    b.n = in.n;
    b.waves = waves_for(in.n, plan.ppl);
    b.integrator = integrator;
    b.dtype = dtype;
    b.active = 1;
    make_coeffs(in.ring, integrator, &b.c);
    for (int64_t w0 = 0; w0 < b.waves; w0 += wpb) {
      if (w0 > INT32_MAX) return fail(LTRK_EINVAL, "bunch %d too large", i);
      tiles.push_back(TileDev{i, static_cast<int32_t>(w0)});
    }
    if (in.moments && in.n > 0) {
      waves_mom += scratch_cols(b.waves);
      any_mom = true;
      max_groups = std::max(max_groups, finalize_groups(b.waves));
      two_stage = two_stage || finalize_groups(b.waves) > 1;
    }
  }
  int64_t K = plan.turns_per_launch;
  int64_t rows = turns;
  if (any_mom) {
    rows = chunk_rows(turns, K, waves_mom, two_stage);
    if (rows < 1) return fail(LTRK_ENOMEM, "scratch cap too small for %lld waves", (long long)waves_mom);
    K = std::min<int64_t>(K, rows);
  }

  DeviceCtx& c = ctx_for(dev);
  std::lock_guard<std::mutex> lock(c.mu);
  void* scratch = nullptr;
  // partial regions of the bunches with moments, then their centres (2 each)
  const size_t part_doubles = static_cast<size_t>(rows) * 5 * waves_mom;
  if (any_mom && (rc = ensure_scratch(c, s, (part_doubles + 2 * static_cast<size_t>(nb)) *
                                                sizeof(double),
                                      &scratch)))
    return rc;
  // Per-bunch partial regions inside the scratch.
  std::vector<FinalizeDev> fin;
  int64_t off = 0;
  int max_rows = static_cast<int>(std::min<int64_t>(rows, turns));
  for (int i = 0; i < nb; ++i) {
    if (bunches[i].moments && bunches[i].n > 0) {
      bd[i].partials = static_cast<double*>(scratch) + off;
      bd[i].centre = static_cast<double*>(scratch) + part_doubles + 2 * i;
      FinalizeDev f;
      std::memset(&f, 0, sizeof(f));
      f.partials = bd[i].partials;
      f.stage = bd[i].partials + rows * 5 * bd[i].waves;
      f.waves = bd[i].waves;
      f.groups = finalize_groups(bd[i].waves);
      f.n = bd[i].n;
      f.out = bunches[i].moments;
      f.centre = bd[i].centre;
      f.rows = max_rows;
      fin.push_back(f);
      off += rows * 5 * scratch_cols(bd[i].waves);
    }
  }

  std::string key;
  key_add(key, 2);
  key_add(key, plan);
  key_add(key, turns);
  key_add(key, scratch);
  key.append(reinterpret_cast<const char*>(bd.data()), bd.size() * sizeof(BunchDev));
  for (const FinalizeDev& f : fin) key_add(key, f.out);

  // Device tables: found with a cached graph, else uploaded now.
  const int64_t expected = count_launches(turns, rows, K, fin.empty() ? 0 : 1) + 1;
  const bool graph_ok = plan.use_graph && s &&
                        expected <= static_cast<int64_t>(max_graph_launches());
  if (graph_ok) {
    const std::string gkey = graph_key(key);
    for (auto it = c.graphs.begin(); it != c.graphs.end(); ++it) {
      if (it->first == gkey) {
        c.graphs.splice(c.graphs.begin(), c.graphs, it);
        hipError_t e = launch_graph(it->second, s);
        return e == hipSuccess ? LTRK_OK : fail_hip(e, "hipGraphLaunch");
      }
    }
  }
  const size_t tb_bytes = bd.size() * sizeof(BunchDev);
  const size_t tt_bytes = tiles.size() * sizeof(TileDev);
  const size_t tf_bytes = std::max<size_t>(fin.size(), 1) * sizeof(FinalizeDev);
  void* tables = nullptr;
  hipError_t e = hipMalloc(&tables, tb_bytes + tt_bytes + tf_bytes + 512);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(LTRK_ENOMEM, "bunch tables");
  }
  char* base = static_cast<char*>(tables);
  BunchDev* d_b = reinterpret_cast<BunchDev*>(base);
  TileDev* d_t = reinterpret_cast<TileDev*>(base + ((tb_bytes + 255) & ~size_t(255)));
  FinalizeDev* d_f = reinterpret_cast<FinalizeDev*>(
      reinterpret_cast<char*>(d_t) + ((tt_bytes + 255) & ~size_t(255)));
  // Synchronous upload: the tables are then fixed for the life of the graph.
  if ((e = hipMemcpy(d_b, bd.data(), tb_bytes, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(d_t, tiles.data(), tt_bytes, hipMemcpyHostToDevice)) != hipSuccess ||
      (!fin.empty() &&
       (e = hipMemcpy(d_f, fin.data(), fin.size() * sizeof(FinalizeDev), hipMemcpyHostToDevice)) !=
           hipSuccess)) {
    hipFree(tables);
    return fail_hip(e, "upload bunch tables");
  }

  LaunchSeq seq(graph_ok ? 0 : expected, s);
  const int64_t ntiles = static_cast<int64_t>(tiles.size());
  const int nf = static_cast<int>(fin.size());
  if (nf > 0)
    seq.push({kTimeFinalize, [=](hipStream_t st) { return launch_centre_bunches(d_b, nb, st); }});
  for (int64_t c0 = 0; c0 < turns; c0 += rows) {
    const int64_t len = std::min(rows, turns - c0);
    for (int64_t j = 0; j < len; j += K) {
      const int32_t tk = static_cast<int32_t>(std::min(K, len - j));
      const int32_t row0 = static_cast<int32_t>(j);
      const ltrk_plan p = plan;
      const bool m = any_mom;
      seq.push({kTimeTrack, [=](hipStream_t st) {
                       return launch_track_tiles(d_b, d_t, ntiles, integrator, dtype, tk, row0,
                                                 p.ppl, p.block, m, st);
                     }});
    }
    if (nf > 0) {
      const int mr = static_cast<int>(len);
      seq.push({kTimeFinalize, [=](hipStream_t st) {
                       return launch_finalize_multi(d_f, nf, mr, c0, max_groups, st);
                     }});
    }
  }
  if (!graph_ok) {
    e = seq.eager() ? seq.flush() : run_eager(seq.seq(), s);
    // tables are freed once the stream has consumed them
    hipError_t se = hipStreamSynchronize(s);
    hipFree(tables);
    if (e != hipSuccess) return fail_hip(e, "kernel launch");
    if (se != hipSuccess) return fail_hip(se, "batched run");
    return LTRK_OK;
  }
  GraphEntry* made = nullptr;
  rc = execute(c, key, seq.seq(), s, true, &made);
  if (rc || !made) {
    // failed, or run eagerly (capture unavailable): the tables are done with
    // once the stream is
    hipStreamSynchronize(s);
    hipFree(tables);
    return rc;
  }
  made->owned.push_back(tables);
  return LTRK_OK;
}

// ---------------------------------------------------------------------------
// Shutdown

static int shutdown_all() {
  std::lock_guard<std::mutex> g(g_ctx_mu);
  int prev = 0;
  hipGetDevice(&prev);
  for (auto& kv : g_ctx) {
    hipSetDevice(kv.first);
    hipDeviceSynchronize();
    DeviceCtx& c = *kv.second;
    std::lock_guard<std::mutex> lock(c.mu);
    clear_graphs(c);
    for (auto& sc : c.scratch)
      if (sc.second.ptr) hipFree(sc.second.ptr);
    c.scratch.clear();
    for (void* r : c.retired) hipFree(r);
    c.retired.clear();
    for (auto& pg : c.progs) {
      if (pg.second.dev) hipFree(pg.second.dev);
      if (pg.second.host) hipHostFree(pg.second.host);
      if (pg.second.copied) hipEventDestroy(pg.second.copied);
    }
    c.progs.clear();
  }
  g_ctx.clear();
  hipSetDevice(prev);
  std::lock_guard<std::mutex> t(g_time_mu);
  for (auto& tl : g_timed) {
    if (tl.owns_a) hipEventDestroy(tl.a);
    hipEventDestroy(tl.b);
  }
  g_timed.clear();
  for (hipEvent_t e : g_event_pool) hipEventDestroy(e);
  g_event_pool.clear();
  return LTRK_OK;
}

static int timing_take(ltrk_timing* out) {
  std::lock_guard<std::mutex> g(g_time_mu);
  ltrk_timing r{0, 0.0, 0, 0.0};
  int rc = LTRK_OK;
  for (auto& tl : g_timed) {
    hipError_t e = hipEventSynchronize(tl.b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, tl.a, tl.b);
    if (e != hipSuccess && rc == LTRK_OK) rc = fail_hip(e, "timing events");
    if (tl.kind == kTimeTrack) {
      r.track_launches += tl.count;
      r.track_ms += ms;
    } else {
      r.finalize_launches += tl.count;
      r.finalize_ms += ms;
    }
    if (tl.owns_a) g_event_pool.push_back(tl.a);
    g_event_pool.push_back(tl.b);
  }
  g_timed.clear();
  if (out) *out = r;
  return rc;
}

}  // namespace ltrk

// ---------------------------------------------------------------------------
// C ABI

using namespace ltrk;

#define LTRK_GUARD(body)                                      \
  try {                                                       \
    clear_error();                                            \
    body                                                      \
  } catch (const std::bad_alloc&) {                           \
    return fail(LTRK_ENOMEM, "host allocation failed");       \
  } catch (...) {                                             \
    return fail(LTRK_EDEVICE, "unexpected internal error");   \
  }

extern "C" {

int ltrk_abi_version(void) { return LTRK_ABI_VERSION; }

int ltrk_derive(const ltrk_ring* ring, ltrk_derived* out) {
  LTRK_GUARD({
    int rc = validate_ring(ring);
    if (rc) return rc;
    if (!out) return fail(LTRK_EINVAL, "out is NULL");
    derive(*ring, out);
    return LTRK_OK;
  })
}

int ltrk_track_f64(double* z, double* dp, int64_t n, int64_t turns, const ltrk_ring* ring,
                   int integrator, ltrk_moments* moments, void* stream) {
  LTRK_GUARD({
    return track_single(z, dp, nullptr, nullptr, n, turns, ring, integrator, LTRK_F64, moments,
                        static_cast<hipStream_t>(stream));
  })
}

int ltrk_track_f64_noalloc(double* z, double* dp, int64_t n, int64_t turns,
                           const ltrk_ring* ring, int integrator, ltrk_moments* moments,
                           void* stream) {
  LTRK_GUARD({
    return track_f64_noalloc(z, dp, n, turns, ring, integrator, moments,
                             static_cast<hipStream_t>(stream));
  })
}

int ltrk_track_f32c(float* z, float* dp, float* z_comp, float* dp_comp, int64_t n,
                    int64_t turns, const ltrk_ring* ring, int integrator, ltrk_moments* moments,
                    void* stream) {
  LTRK_GUARD({
    return track_single(z, dp, z_comp, dp_comp, n, turns, ring, integrator, LTRK_F32C, moments,
                        static_cast<hipStream_t>(stream));
  })
}

int ltrk_track_rf2_f64(double* z, double* dp, int64_t n, int64_t turns, const ltrk_rf2* rf,
                       int integrator, ltrk_moments* moments, void* stream) {
  LTRK_GUARD({
    if (!rf) return fail(LTRK_EINVAL, "rf2 is NULL");
    return track_single(z, dp, nullptr, nullptr, n, turns, &rf->ring, integrator, LTRK_F64,
                        moments, static_cast<hipStream_t>(stream), rf);
  })
}

int ltrk_track_program_f64(double* z, double* dp, int64_t n, int64_t turns, const ltrk_rf2* rf,
                           const ltrk_rf_turn* program, int integrator, ltrk_moments* moments,
                           void* stream) {
  LTRK_GUARD({
    if (!rf) return fail(LTRK_EINVAL, "rf2 is NULL");
    return track_single(z, dp, nullptr, nullptr, n, turns, &rf->ring, integrator, LTRK_F64,
                        moments, static_cast<hipStream_t>(stream), rf, program, true);
  })
}

int ltrk_track_6d_f64(double* z, double* dp, double* x, double* xp, double* y, double* yp,
                      int64_t n, int64_t turns, const ltrk_rf2* rf, const ltrk_twiss* twiss,
                      int integrator, ltrk_moments* moments, void* stream) {
  LTRK_GUARD({
    double* arr[6];
    arr[0] = z;
    arr[1] = dp;
    arr[2] = x;
    arr[3] = xp;
    arr[4] = y;
    arr[5] = yp;
    return track_6d(arr, n, turns, rf, twiss, integrator, moments,
                    static_cast<hipStream_t>(stream));
  })
}

int ltrk_track_wake_f64(double* z, double* dp, int64_t n, int64_t turns, const ltrk_rf2* rf,
                        const ltrk_wake* wake, int integrator, ltrk_moments* moments,
                        void* stream) {
  LTRK_GUARD({
    return track_wake(z, dp, n, turns, rf, wake, integrator, moments,
                      static_cast<hipStream_t>(stream));
  })
}

int ltrk_moments_f64(const double* z, const double* dp, int64_t n, ltrk_moments* out,
                     void* stream) {
  LTRK_GUARD({
    return moments_single(z, dp, nullptr, nullptr, n, LTRK_F64, out,
                          static_cast<hipStream_t>(stream));
  })
}

int ltrk_moments_f32c(const float* z, const float* dp, const float* z_comp,
                      const float* dp_comp, int64_t n, ltrk_moments* out, void* stream) {
  LTRK_GUARD({
    return moments_single(z, dp, z_comp, dp_comp, n, LTRK_F32C, out,
                          static_cast<hipStream_t>(stream));
  })
}

int ltrk_track_batched(const ltrk_bunch* bunches, int nb, int64_t turns, int integrator,
                       int dtype, void* stream) {
  LTRK_GUARD({
    return track_batched(bunches, nb, turns, integrator, dtype, static_cast<hipStream_t>(stream));
  })
}

int ltrk_timing_enable(int on) {
  LTRK_GUARD({
    std::lock_guard<std::mutex> g(g_time_mu);
    g_time_on = on != 0;
    return LTRK_OK;
  })
}

int ltrk_timing_take(ltrk_timing* out) {
  LTRK_GUARD({ return timing_take(out); })
}

const char* ltrk_strerror(int code) {
  switch (code) {
    case LTRK_OK: return "success";
    case LTRK_EINVAL: return "invalid argument";
    case LTRK_ENOMEM: return "out of memory";
    case LTRK_EDEVICE: return "device (HIP) error";
    case LTRK_EAGAIN: return "resource temporarily unavailable";
    case LTRK_EUNSUPPORTED: return "unsupported";
    default: return "unknown error code";
  }
}

int ltrk_last_error(char* buf, size_t len) {
  if (buf && len > 0) {
    std::strncpy(buf, t_err_msg, len - 1);
    buf[len - 1] = '\0';
  }
  return t_err_code;
}

int ltrk_shutdown(void) {
  LTRK_GUARD({ return shutdown_all(); })
}

}  // extern "C"
