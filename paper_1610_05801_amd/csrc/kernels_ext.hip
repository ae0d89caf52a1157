// HIP kernels of libltrk for the extended maps (gfx950):
//   - the double-harmonic RF map with RF phase offsets and a slip factor
//     eta0 + eta1 delta + eta2 delta^2 (two RF kicks and slip-factor and
//     phase evaluations per step, as the paper's hollow-bunch profile shows,
//     section 2.2);
//   - the same map under an RF programme: per-turn voltages, phases and
//     reference momentum from a device table of folded coefficients, read
//     with wave-uniform (scalar) loads once per turn;
//   - the 6-D map: the transverse linear one-turn map of section 1.1.1 with
//     chromatic phase advance, then the longitudinal step.
// They reuse the wave-tile loop, moment staging and flush of wave.h; the
// wave tile holding the end of a bunch runs with TAIL so that its padding
// lanes stay at zero (these maps do not keep (0, 0) fixed).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"
#include "ltrk_device.h"
#include "ltrk_device_ext.h"
#include "sinpi_coeffs.h"
#include "wave.h"

namespace ltrk {

static_assert(kSinPiTerms == kSinTerms, "sine polynomial length");

// ---------------------------------------------------------------------------
// One turn of the extended map, FP64 state.

__device__ __forceinline__ double drift_rf2(double z, double d, const double* __restrict__ nd) {
  const double t = __builtin_fma(__builtin_fma(nd[2], d, nd[1]), d, nd[0]);
  return __builtin_fma(t, d, z);
}

// delta + sum_i w A_i sin(k_i z + phi_i) for the kick weight index wk.
__device__ __forceinline__ double kick_rf2(double d, double z, const CoeffsRf2& c, int wk) {
  const KickTerms a = kick_terms(__builtin_fma(c.s[0], z, c.u0[0]), c.kq[wk][0]);
  double out = __builtin_fma(a.r, a.p, d);
  if (c.harmonics == 2) {
    const KickTerms b = kick_terms(__builtin_fma(c.s[1], z, c.u0[1]), c.kq[wk][1]);
    out = __builtin_fma(b.r, b.p, out);
  }
  return out;
}

__device__ __forceinline__ double force_rf2(double z, const CoeffsRf2& c) {
  return kick_rf2(0.0, z, c, 0);
}

__device__ __forceinline__ double slip_rf2(double d, const CoeffsRf2& c) {
  return drift_rf2(0.0, d, c.nd[0]);
}

template <int INTEG>
__device__ __forceinline__ void turn_rf2(double& z, double& d, const CoeffsRf2& c) {
  if constexpr (INTEG == kEulerCromer) {
    z = drift_rf2(z, d, c.nd[0]);
    d = kick_rf2(d, z, c, 0);
  } else if constexpr (INTEG == kLeapfrog) {
    z = drift_rf2(z, d, c.nd[0]);
    d = kick_rf2(d, z, c, 0);
    z = drift_rf2(z, d, c.nd[0]);
  } else if constexpr (INTEG == kRuth4) {
    z = drift_rf2(z, d, c.nd[0]);
    d = kick_rf2(d, z, c, 0);
    z = drift_rf2(z, d, c.nd[1]);
    d = kick_rf2(d, z, c, 1);
    z = drift_rf2(z, d, c.nd[1]);
    d = kick_rf2(d, z, c, 0);
    z = drift_rf2(z, d, c.nd[0]);
  } else if constexpr (INTEG == kRk4) {
    // slip and force with weight 1: nd[0] = -C eta_j, kq[0] = A_i x polynomial
    const double k1z = slip_rf2(d, c), k1d = force_rf2(z, c);
    const double k2z = slip_rf2(__builtin_fma(0.5, k1d, d), c);
    const double k2d = force_rf2(__builtin_fma(0.5, k1z, z), c);
    const double k3z = slip_rf2(__builtin_fma(0.5, k2d, d), c);
    const double k3d = force_rf2(__builtin_fma(0.5, k2z, z), c);
    const double k4z = slip_rf2(d + k3d, c), k4d = force_rf2(z + k3z, c);
    z = __builtin_fma(1.0 / 6.0, (k1z + 2.0 * k2z) + (2.0 * k3z + k4z), z);
    d = __builtin_fma(1.0 / 6.0, (k1d + 2.0 * k2d) + (2.0 * k3d + k4d), d);
  }
}

// Turn functors handed to the wave loop.
// Turn functor of the extended map.
template <int INTEG>
struct DoubleRf {
  const CoeffsRf2& c;
  __device__ __forceinline__ int at(int) const { return 0; }
  __device__ __forceinline__ void operator()(int, double& z, double& d) const {
    turn_rf2<INTEG>(z, d, c);
  }
};

// ---------------------------------------------------------------------------
// One turn of the extended map under an RF programme: `rec` is the turn's
// record (prog_layout(INTEG)): phase offsets, the eta0 part of each drift,
// the reference step of each kick and each kick's folded sine coefficients.
// The eta1, eta2 parts of the drifts and 2 h_i / C stay in CoeffsRf2. ACCEL
// adds the reference step delta <- (p / p') delta + (p - p') / p' to every
// kick; without it (constant momentum) a turn is bit for bit turn_rf2 with
// the record's settings.

template <int INTEG>
__device__ __forceinline__ double drift_prog(double z, double d, const CoeffsRf2& c,
                                             const double* __restrict__ rec, int j, int wi) {
  constexpr ProgLayout L = prog_layout(INTEG);
  const double t = __builtin_fma(__builtin_fma(c.nd[wi][2], d, c.nd[wi][1]), d, rec[L.nd + j]);
  return __builtin_fma(t, d, z);
}

template <int INTEG, bool ACCEL>
__device__ __forceinline__ double kick_prog(double d, double z, const CoeffsRf2& c,
                                            const double* __restrict__ rec, int j) {
  constexpr ProgLayout L = prog_layout(INTEG);
  double out = d;
  if constexpr (ACCEL) out = __builtin_fma(rec[L.ref + 2 * j], d, rec[L.ref + 2 * j + 1]);
  const KickTerms a =
      kick_terms(__builtin_fma(c.s[0], z, rec[L.u0]), rec + L.kq + (2 * j) * kSinTerms);
  out = __builtin_fma(a.r, a.p, out);
  if (c.harmonics == 2) {
    const KickTerms b =
        kick_terms(__builtin_fma(c.s[1], z, rec[L.u0 + 1]), rec + L.kq + (2 * j + 1) * kSinTerms);
    out = __builtin_fma(b.r, b.p, out);
  }
  return out;
}

template <int INTEG, bool ACCEL>
__device__ __forceinline__ void turn_prog(double& z, double& d, const CoeffsRf2& c,
                                          const double* __restrict__ rec) {
  if constexpr (INTEG == kEulerCromer) {
    z = drift_prog<INTEG>(z, d, c, rec, 0, 0);
    d = kick_prog<INTEG, ACCEL>(d, z, c, rec, 0);
  } else if constexpr (INTEG == kLeapfrog) {
    z = drift_prog<INTEG>(z, d, c, rec, 0, 0);
    d = kick_prog<INTEG, ACCEL>(d, z, c, rec, 0);
    z = drift_prog<INTEG>(z, d, c, rec, 1, 0);
  } else if constexpr (INTEG == kRuth4) {
    z = drift_prog<INTEG>(z, d, c, rec, 0, 0);
    d = kick_prog<INTEG, ACCEL>(d, z, c, rec, 0);
    z = drift_prog<INTEG>(z, d, c, rec, 1, 1);
    d = kick_prog<INTEG, ACCEL>(d, z, c, rec, 1);
    z = drift_prog<INTEG>(z, d, c, rec, 2, 1);
    d = kick_prog<INTEG, ACCEL>(d, z, c, rec, 2);
    z = drift_prog<INTEG>(z, d, c, rec, 3, 0);
  } else if constexpr (INTEG == kRk4) {
    // constant momentum: slip and force of weight 1
    const auto slip = [&](double v) { return drift_prog<INTEG>(0.0, v, c, rec, 0, 0); };
    const auto force = [&](double v) { return kick_prog<INTEG, false>(0.0, v, c, rec, 0); };
    const double k1z = slip(d), k1d = force(z);
    const double k2z = slip(__builtin_fma(0.5, k1d, d));
    const double k2d = force(__builtin_fma(0.5, k1z, z));
    const double k3z = slip(__builtin_fma(0.5, k2d, d));
    const double k3d = force(__builtin_fma(0.5, k2z, z));
    const double k4z = slip(d + k3d), k4d = force(z + k3z);
    z = __builtin_fma(1.0 / 6.0, (k1z + 2.0 * k2z) + (2.0 * k3z + k4z), z);
    d = __builtin_fma(1.0 / 6.0, (k1d + 2.0 * k2d) + (2.0 * k3d + k4d), d);
  }
}

// Turn functor of an RF programme: `prog` is the record of the launch's
// first turn.
template <int INTEG, bool ACCEL>
struct ProgRf {
  const CoeffsRf2& c;
  const double* __restrict__ prog;
  __device__ __forceinline__ const double* at(int t) const {
    return prog + static_cast<int64_t>(t) * prog_layout(INTEG).stride;
  }
  __device__ __forceinline__ void operator()(const double* rec, double& z, double& d) const {
    turn_prog<INTEG, ACCEL>(z, d, c, rec);
  }
};

// ---------------------------------------------------------------------------
// 6-D map: transverse Twiss rotation with chromatic phase, then the extended
// longitudinal step.

// sin(pi u) and cos(pi u) from one reduction: n = rint(u), r = u - n exact,
// sin(pi r) = r g(r^2) and cos(pi r) = sin(pi t) = t g(t^2) with t = 1/2 - |r|,
// both times (-1)^n.
__device__ __forceinline__ void sincos_pi(double u, double& s, double& c) {
  const double n = __builtin_rint(u);
  const double r = u - n;
  const double t = 0.5 - __builtin_fabs(r);
  const double r2 = r * r, t2 = t * t;
  double ps = kSinPiCoeff[kSinTerms - 1], pc = kSinPiCoeff[kSinTerms - 1];
#pragma unroll
  for (int j = kSinTerms - 2; j >= 0; --j) {
    ps = __builtin_fma(ps, r2, kSinPiCoeff[j]);
    pc = __builtin_fma(pc, t2, kSinPiCoeff[j]);
  }
  const double m = __builtin_fabs(n) + 0x1p52;
  const uint64_t odd = (__builtin_bit_cast(uint64_t, m) & 1ull) << 63;
  s = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, r * ps) ^ odd);
  c = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, t * pc) ^ odd);
}

__device__ __forceinline__ void rotate(double& u, double& v, double d, const PlaneDev& p) {
  double s, c;
  sincos_pi(__builtin_fma(p.u1, d, p.u0), s, c);
  const double a11 = __builtin_fma(p.alpha, s, c);
  const double a22 = __builtin_fma(-p.alpha, s, c);
  const double a12 = p.beta * s;
  const double a21 = p.neg_gamma * s;
  const double un = __builtin_fma(a11, u, a12 * v);
  v = __builtin_fma(a21, u, a22 * v);
  u = un;
}

// One wave tile of a 6-D bunch for `turns` turns: per turn the two
// transverse rotations with the turn's starting delta, then the extended
// longitudinal step; per-turn sums of the three planes (15 per lane) staged
// in the wave's LDS rows and flushed every kFlushTurns6d turns.
template <int INTEG, int P, bool MOM, bool TAIL>
__device__ __forceinline__ void wave_6d(const Bunch6Dev& b, const Coeffs6d& c, int64_t w,
                                        int turns, int row0, double* buf) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t first = w * static_cast<int64_t>(kWave * P) + lane;
  double* __restrict__ arr[6] = {b.z, b.dp, b.x, b.xp, b.y, b.yp};
  double s6[6][P];
  bool live[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int64_t i = first + static_cast<int64_t>(p) * kWave;
    live[p] = i < b.n;
#pragma unroll
    for (int k = 0; k < 6; ++k) s6[k][p] = i < b.n ? __builtin_nontemporal_load(&arr[k][i]) : 0.0;
  }
  double* out = MOM ? b.partials + static_cast<int64_t>(row0) * 15 * b.waves + w : nullptr;
  for (int t = 0; t < turns; t += kFlushTurns6d) {
    const int nb = turns - t < kFlushTurns6d ? turns - t : kFlushTurns6d;
    for (int j = 0; j < nb; ++j) {
      Sums sl{0.0, 0.0, 0.0, 0.0, 0.0}, sx{0.0, 0.0, 0.0, 0.0, 0.0}, sy{0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int p = 0; p < P; ++p) {
        if (!TAIL || live[p]) {
          rotate(s6[2][p], s6[3][p], s6[1][p], c.plane[0]);
          rotate(s6[4][p], s6[5][p], s6[1][p], c.plane[1]);
          turn_rf2<INTEG>(s6[0][p], s6[1][p], c.rf);
        }
        if constexpr (MOM) {
          accumulate(sl, s6[0][p], s6[1][p]);
          accumulate(sx, s6[2][p], s6[3][p]);
          accumulate(sy, s6[4][p], s6[5][p]);
        }
      }
      if constexpr (MOM) {
        stage_sums(buf, 3 * j + 0, sl, lane);
        stage_sums(buf, 3 * j + 1, sx, lane);
        stage_sums(buf, 3 * j + 2, sy, lane);
      }
    }
    if constexpr (MOM) {
      wave_sync();
      flush_rows(buf, nb * 15, out + static_cast<int64_t>(t) * 15 * b.waves, b.waves, lane);
      wave_sync();
    }
  }
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int64_t i = first + static_cast<int64_t>(p) * kWave;
    if (i < b.n) {
#pragma unroll
      for (int k = 0; k < 6; ++k) __builtin_nontemporal_store(s6[k][p], &arr[k][i]);
    }
  }
}

template <int INTEG, int P>
__global__ __launch_bounds__(kMaxBlock) void k_track_6d(Bunch6Dev b, Coeffs6d c, int32_t row0) {
  extern __shared__ double lds[];
  const int wib = threadIdx.x >> 6;
  const int64_t w = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + wib;
  if (w >= b.waves) return;
  double* buf = lds + wib * lds_doubles_per_wave_6d(b.turns);
  const bool tail = (w + 1) * static_cast<int64_t>(kWave * P) > b.n;
  if (b.partials) {
    if (tail)
      wave_6d<INTEG, P, true, true>(b, c, w, b.turns, row0, buf);
    else
      wave_6d<INTEG, P, true, false>(b, c, w, b.turns, row0, buf);
  } else {
    if (tail)
      wave_6d<INTEG, P, false, true>(b, c, w, b.turns, row0, buf);
    else
      wave_6d<INTEG, P, false, false>(b, c, w, b.turns, row0, buf);
  }
}

// ---------------------------------------------------------------------------
// Kernels of the extended map and the RF programme

template <int INTEG, int P, class Turn>
__device__ __forceinline__ void run_wave_ext(const BunchDev& b, const Turn& turn, int64_t w,
                                             int row0, double* buf) {
  const bool tail = (w + 1) * static_cast<int64_t>(kWave * P) > b.n;
  if (b.partials) {
    if (tail)
      wave_f64<INTEG, P, true, true>(b, turn, w, b.turns, row0, buf);
    else
      wave_f64<INTEG, P, true, false>(b, turn, w, b.turns, row0, buf);
  } else {
    if (tail)
      wave_f64<INTEG, P, false, true>(b, turn, w, b.turns, row0, buf);
    else
      wave_f64<INTEG, P, false, false>(b, turn, w, b.turns, row0, buf);
  }
}

// One bunch through the extended map (FP64 state).
template <int INTEG, int P>
__global__ __launch_bounds__(kMaxBlock) void k_track_rf2(BunchDev b, CoeffsRf2 c, int32_t row0) {
  extern __shared__ double lds[];
  const int wib = threadIdx.x >> 6;
  const int64_t w = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + wib;
  if (w >= b.waves) return;
  run_wave_ext<INTEG, P>(b, DoubleRf<INTEG>{c}, w, row0,
                         lds + wib * lds_doubles_per_wave(b.turns));
}

// One bunch through an RF programme; turn t of the launch reads record
// turn0 + t of `prog`.
template <int INTEG, int P, bool ACCEL>
__global__ __launch_bounds__(kMaxBlock) void k_track_prog(BunchDev b, CoeffsRf2 c,
                                                          const double* __restrict__ prog,
                                                          int32_t turn0, int32_t row0) {
  extern __shared__ double lds[];
  const int wib = threadIdx.x >> 6;
  const int64_t w = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + wib;
  if (w >= b.waves) return;
  const ProgRf<INTEG, ACCEL> turn{
      c, prog + static_cast<int64_t>(turn0) * prog_layout(INTEG).stride};
  run_wave_ext<INTEG, P>(b, turn, w, row0, lds + wib * lds_doubles_per_wave(b.turns));
}

// ---------------------------------------------------------------------------
// Host-side launchers

namespace {

using Rf2Fn = void (*)(BunchDev, CoeffsRf2, int32_t);
using ProgFn = void (*)(BunchDev, CoeffsRf2, const double*, int32_t, int32_t);
using SixdFn = void (*)(Bunch6Dev, Coeffs6d, int32_t);

template <int I>
Rf2Fn rf2_fn(int pi) {
  return pi == 0 ? k_track_rf2<I, 1>
       : pi == 1 ? k_track_rf2<I, 2>
       : pi == 2 ? k_track_rf2<I, 4>
                 : k_track_rf2<I, 8>;
}

template <int I, bool A>
ProgFn prog_fn(int pi) {
  return pi == 0 ? k_track_prog<I, 1, A>
       : pi == 1 ? k_track_prog<I, 2, A>
       : pi == 2 ? k_track_prog<I, 4, A>
                 : k_track_prog<I, 8, A>;
}

template <int I>
SixdFn sixd_fn(int pi) {
  return pi == 0 ? k_track_6d<I, 1>
       : pi == 1 ? k_track_6d<I, 2>
       : pi == 2 ? k_track_6d<I, 4>
                 : k_track_6d<I, 8>;
}

bool valid_block(int block) { return block > 0 && block <= kMaxBlock && block % kWave == 0; }

}  // namespace

hipError_t launch_track_rf2(const BunchDev& b, const CoeffsRf2& c, int32_t row0, int ppl,
                            int block, hipStream_t s) {
  const int pi = ppl_index(ppl);
  if (pi < 0 || !valid_block(block)) return hipErrorInvalidValue;
  Rf2Fn fn = nullptr;
  switch (b.integrator) {
    case kEulerCromer: fn = rf2_fn<kEulerCromer>(pi); break;
    case kLeapfrog: fn = rf2_fn<kLeapfrog>(pi); break;
    case kRuth4: fn = rf2_fn<kRuth4>(pi); break;
    case kRk4: fn = rf2_fn<kRk4>(pi); break;
    default: return hipErrorInvalidValue;
  }
  const int wpb = block / kWave;
  const int64_t blocks = (b.waves + wpb - 1) / wpb;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(blocks)), dim3(block),
                     lds_bytes(block, b.partials != nullptr, b.turns), s, b, c, row0);
  return hipGetLastError();
}

hipError_t launch_track_prog(const BunchDev& b, const CoeffsRf2& c, const double* prog,
                             int32_t turn0, int32_t row0, int ppl, int block, bool accel,
                             hipStream_t s) {
  const int pi = ppl_index(ppl);
  if (pi < 0 || !valid_block(block) || !prog || turn0 < 0) return hipErrorInvalidValue;
  ProgFn fn = nullptr;
  switch (b.integrator) {
    case kEulerCromer: fn = accel ? prog_fn<kEulerCromer, true>(pi) : prog_fn<kEulerCromer, false>(pi); break;
    case kLeapfrog: fn = accel ? prog_fn<kLeapfrog, true>(pi) : prog_fn<kLeapfrog, false>(pi); break;
    case kRuth4: fn = accel ? prog_fn<kRuth4, true>(pi) : prog_fn<kRuth4, false>(pi); break;
    case kRk4:  // constant momentum only (checked by the host)
      if (accel) return hipErrorInvalidValue;
      fn = prog_fn<kRk4, false>(pi);
      break;
    default: return hipErrorInvalidValue;
  }
  const int wpb = block / kWave;
  const int64_t blocks = (b.waves + wpb - 1) / wpb;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(blocks)), dim3(block),
                     lds_bytes(block, b.partials != nullptr, b.turns), s, b, c, prog, turn0, row0);
  return hipGetLastError();
}

hipError_t launch_track_6d(const Bunch6Dev& b, const Coeffs6d& c, int32_t row0, int ppl,
                           int block, hipStream_t s) {
  const int pi = ppl_index(ppl);
  if (pi < 0 || !valid_block(block)) return hipErrorInvalidValue;
  SixdFn fn = nullptr;
  switch (b.integrator) {
    case kEulerCromer: fn = sixd_fn<kEulerCromer>(pi); break;
    case kLeapfrog: fn = sixd_fn<kLeapfrog>(pi); break;
    case kRuth4: fn = sixd_fn<kRuth4>(pi); break;
    case kRk4: fn = sixd_fn<kRk4>(pi); break;
    default: return hipErrorInvalidValue;
  }
  const int wpb = block / kWave;
  const int64_t blocks = (b.waves + wpb - 1) / wpb;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const size_t lds = b.partials ? static_cast<size_t>(wpb) * lds_doubles_per_wave_6d(b.turns) *
                                      sizeof(double)
                                : 0;
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(blocks)), dim3(block), lds, s, b, c, row0);
  return hipGetLastError();
}

}  // namespace ltrk
