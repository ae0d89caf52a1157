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
//
// A turn runs stage by stage over the P particles of a lane (turn_ext.h):
// all drifts of one stage, then all kicks of the next, so each stage's
// coefficients are loaded once per turn and stay in scalar registers (a
// particle-by-particle loop over a two-harmonic Ruth step needs ~100
// coefficients at once and re-loads them per particle).
//
// The wave tile that holds the end of a bunch runs with TAIL: its padding
// lanes skip the map (these maps do not keep (0, 0) fixed). Moments use the
// LDS row staging and flush of wave.h.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "kernels.h"
#include "ltrk_device.h"
#include "ltrk_device_ext.h"
#include "sinpi_coeffs.h"
#include "turn_ext.h"
#include "wave.h"

namespace ltrk {

static_assert(kSinPiTerms == kSinTerms, "sine polynomial length");

// Turn functors for wave_ext: at(t) gives the turn's data (t from the
// launch's first turn), all(data, z, d, live) applies one turn to P particles.
template <int INTEG, int H>
struct DoubleRf {
  const CoeffsRf2& c;
  __device__ __forceinline__ int at(int) const { return 0; }
  template <int P, bool TAIL>
  __device__ __forceinline__ void all(int, double (&z)[P], double (&d)[P],
                                      const bool (&live)[P]) const {
    turn_ext<INTEG, false, H, P, TAIL>(z, d, live, c, Rf2Src{c});
  }
};

template <int INTEG, bool ACCEL, int H>
struct ProgRf {
  const CoeffsRf2& c;
  const double* __restrict__ prog;  // record of the launch's first turn
  __device__ __forceinline__ const double* at(int t) const {
    return prog + static_cast<int64_t>(t) * prog_layout(INTEG).stride;
  }
  template <int P, bool TAIL>
  __device__ __forceinline__ void all(const double* rec, double (&z)[P], double (&d)[P],
                                      const bool (&live)[P]) const {
    turn_ext<INTEG, ACCEL, H, P, TAIL>(z, d, live, c, ProgSrc<INTEG>{rec});
  }
};

// One wave tile for `turns` turns (the FP64 wave loop of wave.h with a
// stage-major turn).
template <int P, bool MOM, bool TAIL, class Turn>
__device__ __forceinline__ void wave_ext(const BunchDev& b, const Turn& turn, int64_t w,
                                         int turns, int row0, double* buf) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t first = w * static_cast<int64_t>(kWave * P) + lane;
  double* __restrict__ zp = static_cast<double*>(b.z);
  double* __restrict__ dpp = static_cast<double*>(b.dp);
  double z[P], d[P];
  bool live[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int64_t i = first + static_cast<int64_t>(p) * kWave;
    z[p] = 0.0;
    d[p] = 0.0;
    live[p] = i < b.n;
    if (i < b.n) {
      z[p] = __builtin_nontemporal_load(&zp[i]);
      d[p] = __builtin_nontemporal_load(&dpp[i]);
    }
  }
  double* out = MOM ? b.partials + static_cast<int64_t>(row0) * 5 * b.waves +
                           partial_col(w, b.waves)
                     : nullptr;
  const Centre cen = MOM ? centre_of(b.centre) : Centre{0.0, 0.0};
  auto loop = [&](auto shift) {
    constexpr bool SHIFT = decltype(shift)::value;
    for (int t = 0; t < turns; t += kFlushTurns) {
      const int nb = turns - t < kFlushTurns ? turns - t : kFlushTurns;
      for (int j = 0; j < nb; ++j) {
        turn.template all<P, TAIL>(turn.at(t + j), z, d, live);
        if constexpr (MOM) {
          Sums s;
#pragma unroll
          for (int p = 0; p < P; ++p) add_particle<SHIFT, TAIL>(s, p, z[p], d[p], cen, live[p]);
          stage_sums(buf, j, s, lane);
        }
      }
      if constexpr (MOM) {
        wave_sync();
        flush_rows(buf, nb * 5, out + static_cast<int64_t>(t) * 5 * b.waves, b.waves, lane);
        wave_sync();
      }
    }
  };
  if (is_zero(cen))
    loop(std::false_type{});
  else
    loop(std::true_type{});
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int64_t i = first + static_cast<int64_t>(p) * kWave;
    if (i < b.n) {
      __builtin_nontemporal_store(z[p], &zp[i]);
      __builtin_nontemporal_store(d[p], &dpp[i]);
    }
  }
}

template <int P, class Turn>
__device__ __forceinline__ void run_wave_ext(const BunchDev& b, const Turn& turn, int64_t w,
                                             int row0, double* buf) {
  const bool tail = (w + 1) * static_cast<int64_t>(kWave * P) > b.n;
  if (b.partials) {
    if (tail)
      wave_ext<P, true, true>(b, turn, w, b.turns, row0, buf);
    else
      wave_ext<P, true, false>(b, turn, w, b.turns, row0, buf);
  } else {
    if (tail)
      wave_ext<P, false, true>(b, turn, w, b.turns, row0, buf);
    else
      wave_ext<P, false, false>(b, turn, w, b.turns, row0, buf);
  }
}

// ---------------------------------------------------------------------------
// 6-D map: transverse Twiss rotation with chromatic phase, then the extended
// longitudinal step.

// sin(pi u) and cos(pi u) from one reduction: n = rint(u), r = u - n exact,
// sin(pi r) = r g(r^2) and cos(pi r) = sin(pi t) = t g(t^2) with t = 1/2 - |r|,
// both times (-1)^n (the parity from the last mantissa bit of |n| + 2^52, as
// in kick_terms).
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
  s = parity_signed(r * ps, m);
  c = parity_signed(t * pc, m);
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
template <int INTEG, int H, int P, bool MOM, bool TAIL>
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
  const Rf2Src src{c.rf};
  double* out = MOM ? b.partials + static_cast<int64_t>(row0) * 15 * b.waves +
                           partial_col(w, b.waves)
                     : nullptr;
  // the (z, dp) sums about the call's centre (the transverse centroids turn
  // with the betatron phase, so no fixed centre follows them: theirs is 0)
  const Centre cen = MOM ? centre_of(b.centre) : Centre{0.0, 0.0};
  for (int t = 0; t < turns; t += kFlushTurns6d) {
    const int nb = turns - t < kFlushTurns6d ? turns - t : kFlushTurns6d;
    for (int j = 0; j < nb; ++j) {
#pragma unroll
      for (int p = 0; p < P; ++p) {
        if (!TAIL || live[p]) {
          rotate(s6[2][p], s6[3][p], s6[1][p], c.plane[0]);
          rotate(s6[4][p], s6[5][p], s6[1][p], c.plane[1]);
        }
      }
      turn_ext<INTEG, false, H, P, TAIL>(s6[0], s6[1], live, c.rf, src);
      if constexpr (MOM) {
        Sums sl, sx, sy;
#pragma unroll
        for (int p = 0; p < P; ++p) {
          add_particle<true, TAIL>(sl, p, s6[0][p], s6[1][p], cen, live[p]);
          add_particle<false, TAIL>(sx, p, s6[2][p], s6[3][p], cen, live[p]);
          add_particle<false, TAIL>(sy, p, s6[4][p], s6[5][p], cen, live[p]);
        }
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

// ---------------------------------------------------------------------------
// Kernels

// One bunch through the extended map (FP64 state).
template <int INTEG, int P, int H>
__global__ __launch_bounds__(kMaxBlock) void k_track_rf2(BunchDev b, CoeffsRf2 c, int32_t row0) {
  extern __shared__ double lds[];
  const int wib = threadIdx.x >> 6;
  const int64_t w = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + wib;
  if (w >= b.waves) return;
  run_wave_ext<P>(b, DoubleRf<INTEG, H>{c}, w, row0, lds + wib * lds_doubles_per_wave(b.turns));
}

// One bunch through an RF programme; turn t of the launch reads record
// turn0 + t of `prog`.
template <int INTEG, int P, bool ACCEL, int H>
__global__ __launch_bounds__(kMaxBlock) void k_track_prog(BunchDev b, CoeffsRf2 c,
                                                          const double* __restrict__ prog,
                                                          int32_t turn0, int32_t row0) {
  extern __shared__ double lds[];
  const int wib = threadIdx.x >> 6;
  const int64_t w = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + wib;
  if (w >= b.waves) return;
  const ProgRf<INTEG, ACCEL, H> turn{
      c, prog + static_cast<int64_t>(turn0) * prog_layout(INTEG).stride};
  run_wave_ext<P>(b, turn, w, row0, lds + wib * lds_doubles_per_wave(b.turns));
}

// One bunch with a 6-D state.
template <int INTEG, int P, int H>
__global__ __launch_bounds__(kMaxBlock) void k_track_6d(Bunch6Dev b, Coeffs6d c, int32_t row0) {
  extern __shared__ double lds[];
  const int wib = threadIdx.x >> 6;
  const int64_t w = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + wib;
  if (w >= b.waves) return;
  double* buf = lds + wib * lds_doubles_per_wave_6d(b.turns);
  const bool tail = (w + 1) * static_cast<int64_t>(kWave * P) > b.n;
  if (b.partials) {
    if (tail)
      wave_6d<INTEG, H, P, true, true>(b, c, w, b.turns, row0, buf);
    else
      wave_6d<INTEG, H, P, true, false>(b, c, w, b.turns, row0, buf);
  } else {
    if (tail)
      wave_6d<INTEG, H, P, false, true>(b, c, w, b.turns, row0, buf);
    else
      wave_6d<INTEG, H, P, false, false>(b, c, w, b.turns, row0, buf);
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers. The extended kernels are built for 4 and 8 particles
// per lane (the host raises smaller plans to 4) and 1 or 2 RF harmonics.

namespace {

using Rf2Fn = void (*)(BunchDev, CoeffsRf2, int32_t);
using ProgFn = void (*)(BunchDev, CoeffsRf2, const double*, int32_t, int32_t);
using SixdFn = void (*)(Bunch6Dev, Coeffs6d, int32_t);

template <int I, int H>
Rf2Fn rf2_fn(int ppl) {
  return ppl == 8 ? k_track_rf2<I, 8, H> : k_track_rf2<I, 4, H>;
}

template <int I, bool A, int H>
ProgFn prog_fn(int ppl) {
  return ppl == 8 ? k_track_prog<I, 8, A, H> : k_track_prog<I, 4, A, H>;
}

template <int I, int H>
SixdFn sixd_fn(int ppl) {
  return ppl == 8 ? k_track_6d<I, 8, H> : k_track_6d<I, 4, H>;
}

bool valid_block(int block) { return block > 0 && block <= kMaxBlock && block % kWave == 0; }

template <template <int, int> class Pick, class Fn>
Fn by_scheme(int integrator, int harmonics, int ppl) {
  const bool two = harmonics == 2;
  switch (integrator) {
    case kEulerCromer: return two ? Pick<kEulerCromer, 2>::get(ppl) : Pick<kEulerCromer, 1>::get(ppl);
    case kLeapfrog: return two ? Pick<kLeapfrog, 2>::get(ppl) : Pick<kLeapfrog, 1>::get(ppl);
    case kRuth4: return two ? Pick<kRuth4, 2>::get(ppl) : Pick<kRuth4, 1>::get(ppl);
    case kRk4: return two ? Pick<kRk4, 2>::get(ppl) : Pick<kRk4, 1>::get(ppl);
    default: return nullptr;
  }
}

template <int I, int H>
struct PickRf2 {
  static Rf2Fn get(int ppl) { return rf2_fn<I, H>(ppl); }
};
template <int I, int H>
struct PickSixd {
  static SixdFn get(int ppl) { return sixd_fn<I, H>(ppl); }
};
template <int I, int H>
struct PickProgAccel {
  static ProgFn get(int ppl) { return prog_fn<I, true, H>(ppl); }
};
template <int H>
struct PickProgAccel<kRk4, H> {  // RK4 has no reference step
  static ProgFn get(int) { return nullptr; }
};
template <int I, int H>
struct PickProgFlat {
  static ProgFn get(int ppl) { return prog_fn<I, false, H>(ppl); }
};

int64_t blocks_for(int64_t waves, int block) {
  const int wpb = block / kWave;
  return (waves + wpb - 1) / wpb;
}

}  // namespace

hipError_t launch_track_rf2(const BunchDev& b, const CoeffsRf2& c, int32_t row0, int ppl,
                            int block, hipStream_t s) {
  if ((ppl != 4 && ppl != 8) || !valid_block(block)) return hipErrorInvalidValue;
  Rf2Fn fn = by_scheme<PickRf2, Rf2Fn>(b.integrator, c.harmonics, ppl);
  if (!fn) return hipErrorInvalidValue;
  const int64_t blocks = blocks_for(b.waves, block);
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(blocks)), dim3(block),
                     lds_bytes(block, b.partials != nullptr, b.turns), s, b, c, row0);
  return hipGetLastError();
}

hipError_t launch_track_prog(const BunchDev& b, const CoeffsRf2& c, const double* prog,
                             int32_t turn0, int32_t row0, int ppl, int block, bool accel,
                             hipStream_t s) {
  if ((ppl != 4 && ppl != 8) || !valid_block(block) || !prog || turn0 < 0)
    return hipErrorInvalidValue;
  // RK4 has no reference step: constant momentum only (checked by the host)
  ProgFn fn = accel ? by_scheme<PickProgAccel, ProgFn>(b.integrator, c.harmonics, ppl)
                    : by_scheme<PickProgFlat, ProgFn>(b.integrator, c.harmonics, ppl);
  if (!fn) return hipErrorInvalidValue;
  const int64_t blocks = blocks_for(b.waves, block);
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(blocks)), dim3(block),
                     lds_bytes(block, b.partials != nullptr, b.turns), s, b, c, prog, turn0, row0);
  return hipGetLastError();
}

hipError_t launch_track_6d(const Bunch6Dev& b, const Coeffs6d& c, int32_t row0, int ppl,
                           int block, hipStream_t s) {
  if ((ppl != 4 && ppl != 8) || !valid_block(block)) return hipErrorInvalidValue;
  SixdFn fn = by_scheme<PickSixd, SixdFn>(b.integrator, c.rf.harmonics, ppl);
  if (!fn) return hipErrorInvalidValue;
  const int64_t blocks = blocks_for(b.waves, block);
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const size_t lds = b.partials ? static_cast<size_t>(block / kWave) *
                                      lds_doubles_per_wave_6d(b.turns) * sizeof(double)
                                : 0;
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(blocks)), dim3(block), lds, s, b, c, row0);
  return hipGetLastError();
}

}  // namespace ltrk
