// Descriptors shared by the HIP kernels and the host runtime of libltrk.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ltrk.h"

namespace ltrk {

constexpr int kWave = 64;
// Turns whose per-lane moment sums are buffered in LDS before one cross-lane
// reduction ("flush"). Each of the 5 sums of a turn is reduced by 2 lanes
// holding 32 of the 64 lane values each, so a flush covers 6 turns x 5 sums =
// 30 rows on 60 lanes (measured ~3% faster than 3 turns on 4 lanes per row).
constexpr int kFlushTurns = 6;
constexpr int kLanesPerRow = 2;
constexpr int kRowStride = 66;  // doubles per LDS row: 64 lane values + 2 pad
constexpr int kLdsDoublesPerWave = kFlushTurns * 5 * kRowStride;
constexpr int kMaxBlock = 256;

enum Integrator : int32_t {
  kEulerCromer = LTRK_EULER_CROMER,
  kLeapfrog = LTRK_LEAPFROG,
  kRuth4 = LTRK_RUTH4,
  kRk4 = LTRK_RK4,
  kMeasureOnly = 7,  // no turn applied: moments of the current state
};
enum DType : int32_t { kF64 = LTRK_F64, kF32C = LTRK_F32C };

// Terms of the polynomial for sin(pi r) / r in r^2 (see sinpi_coeffs.h).
constexpr int kSinTerms = 8;

// |s z| below which a wave may reduce the RF phase from the unrounded
// product (the reduction itself holds to 2^51; a factor 2 of margin).
constexpr double kExactRange = 0x1p50;

// Per-bunch coefficients, derived on the host in FP64 once per call.
struct Coeffs {
  double half_rev_per_m;       // s = 2h/C: k z = pi * (s z)
  double nd[2];                // negated drift weights times D (scheme specific)
  double kq[2][kSinTerms];     // kick weight x A x the sin(pi r)/r polynomial: a kick is
                               // delta += r * sum_j kq[j] r^2j (scheme specific; RK4: kq[0]
                               // carries A)
  double neg_D;                // -D (RK4 field)
  double z_exact;              // 2^50 / s: the exact-product phase reduction holds for |z| below
  double reach_d, reach_k;     // per-turn bounds: |dz| <= reach_d (|delta| + reach_k),
                               // |d delta| <= reach_k (in_exact_range)
  float nd_f[2][2];            // nd split into FP32 hi + lo (F32C drift increments:
                               // fma(hi, v, lo * v) carries the coefficient to ~2^-48)
  float ka_f[2][2];            // kick weight x A x pi split into FP32 hi + lo (F32C
                               // kicks, the FP32 sine; RK4 F32C keeps the FP64 sine)
};

// One bunch as the kernels see it.
struct BunchDev {
  void* z;
  void* dp;
  void* z_comp;
  void* dp_comp;
  int64_t n;
  int64_t waves;      // ceil(n / (64 * ppl)) wave tiles
  double* partials;   // [rows][5][waves] per-wave moment sums of this launch's
                      // first turn row; NULL = no moments
  const double* centre;  // (c_z, c_dp) the moment sums are taken about (see
                         // k_centre), or NULL for (0, 0)
  Coeffs c;
  int32_t integrator;
  int32_t dtype;
  int32_t turns;      // turns of this launch (engine: min(k, turns left))
  int32_t active;     // engine: 0 = skip
};

// A block's unit of work in tiled launches: `waves_per_block` consecutive
// wave tiles of one bunch starting at wave0.
struct TileDev {
  int32_t bunch;
  int32_t wave0;
};

// Moment sums about a centre. One-pass moments from raw sums (sum z, sum z^2,
// ...) lose (|mean| / rms)^2 ulp of the variance to cancellation, so the
// sums are taken of z - c_z and dp - c_dp with a centre fixed for a whole
// call: the mean of an evenly strided sample of up to kCentreSample particles
// of the call's initial state (k_centre), used where it lies more than
// kCentreRatio sample rms from zero and (0, 0) elsewhere. A wave whose
// centre is (0, 0) runs the loop without the two subtractions.
constexpr int kCentreSample = 1024;
constexpr double kCentreRatio = 4.0;
constexpr int kCentreDoubles = 32;  // scratch doubles reserved per centre (256 B)

// Input of k_centre: one bunch's state and where its centre goes.
struct CentreDev {
  const void* z;
  const void* dp;
  const void* z_comp;  // F32C only
  const void* dp_comp;
  int64_t n;
  int32_t dtype;
  double* out;  // (c_z, c_dp)
};

// Per-wave partial sums are added over wave tiles in groups of kGroupWaves;
// a bunch with more wave tiles than that is reduced in two stages (groups,
// then the group sums), so the order depends only on the number of tiles.
constexpr int kGroupWaves = 2048;

__host__ __device__ inline int64_t finalize_groups(int64_t waves) {
  return waves <= kGroupWaves ? 1 : (waves + kGroupWaves - 1) / kGroupWaves;
}

// Finalize work: reduce rows of per-wave partial sums of one bunch.
struct FinalizeDev {
  const double* partials;  // [rows][planes][5][waves], at this plane
  double* stage;           // [rows][5][groups] group sums when groups > 1
  int64_t waves;
  int64_t groups;
  int64_t n;
  ltrk_moments* out;
  const double* centre;  // the sums' centre (c_z, c_dp) of this plane, or NULL
  int32_t rows;
  int32_t planes;  // planes interleaved per row (0 or 1: one; the 6-D map: 3):
                   // partial rows are 5 * planes * waves apart, the plane's
                   // own sums start at `partials`, and row r is written to
                   // out[r * planes]
};

__host__ __device__ inline int planes_of(const FinalizeDev& f) {
  return f.planes > 1 ? f.planes : 1;
}

}  // namespace ltrk
