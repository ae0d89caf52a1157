// Descriptors of the extended maps shared by kernels_ext.hip and the host
// runtime: the double-harmonic RF map with slip factor orders, per-turn RF
// programme records and the 6-D (transverse + longitudinal) map.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ltrk_device.h"

namespace ltrk {

// Coefficients of the extended map (double-harmonic RF with phase offsets,
// slip factor eta0 + eta1 delta + eta2 delta^2), derived on the host in FP64.
struct CoeffsRf2 {
  double s[2];                     // 2 h_i / C
  double u0[2];                    // phi_i / pi: phase offsets in half revolutions
  double kq[2][2][kSinTerms];      // [kick weight][harmonic]: w A_i x sin(pi r)/r polynomial
  double nd[2][3];                 // [drift weight][j]: -w C eta_j (drift: z += delta * sum_j nd_j delta^j)
  int32_t harmonics;               // 1 or 2
  int32_t pad;
};

// Record layout of an RF programme (doubles per turn), shared by the host
// that fills it and the kernel that reads it: the phase offsets, the eta0
// part of every drift, the reference step (p / p', (p - p') / p') of every
// kick, and every kick's folded sine coefficients per harmonic. Records are
// padded to a multiple of 8 doubles (64 B).
struct ProgLayout {
  int drifts, kicks;
  int u0, nd, ref, kq, stride;
};

__host__ __device__ constexpr ProgLayout prog_layout(int integrator) {
  const int drifts = integrator == kRuth4 ? 4 : integrator == kLeapfrog ? 2 : 1;
  const int kicks = integrator == kRuth4 ? 3 : 1;
  const int u0 = 0, nd = 2, ref = nd + drifts, kq = ref + 2 * kicks;
  const int size = kq + 2 * kicks * kSinTerms;
  return ProgLayout{drifts, kicks, u0, nd, ref, kq, (size + 7) / 8 * 8};
}

// Transverse plane of the 6-D map: phase in half revolutions
// u = u1 delta + u0 with u0 = 2 frac(Q), u1 = 2 Q'; Twiss matrix terms.
struct PlaneDev {
  double u0, u1;
  double alpha, beta, neg_gamma;
};

struct Coeffs6d {
  CoeffsRf2 rf;
  PlaneDev plane[2];  // x, y
};

// One bunch with a 6-D FP64 state of n particles.
struct Bunch6Dev {
  double* z;
  double* dp;
  double* x;
  double* xp;
  double* y;
  double* yp;
  double* partials;  // [rows][3][5][waves] per-wave sums of the launch's first row, or NULL
  const double* centre;  // (c_z, c_dp) of the (z, dp) sums, or NULL
  int64_t n;
  int64_t waves;     // ceil(n / (64 * ppl))
  int32_t turns;     // turns of this launch
  int32_t integrator;
};

// The 6-D map stages 15 sums per turn (5 per plane): 2 turns fill the 30 LDS
// rows that 6 turns of 5 sums fill for the longitudinal map.
constexpr int kFlushTurns6d = 2;

__host__ __device__ inline int lds_doubles_per_wave_6d(int turns) {
  return (turns < kFlushTurns6d ? (turns > 0 ? turns : 1) : kFlushTurns6d) * 15 * kRowStride;
}

// Longitudinal wake kick: uniform slices over [z_lo, z_lo + n_slices dz),
// the wake at the lags between slice centres, the slice counts of the last
// map step and the potential at the slice centres.
constexpr int kWakeMaxSlices = 4096;
constexpr int kWakeMaxBlocks = 8192;
constexpr int kWakeMinBlocks = 1024;  // blocks per round when the runtime cannot tell
constexpr int kWakePotThreads = 256;    // block of the potential kernel
constexpr int kWakePotSlices = 32;      // slices whose potential one block forms
constexpr int kWakeStageSlices = 2048;  // wake table staged in LDS up to this many slices
// The global slice counts are held in kWakeCountCopies copies, kWakeCountStride(n)
// counters apart; block b adds into copy b % kWakeCountCopies, which spreads
// the blocks' end-of-turn atomic adds over eight addresses per slice.
constexpr int kWakeCountCopies = 8;
__host__ __device__ constexpr int kWakeCountStride(int n_slices) { return (n_slices + 63) & ~63; }

struct WakeDev {
  double z_lo;
  double dz;
  double per_dz;         // n_slices / (z_hi - z_lo): slice coordinate per metre
  double kappa;          // q Q_mp / (beta p0 c): delta kick per volt of potential
  const double* wtab;    // [n_slices] W(m dz / (beta c)), W(0) half the limit
  uint32_t* counts;      // [kWakeCountCopies][stride] counts of the last map step: the
                         // buffer of this turn's parity (two alternate, turn by turn)
  uint32_t* clear;       // the other parity's buffer: the potential kernel zeroes it
                         // for the next map step
  double* pot;           // [n_slices] potential of the last counts
  int32_t n_slices;
  int32_t pad;
};

}  // namespace ltrk
