// Stage-major turn of the extended longitudinal map over the P particles of
// a lane, shared by the extended, programme, 6-D and wake kernels: each drift
// or kick stage runs over all P particles, so a stage's coefficients are
// loaded once per turn and stay live only for that stage; the number of RF
// harmonics is a template parameter (no branch in the particle loop). Per
// particle the operations do not depend on P or on the stage order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ltrk_device.h"
#include "ltrk_device_ext.h"
#include "wave.h"

namespace ltrk {

// ---------------------------------------------------------------------------
// Coefficient sources of a turn

// The extended map: fixed coefficients (kick j of Ruth4 uses weight index 1
// for the middle kick, 0 otherwise).
struct Rf2Src {
  const CoeffsRf2& c;
  __device__ __forceinline__ double nd0(int, int wi) const { return c.nd[wi][0]; }
  __device__ __forceinline__ const double* kq(int j, int h) const { return c.kq[j == 1 ? 1 : 0][h]; }
  __device__ __forceinline__ double u0(int h) const { return c.u0[h]; }
  __device__ __forceinline__ double r(int) const { return 1.0; }
  __device__ __forceinline__ double dr(int) const { return 0.0; }
};

// An RF programme: the turn's record (prog_layout(INTEG)) supplies the phase
// offsets, the eta0 part of each drift, each kick's reference step and its
// folded sine coefficients; the eta1, eta2 parts and 2 h_i / C stay in
// CoeffsRf2.
template <int INTEG>
struct ProgSrc {
  const double* __restrict__ rec;
  static constexpr ProgLayout L = prog_layout(INTEG);
  __device__ __forceinline__ double nd0(int j, int) const { return rec[L.nd + j]; }
  __device__ __forceinline__ const double* kq(int j, int h) const {
    return rec + L.kq + (2 * j + h) * kSinTerms;
  }
  __device__ __forceinline__ double u0(int h) const { return rec[L.u0 + h]; }
  __device__ __forceinline__ double r(int j) const { return rec[L.ref + 2 * j]; }
  __device__ __forceinline__ double dr(int j) const { return rec[L.ref + 2 * j + 1]; }
};

// ---------------------------------------------------------------------------
// One turn of the extended map over the P particles of a lane.
//   drift j (drift weight index wi): z += (n0 + n1 delta + n2 delta^2) delta
//   kick j: delta <- [ACCEL: r_j delta + dr_j] + sum_h kq_jh-polynomial of phase h
// H is the number of RF harmonics (1 or 2).

template <int H, int P, bool TAIL, class Src>
__device__ __forceinline__ void drift_stage(double (&z)[P], const double (&d)[P],
                                            const bool (&live)[P], const CoeffsRf2& c,
                                            const Src& src, int j, int wi) {
  const double n0 = src.nd0(j, wi), n1 = c.nd[wi][1], n2 = c.nd[wi][2];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    if (!TAIL || live[p]) {
      const double t = __builtin_fma(__builtin_fma(n2, d[p], n1), d[p], n0);
      z[p] = __builtin_fma(t, d[p], z[p]);
    }
  }
}

// The RF term of kick j at z added to `base`.
template <int H, class Src>
__device__ __forceinline__ double rf_terms(double base, double z, const CoeffsRf2& c,
                                           const Src& src, int j) {
  const KickTerms a = kick_terms(__builtin_fma(c.s[0], z, src.u0(0)), src.kq(j, 0));
  double out = __builtin_fma(a.r, a.p, base);
  if constexpr (H == 2) {
    const KickTerms b = kick_terms(__builtin_fma(c.s[1], z, src.u0(1)), src.kq(j, 1));
    out = __builtin_fma(b.r, b.p, out);
  }
  return out;
}

template <bool ACCEL, int H, int P, bool TAIL, class Src>
__device__ __forceinline__ void kick_stage(const double (&z)[P], double (&d)[P],
                                           const bool (&live)[P], const CoeffsRf2& c,
                                           const Src& src, int j) {
#pragma unroll
  for (int p = 0; p < P; ++p) {
    if (!TAIL || live[p]) {
      double base = d[p];
      if constexpr (ACCEL) base = __builtin_fma(src.r(j), d[p], src.dr(j));
      d[p] = rf_terms<H>(base, z[p], c, src, j);
    }
  }
}

template <int INTEG, bool ACCEL, int H, int P, bool TAIL, class Src>
__device__ __forceinline__ void turn_ext(double (&z)[P], double (&d)[P], const bool (&live)[P],
                                         const CoeffsRf2& c, const Src& src) {
  if constexpr (INTEG == kEulerCromer) {
    drift_stage<H, P, TAIL>(z, d, live, c, src, 0, 0);
    kick_stage<ACCEL, H, P, TAIL>(z, d, live, c, src, 0);
  } else if constexpr (INTEG == kLeapfrog) {
    drift_stage<H, P, TAIL>(z, d, live, c, src, 0, 0);
    kick_stage<ACCEL, H, P, TAIL>(z, d, live, c, src, 0);
    drift_stage<H, P, TAIL>(z, d, live, c, src, 1, 0);
  } else if constexpr (INTEG == kRuth4) {
    drift_stage<H, P, TAIL>(z, d, live, c, src, 0, 0);
    kick_stage<ACCEL, H, P, TAIL>(z, d, live, c, src, 0);
    drift_stage<H, P, TAIL>(z, d, live, c, src, 1, 1);
    kick_stage<ACCEL, H, P, TAIL>(z, d, live, c, src, 1);
    drift_stage<H, P, TAIL>(z, d, live, c, src, 2, 1);
    kick_stage<ACCEL, H, P, TAIL>(z, d, live, c, src, 2);
    drift_stage<H, P, TAIL>(z, d, live, c, src, 3, 0);
  } else if constexpr (INTEG == kRk4) {
    // constant momentum: slip and force of weight 1, particle by particle
    const double n0 = src.nd0(0, 0), n1 = c.nd[0][1], n2 = c.nd[0][2];
    const auto slip = [&](double v) {
      const double t = __builtin_fma(__builtin_fma(n2, v, n1), v, n0);
      return __builtin_fma(t, v, 0.0);
    };
    const auto force = [&](double v) { return rf_terms<H>(0.0, v, c, src, 0); };
#pragma unroll
    for (int p = 0; p < P; ++p) {
      if (!TAIL || live[p]) {
        const double zz = z[p], dd = d[p];
        const double k1z = slip(dd), k1d = force(zz);
        const double k2z = slip(__builtin_fma(0.5, k1d, dd));
        const double k2d = force(__builtin_fma(0.5, k1z, zz));
        const double k3z = slip(__builtin_fma(0.5, k2d, dd));
        const double k3d = force(__builtin_fma(0.5, k2z, zz));
        const double k4z = slip(dd + k3d), k4d = force(zz + k3z);
        z[p] = __builtin_fma(1.0 / 6.0, (k1z + 2.0 * k2z) + (2.0 * k3z + k4z), zz);
        d[p] = __builtin_fma(1.0 / 6.0, (k1d + 2.0 * k2d) + (2.0 * k3d + k4d), dd);
      }
    }
  }
}

}  // namespace ltrk
