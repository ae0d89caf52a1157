// Device building blocks shared by the kernel files of libltrk: the sine
// terms of the RF kick, per-turn moment sums staged in the wave's LDS rows
// and flushed without block barriers, and the FP64 wave-tile loop over a
// turn map. Host helpers for launch shapes at the end.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ltrk_device.h"

namespace ltrk {

// ---------------------------------------------------------------------------
// Elementary operations

// Kick terms for phase u (in half revolutions): returns r' and p with
// r' * p = (scale) * sin(pi u), where q holds scale * kSinPiCoeff. n = rint(u),
// r = u - n is exact (|r| <= 1/2), p = sum_j q[j] r^2j, and the sign (-1)^n is
// applied to r: for |n| < 2^52 the parity of n is the last mantissa bit of
// |n| + 2^52; larger |u| has r = 0, where the sign is moot.
struct KickTerms {
  double r, p;
};

__device__ __forceinline__ KickTerms kick_terms(double u, const double* __restrict__ q) {
  const double n = __builtin_rint(u);
  const double r = u - n;
  const double s = r * r;
  double p = q[kSinTerms - 1];
#pragma unroll
  for (int j = kSinTerms - 2; j >= 0; --j) p = __builtin_fma(p, s, q[j]);
  const double t = __builtin_fabs(n) + 0x1p52;
  const uint64_t odd = (__builtin_bit_cast(uint64_t, t) & 1ull) << 63;
  return KickTerms{__builtin_bit_cast(double, __builtin_bit_cast(uint64_t, r) ^ odd), p};
}

// scale * sin(pi u) as one product.
__device__ __forceinline__ double scaled_sin(double u, const double* __restrict__ q) {
  const KickTerms k = kick_terms(u, q);
  return k.r * k.p;
}

// delta + scale * sin(pi u) with the last product fused into the update.
__device__ __forceinline__ double kicked(double d, double u, const double* __restrict__ q) {
  const KickTerms k = kick_terms(u, q);
  return __builtin_fma(k.r, k.p, d);
}

// Kahan-compensated x += inc with the running compensation c (value = x - c).
// ---------------------------------------------------------------------------
// Moment sums

struct Sums {
  double z, zz, d, dd, zd;
};

__device__ __forceinline__ void accumulate(Sums& s, double z, double d) {
  s.z += z;
  s.zz = __builtin_fma(z, z, s.zz);
  s.d += d;
  s.dd = __builtin_fma(d, d, s.dd);
  s.zd = __builtin_fma(z, d, s.zd);
}

// Wave-scope ordering of LDS accesses (all lanes of one wave; no block barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void stage_sums(double* buf, int j, const Sums& s, int lane) {
  double* r = buf + j * 5 * kRowStride + lane;
  r[0 * kRowStride] = s.z;
  r[1 * kRowStride] = s.zz;
  r[2 * kRowStride] = s.d;
  r[3 * kRowStride] = s.dd;
  r[4 * kRowStride] = s.zd;
}

// Reduce `rows` staged LDS rows of 64 lane values each; row r goes to
// out[r * stride]. Row r is summed by kLanesPerRow lanes (r, r + R, r + 2R, ...
// with R = 64 / kLanesPerRow), each adding its 64 / kLanesPerRow consecutive
// values in a pairwise tree; the partial sums are then combined by xor
// shuffles over R, 2R, ..., which gives every lane of the row the same total.
__device__ __forceinline__ void flush_rows(const double* buf, int rows, double* out,
                                           int64_t stride, int lane) {
  constexpr int R = kWave / kLanesPerRow;   // row slots per flush
  constexpr int V = kWave / kLanesPerRow;   // values per lane
  static_assert(kFlushTurns * 5 <= R, "flush rows exceed row slots");
  const int row = lane & (R - 1);
  const int part = lane / R;
  double part_sum = 0.0;
  if (row < rows) {
    const double2* src = reinterpret_cast<const double2*>(buf + row * kRowStride + part * V);
    double q[V / 2];
#pragma unroll
    for (int j = 0; j < V / 2; ++j) {
      const double2 v = src[j];
      q[j] = v.x + v.y;
    }
#pragma unroll
    for (int w = V / 4; w >= 1; w >>= 1) {
#pragma unroll
      for (int j = 0; j < w; ++j) q[j] = q[2 * j] + q[2 * j + 1];
    }
    part_sum = q[0];
  }
  double x = part_sum;
#pragma unroll
  for (int off = R; off < kWave; off <<= 1) x = x + __shfl_xor(x, off);
  if (part == 0 && row < rows) out[static_cast<int64_t>(row) * stride] = x;
}

// LDS doubles per wave for a launch of `turns` turns (the row buffer holds at
// most kFlushTurns turns of 5 sums).
__host__ __device__ __forceinline__ int lds_doubles_per_wave(int turns) {
  return (turns < kFlushTurns ? (turns > 0 ? turns : 1) : kFlushTurns) * 5 * kRowStride;
}

// ---------------------------------------------------------------------------
// One wave tile for `turns` turns.

// A Turn functor gives per-turn data with at(t) (t counted from the launch's
// first turn; nothing for maps with fixed coefficients) and applies one turn
// with turn(data, z, d). TAIL marks the wave tile holding the end of the
// bunch: its lanes past n skip the map, so they stay at zero and add nothing
// to the moment sums (the single-harmonic map keeps (0, 0) fixed, so its
// kernels skip the check; maps with RF phase offsets or momentum steps move
// it).
template <int INTEG, int P, bool MOM, bool TAIL, class Turn>
__device__ __forceinline__ void wave_f64(const BunchDev& b, const Turn& turn, int64_t w,
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
  double* out = MOM ? b.partials + static_cast<int64_t>(row0) * 5 * b.waves + w : nullptr;
  for (int t = 0; t < turns; t += kFlushTurns) {
    const int nb = turns - t < kFlushTurns ? turns - t : kFlushTurns;
    for (int j = 0; j < nb; ++j) {
      const auto tc = turn.at(t + j);
      Sums s{0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int p = 0; p < P; ++p) {
        if constexpr (INTEG != kMeasureOnly) {
          if (!TAIL || live[p]) turn(tc, z[p], d[p]);
        }
        if constexpr (MOM) accumulate(s, z[p], d[p]);
      }
      if constexpr (MOM) stage_sums(buf, j, s, lane);
    }
    if constexpr (MOM) {
      wave_sync();
      flush_rows(buf, nb * 5, out + static_cast<int64_t>(t) * 5 * b.waves, b.waves, lane);
      wave_sync();
    }
  }
  if constexpr (INTEG != kMeasureOnly) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int64_t i = first + static_cast<int64_t>(p) * kWave;
      if (i < b.n) {
        __builtin_nontemporal_store(z[p], &zp[i]);
        __builtin_nontemporal_store(d[p], &dpp[i]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Launch-shape helpers (host)

// Index of a particles-per-lane value among the compiled ones (1, 2, 4, 8).
inline int ppl_index(int ppl) {
  switch (ppl) {
    case 1: return 0;
    case 2: return 1;
    case 4: return 2;
    case 8: return 3;
    default: return -1;
  }
}

// Dynamic LDS of a block of `block` threads whose waves stage moment rows.
inline size_t lds_bytes(int block, bool moments, int turns) {
  return moments ? static_cast<size_t>(block / kWave) * lds_doubles_per_wave(turns) *
                       sizeof(double)
                 : 0;
}

}  // namespace ltrk
