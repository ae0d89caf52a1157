// Device building blocks shared by the kernel files of libltrk: the sine
// terms of the RF kick, per-turn moment sums staged in the wave's LDS rows
// and flushed without block barriers, and the FP64 wave-tile loop over a
// turn map. Host helpers for launch shapes at the end.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ltrk_device.h"
#include "sinpi32_coeffs.h"

namespace ltrk {

// ---------------------------------------------------------------------------
// Elementary operations

// Kick terms: r' and p with r' * p = (scale) * sin(pi u) for a phase u in
// half revolutions, where q holds scale * kSinPiCoeff. n = rint(u), r = u - n
// (|r| <= 1/2), p = sum_j q[j] r^2j, and the sign (-1)^n is applied to r.
// Two reductions:
//   - kick_terms(u): u is a double; r = u - n is exact (Sterbenz). For
//     |n| < 2^52 the parity of n is the last mantissa bit of |n| + 2^52;
//     larger |u| are integers, r = 0 and the sign is moot. Exact for every
//     finite u.
//   - kick_terms_at(z, s): u = s z is never rounded on its own. t = s z +
//     1.5 * 2^52 in one FMA lands in [2^52, 2^53) for |s z| < 2^51, where
//     the doubles are the integers, so t = 1.5 * 2^52 + rint(s z) (ties to
//     even, 1.5 * 2^52 being even) and its last mantissa bit is the parity;
//     n = t - 1.5 * 2^52 is exact and r = s z - n takes a second FMA with one
//     rounding. Two instructions fewer than forming u first. Outside
//     |s z| < 2^51 r is unbounded, so callers use it only for waves whose
//     positions in_exact_range() has bounded for the whole launch.
constexpr double kRoundMagic = 0x1.8p52;

struct KickTerms {
  double r, p;
};

// r with its sign flipped when the last mantissa bit of t is set: that bit
// moved to bit 31 of r's high word and added there flips the sign (the carry
// out of the word is dropped). Written as one v_lshl_add_u32: from plain C++
// the compiler widens the add to 64 bits and spends four or five
// instructions on it.
struct Words {
  uint32_t lo, hi;
};

__device__ __forceinline__ double parity_signed(double r, double t) {
  Words w = __builtin_bit_cast(Words, r);
  const uint32_t tl = __builtin_bit_cast(Words, t).lo;
  uint32_t hi;
  asm("v_lshl_add_u32 %0, %1, 31, %2" : "=v"(hi) : "v"(tl), "v"(w.hi));
  w.hi = hi;
  return __builtin_bit_cast(double, w);
}

__device__ __forceinline__ KickTerms terms_of(double r, double t, const double* __restrict__ q) {
  const double s = r * r;
  double p = q[kSinTerms - 1];
#pragma unroll
  for (int j = kSinTerms - 2; j >= 0; --j) p = __builtin_fma(p, s, q[j]);
  return KickTerms{parity_signed(r, t), p};
}

// The reductions alone: r = u - n and a double t whose last mantissa bit is
// the parity of n.
struct Reduced {
  double r, t;
};

__device__ __forceinline__ Reduced reduce_u(double u) {
  const double n = __builtin_rint(u);
  return Reduced{u - n, __builtin_fabs(n) + 0x1p52};
}

__device__ __forceinline__ Reduced reduce_at(double z, double s) {
  const double t = __builtin_fma(z, s, kRoundMagic);
  const double n = t - kRoundMagic;
  return Reduced{__builtin_fma(z, s, -n), t};
}

template <bool EXACT>
__device__ __forceinline__ Reduced reduce_sz(double z, double s) {
  if constexpr (EXACT)
    return reduce_at(z, s);
  else
    return reduce_u(z * s);
}

__device__ __forceinline__ KickTerms kick_terms(double u, const double* __restrict__ q) {
  const Reduced x = reduce_u(u);
  return terms_of(x.r, x.t, q);
}

__device__ __forceinline__ KickTerms kick_terms_at(double z, double s,
                                                   const double* __restrict__ q) {
  const Reduced x = reduce_at(z, s);
  return terms_of(x.r, x.t, q);
}

// Kick terms of the phase s z by either reduction.
template <bool EXACT>
__device__ __forceinline__ KickTerms kick_terms_sz(double z, double s,
                                                   const double* __restrict__ q) {
  const Reduced x = reduce_sz<EXACT>(z, s);
  return terms_of(x.r, x.t, q);
}

// scale * sin(pi s z) as one product.
template <bool EXACT>
__device__ __forceinline__ double scaled_sin(double z, double s, const double* __restrict__ q) {
  const KickTerms k = kick_terms_sz<EXACT>(z, s, q);
  return k.r * k.p;
}

// delta + scale * sin(pi s z) with the last product fused into the update.
template <bool EXACT>
__device__ __forceinline__ double kicked(double d, double z, double s,
                                        const double* __restrict__ q) {
  const KickTerms k = kick_terms_sz<EXACT>(z, s, q);
  return __builtin_fma(k.r, k.p, d);
}

// The same sign flip on an FP32 value.
__device__ __forceinline__ float parity_signed(float v, double t) {
  const uint32_t tl = __builtin_bit_cast(Words, t).lo;
  uint32_t o;
  asm("v_lshl_add_u32 %0, %1, 31, %2" : "=v"(o) : "v"(tl), "v"(__builtin_bit_cast(uint32_t, v)));
  return __builtin_bit_cast(float, o);
}

// a * sin(pi s z) in FP32 from the FP64 phase reduction (the F32C kick): r is
// rounded to FP32 once, sin(pi r) / (pi r) comes from the FP32 polynomial of
// sinpi32_coeffs.h, and a = a[0] + a[1] (amplitude times pi as two FP32
// parts, so the kick strength itself is not rounded to FP32: a single FP32
// amplitude would shift the synchrotron tune by up to 2^-25 relative, a bias
// that does not average out over turns).
template <bool EXACT>
__device__ __forceinline__ float scaled_sin_f32(double z, double s, const float* __restrict__ a) {
  const Reduced x = reduce_sz<EXACT>(z, s);
  const float r = static_cast<float>(x.r);
  const float r2 = r * r;
  float p = kSinPi32Coeff[kSinPi32Terms - 1];
#pragma unroll
  for (int j = kSinPi32Terms - 2; j >= 0; --j) p = __builtin_fmaf(p, r2, kSinPi32Coeff[j]);
  const float v = parity_signed(r * p, x.t);
  return __builtin_fmaf(a[0], v, a[1] * v);
}

// Whether every position a wave reaches in a launch of `turns` turns keeps
// |s z| < 2^50, so its turns may use the exact-product reduction. Per turn a
// particle's momentum moves by at most reach_k and its position (also at the
// intermediate stages of a turn) by at most reach_d * (|delta| + reach_k), so
// after t < turns turns |z| <= |z0| + turns * reach_d * (|delta0| +
// turns * reach_k) (host: reach_d = |D| and reach_k = |A| times the summed
// absolute drift and kick weights of the scheme). Non-finite values fail the
// test. The result is the same for every lane of the wave.
template <int P>
__device__ __forceinline__ bool in_exact_range(const Coeffs& c, const double (&z)[P],
                                               const double (&d)[P], int turns) {
  const double k = static_cast<double>(turns);
  const double kd = k * c.reach_d;
  bool ok = true;
#pragma unroll
  for (int p = 0; p < P; ++p)
    ok = ok && __builtin_fma(kd, __builtin_fma(k, c.reach_k, __builtin_fabs(d[p])),
                             __builtin_fabs(z[p])) < c.z_exact;
  return __all(ok);
}

// ---------------------------------------------------------------------------
// Moment sums

struct Sums {
  double z, zz, d, dd, zd;
};

// The sums of a lane's first particle: what accumulate() into zero sums
// gives (up to the sign of a zero), without the additions of zero.
__device__ __forceinline__ Sums first_sums(double z, double d) {
  return Sums{z, z * z, d, d * d, z * d};
}

__device__ __forceinline__ void accumulate(Sums& s, double z, double d) {
  s.z += z;
  s.zz = __builtin_fma(z, z, s.zz);
  s.d += d;
  s.dd = __builtin_fma(d, d, s.dd);
  s.zd = __builtin_fma(z, d, s.zd);
}

// The centre (c_z, c_dp) of a call's moment sums (see kCentreSample).
struct Centre {
  double z, d;
};

__device__ __forceinline__ Centre centre_of(const double* c) {
  return c ? Centre{c[0], c[1]} : Centre{0.0, 0.0};
}

__device__ __forceinline__ bool is_zero(const Centre& c) { return c.z == 0.0 && c.d == 0.0; }

// Particle p's contribution to a lane's sums about the centre; SHIFT false
// skips the subtractions (the centre is then (0, 0): x - 0 is x exactly, so
// both forms give the same bits). The padding lanes past the end of a bunch
// hold (0, 0) and add nothing to sums about (0, 0); about another centre
// they would add -c, so in the wave tile that holds the end of the bunch
// (TAIL) they add zeros instead.
template <bool SHIFT, bool TAIL>
__device__ __forceinline__ void add_particle(Sums& s, int p, double z, double d,
                                             const Centre& c, bool live) {
  double zs = SHIFT ? z - c.z : z;
  double ds = SHIFT ? d - c.d : d;
  if constexpr (SHIFT && TAIL) {
    zs = live ? zs : 0.0;
    ds = live ? ds : 0.0;
  }
  if (p == 0)
    s = first_sums(zs, ds);
  else
    accumulate(s, zs, ds);
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
    // All LDS reads are issued before the first add (the scheduling barrier
    // keeps the compiler from interleaving them in groups of four, each
    // group waiting out the LDS latency: measured +3.5% on the fused kernel).
    double q[V / 2];
    double2 v[V / 2];
#pragma unroll
    for (int j = 0; j < V / 2; ++j) v[j] = src[j];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < V / 2; ++j) q[j] = v[j].x + v[j].y;
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

// Column of wave tile w in a row of per-wave partial sums (W tiles). A
// flush writes one double per (turn, moment) into the wave's column, so the
// 16 columns of a 128-B line are written by 16 different waves; with
// columns in wave order those came from four blocks on four XCDs (blocks go
// to the 8 XCDs in turn), each XCD's L2 holding and writing back a partial
// line. Columns are therefore dealt so that a line's 16 waves belong to
// blocks of 4 waves on one XCD: in each group of 128 tiles, tile r = 4b + i
// (block b = 8s + x of the group, wave i) takes column 16x + 4s + i. The
// order depends on w and W only (the finalize adds columns 0, 1, ... in
// order), so results stay the same for every launch shape; the last partial
// group keeps wave order.
__host__ __device__ __forceinline__ int64_t partial_col(int64_t w, int64_t W) {
  const int64_t full = W & ~int64_t(127);
  if (w >= full) return w;
  const int r = static_cast<int>(w & 127);
  const int b = r >> 2, i = r & 3;
  return (w - r) + ((b & 7) << 4) + ((b >> 3) << 2) + i;
}

// LDS doubles per wave for a launch of `turns` turns (the row buffer holds at
// most kFlushTurns turns of 5 sums).
__host__ __device__ __forceinline__ int lds_doubles_per_wave(int turns) {
  return (turns < kFlushTurns ? (turns > 0 ? turns : 1) : kFlushTurns) * 5 * kRowStride;
}

// ---------------------------------------------------------------------------
// One wave tile for `turns` turns.

// The turn loop of one wave tile over its P particles per lane, with the
// per-turn moment sums staged in LDS rows and flushed every kFlushTurns turns.
// A Turn functor gives per-turn data with at(t) (t counted from the launch's
// first turn; nothing for maps with fixed coefficients) and applies one turn
// with turn(data, z, d). TAIL marks the wave tile holding the end of the
// bunch: its lanes past n skip the map, so they stay at zero and add nothing
// to the moment sums (the single-harmonic map keeps (0, 0) fixed, so its
// kernels skip the check; maps with RF phase offsets or momentum steps move
// it).
template <int INTEG, int P, bool MOM, bool TAIL, bool SHIFT, class Turn>
__device__ __forceinline__ void turn_loop(const Turn& turn, double (&z)[P], double (&d)[P],
                                          const bool (&live)[P], int turns, double* buf,
                                          double* out, int64_t waves, int lane,
                                          const Centre& cen) {
  for (int t = 0; t < turns; t += kFlushTurns) {
    const int nb = turns - t < kFlushTurns ? turns - t : kFlushTurns;
    for (int j = 0; j < nb; ++j) {
      const auto tc = turn.at(t + j);
      Sums s;
#pragma unroll
      for (int p = 0; p < P; ++p) {
        if constexpr (INTEG != kMeasureOnly) {
          if (!TAIL || live[p]) turn(tc, z[p], d[p]);
        }
        if constexpr (MOM) add_particle<SHIFT, TAIL>(s, p, z[p], d[p], cen, live[p]);
      }
      if constexpr (MOM) stage_sums(buf, j, s, lane);
    }
    if constexpr (MOM) {
      wave_sync();
      flush_rows(buf, nb * 5, out + static_cast<int64_t>(t) * 5 * waves, waves, lane);
      wave_sync();
    }
  }
}

// One wave tile for `turns` turns: load, turn_loop, store. Exact is the turn
// functor for waves that in_exact_range() admits, Safe the one for the rest
// (the same type for maps with one reduction).
template <int INTEG, int P, bool MOM, bool TAIL, class Exact, class Safe>
__device__ __forceinline__ void wave_f64(const BunchDev& b, const Exact& exact, const Safe& safe,
                                         int64_t w, int turns, int row0, double* buf) {
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
  // the tile holding the end of the bunch masks its padding lanes out of
  // sums about a centre (add_particle)
  const bool tail = TAIL || (w + 1) * static_cast<int64_t>(kWave * P) > b.n;
  auto shifted = [&](const auto& turn) {
    if (tail)
      turn_loop<INTEG, P, MOM, true, true>(turn, z, d, live, turns, buf, out, b.waves, lane, cen);
    else
      turn_loop<INTEG, P, MOM, TAIL, true>(turn, z, d, live, turns, buf, out, b.waves, lane, cen);
  };
  if constexpr (INTEG == kMeasureOnly) {
    shifted(exact);
  } else {
    // The exact-product reduction with and without the centre, and the
    // rounded-phase reduction (rare: far-escaped particles) with it.
    if (in_exact_range<P>(b.c, z, d, turns)) {
      if (is_zero(cen))
        turn_loop<INTEG, P, MOM, TAIL, false>(exact, z, d, live, turns, buf, out, b.waves, lane,
                                              cen);
      else
        shifted(exact);
    } else {
      shifted(safe);
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

// Index of a particles-per-lane value among the compiled ones (1, 2, 4, 8;
// 16 for the single-bunch and tile kernels, not the extended-map, wake or
// engine kernels).
inline int ppl_index(int ppl) {
  switch (ppl) {
    case 1: return 0;
    case 2: return 1;
    case 4: return 2;
    case 8: return 3;
    case 16: return 4;
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
