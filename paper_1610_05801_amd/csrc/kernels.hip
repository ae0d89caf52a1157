// HIP kernels of libltrk for gfx950 (CDNA4): the single-harmonic map (FP64
// and FP32 + Kahan), batched and engine launches, and the moment finalize.
// The extended map, RF programmes and the 6-D map are in kernels_ext.hip;
// the shared wave-tile machinery is in wave.h.
//
// The hot path is the per-particle turn map of Oeftiger 2014, section 1.1.2
// (drift z -= w eta C delta, kick delta += w A sin(2 pi h z / C)) applied by
// one of four schemes, with the turn loop fused inside the kernel (the
// paper's "hybrid" design of section 2.3: a long enough in-register loop per
// thread, re-launched from the host to cover all turns).
//
// Layout and mapping (MI355X-first):
//   - state is structure-of-arrays in HBM; a wave tile owns 64 * P
//     consecutive particles, lane l holding particles tile + p*64 + l, so each
//     load/store instruction moves 64 consecutive elements; the state is read
//     and written with nontemporal hints (it streams: each element is touched
//     once per launch; measured +12% HBM throughput for one launch per turn
//     at 2.5e8 particles);
//   - P particles per lane give P independent dependency chains per lane
//     (ILP for the FP64 VALU, which is the bound once turns are fused);
//   - per-turn moment sums: each lane sums its P particles, the 5 lane sums
//     of a turn go to a per-wave LDS row buffer, and every kFlushTurns turns
//     the 30 rows (6 turns x 5 sums) are reduced by 2 lanes each and written
//     as one double per (turn, moment, wave) to HBM. No block barrier and no atomics are used,
//     so waves never wait on each other and every sum has a fixed order;
//   - a separate finalize kernel adds the per-wave sums of each turn in a
//     fixed order that depends only on the number of waves, so the moments
//     are bit-identical for any K, block size or batching with the same P.
//
// The RF kick evaluates sin(k z) as sin(pi u), u = (2h/C) z in half
// revolutions: n = rint(u), r = u - n with |r| <= 1/2, the polynomial of
// gen_sinpi.py (with the kick weight folded into its coefficients on the
// host) gives the scaled sin(pi r), and (-1)^n restores the sign. A wave
// whose positions stay below 2^50 C/(2h) in magnitude for the whole launch
// (in_exact_range, checked once after the load) reduces the product (2h/C) z
// without rounding it first, two FMAs giving n and r (exact_product); other
// waves round u first and reduce it exactly for any finite z. Both are
// branch-free, so particles that left the bucket (large z) cost the same as
// the core.
//
// All arithmetic is written with explicit fma(); the library is compiled with
// -ffp-contract=off so the rounding of every operation is fixed by the source.


#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "kernels.h"
#include "ltrk_device.h"
#include "wave.h"

namespace ltrk {

// ---------------------------------------------------------------------------
// FP32 + Kahan helper

__device__ __forceinline__ void kahan_add(float& x, float& c, float inc) {
  const float y = inc - c;
  const float t = x + y;
  c = (t - x) - y;
  x = t;
}

// ---------------------------------------------------------------------------
// One turn, FP64 state

template <int INTEG, bool EXACT>
__device__ __forceinline__ void turn_f64(double& z, double& d, const Coeffs& c) {
  const double s = c.half_rev_per_m;
  if constexpr (INTEG == kEulerCromer) {
    z = __builtin_fma(c.nd[0], d, z);
    d = kicked<EXACT>(d, z, s, c.kq[0]);
  } else if constexpr (INTEG == kLeapfrog) {
    z = __builtin_fma(c.nd[0], d, z);
    d = kicked<EXACT>(d, z, s, c.kq[0]);
    z = __builtin_fma(c.nd[0], d, z);
  } else if constexpr (INTEG == kRuth4) {
    z = __builtin_fma(c.nd[0], d, z);
    d = kicked<EXACT>(d, z, s, c.kq[0]);
    z = __builtin_fma(c.nd[1], d, z);
    d = kicked<EXACT>(d, z, s, c.kq[1]);
    z = __builtin_fma(c.nd[1], d, z);
    d = kicked<EXACT>(d, z, s, c.kq[0]);
    z = __builtin_fma(c.nd[0], d, z);
  } else if constexpr (INTEG == kRk4) {
    const double k1z = c.neg_D * d, k1d = scaled_sin<EXACT>(z, s, c.kq[0]);
    const double z2 = __builtin_fma(0.5, k1z, z), d2 = __builtin_fma(0.5, k1d, d);
    const double k2z = c.neg_D * d2, k2d = scaled_sin<EXACT>(z2, s, c.kq[0]);
    const double z3 = __builtin_fma(0.5, k2z, z), d3 = __builtin_fma(0.5, k2d, d);
    const double k3z = c.neg_D * d3, k3d = scaled_sin<EXACT>(z3, s, c.kq[0]);
    const double z4 = z + k3z, d4 = d + k3d;
    const double k4z = c.neg_D * d4, k4d = scaled_sin<EXACT>(z4, s, c.kq[0]);
    z = __builtin_fma(1.0 / 6.0, (k1z + 2.0 * k2z) + (2.0 * k3z + k4z), z);
    d = __builtin_fma(1.0 / 6.0, (k1d + 2.0 * k2d) + (2.0 * k3d + k4d), d);
  }
}

// ---------------------------------------------------------------------------
// One turn, FP32 + Kahan state. Drift increments are FP32 products of the FP32
// momentum value with the drift coefficient carried as an FP32 hi + lo pair (a
// coefficient rounded to FP32 alone would shift the synchrotron tune by up to
// 2^-25 relative, a systematic phase error). Kick increments take the phase
// reduction in FP64 from the FP64 value hi - comp and the sine in FP32
// (scaled_sin_f32). RK4 evaluates its stages, sine included, in FP64 from the
// FP64 state value and adds FP32-rounded increments.

template <int INTEG, bool EXACT>
__device__ __forceinline__ void turn_f32c(float& zh, float& zc, float& dh, float& dc,
                                          const Coeffs& c) {
  const double s = c.half_rev_per_m;
  auto drift = [&](const float* ndf) {
    const float v = dh - dc;
    kahan_add(zh, zc, __builtin_fmaf(ndf[0], v, ndf[1] * v));
  };
  auto kick = [&](const float* a) {
    const double zv = static_cast<double>(zh) - static_cast<double>(zc);
    kahan_add(dh, dc, scaled_sin_f32<EXACT>(zv, s, a));
  };
  if constexpr (INTEG == kEulerCromer) {
    drift(c.nd_f[0]);
    kick(c.ka_f[0]);
  } else if constexpr (INTEG == kLeapfrog) {
    drift(c.nd_f[0]);
    kick(c.ka_f[0]);
    drift(c.nd_f[0]);
  } else if constexpr (INTEG == kRuth4) {
    drift(c.nd_f[0]);
    kick(c.ka_f[0]);
    drift(c.nd_f[1]);
    kick(c.ka_f[1]);
    drift(c.nd_f[1]);
    kick(c.ka_f[0]);
    drift(c.nd_f[0]);
  } else if constexpr (INTEG == kRk4) {
    const double z = static_cast<double>(zh) - static_cast<double>(zc);
    const double d = static_cast<double>(dh) - static_cast<double>(dc);
    const double k1z = c.neg_D * d, k1d = scaled_sin<EXACT>(z, s, c.kq[0]);
    const double z2 = __builtin_fma(0.5, k1z, z), d2 = __builtin_fma(0.5, k1d, d);
    const double k2z = c.neg_D * d2, k2d = scaled_sin<EXACT>(z2, s, c.kq[0]);
    const double z3 = __builtin_fma(0.5, k2z, z), d3 = __builtin_fma(0.5, k2d, d);
    const double k3z = c.neg_D * d3, k3d = scaled_sin<EXACT>(z3, s, c.kq[0]);
    const double z4 = z + k3z, d4 = d + k3d;
    const double k4z = c.neg_D * d4, k4d = scaled_sin<EXACT>(z4, s, c.kq[0]);
    kahan_add(zh, zc, static_cast<float>((1.0 / 6.0) * ((k1z + 2.0 * k2z) + (2.0 * k3z + k4z))));
    kahan_add(dh, dc, static_cast<float>((1.0 / 6.0) * ((k1d + 2.0 * k2d) + (2.0 * k3d + k4d))));
  }
}

// Turn functor of the single-harmonic map for wave_f64 (EXACT: the
// exact-product phase reduction).
template <int INTEG, bool EXACT>
struct SingleRf {
  const Coeffs& c;
  __device__ __forceinline__ int at(int) const { return 0; }
  __device__ __forceinline__ void operator()(int, double& z, double& d) const {
    turn_f64<INTEG, EXACT>(z, d, c);
  }
};

template <int INTEG, int P, bool MOM>
__device__ __forceinline__ void wave_f32c(const BunchDev& b, int64_t w, int turns, int row0,
                                          double* buf) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t first = w * static_cast<int64_t>(kWave * P) + lane;
  float* __restrict__ zp = static_cast<float*>(b.z);
  float* __restrict__ dpp = static_cast<float*>(b.dp);
  float* __restrict__ zcp = static_cast<float*>(b.z_comp);
  float* __restrict__ dcp = static_cast<float*>(b.dp_comp);
  float zh[P], zc[P], dh[P], dc[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int64_t i = first + static_cast<int64_t>(p) * kWave;
    zh[p] = zc[p] = dh[p] = dc[p] = 0.0f;
    if (i < b.n) {
      zh[p] = __builtin_nontemporal_load(&zp[i]);
      zc[p] = __builtin_nontemporal_load(&zcp[i]);
      dh[p] = __builtin_nontemporal_load(&dpp[i]);
      dc[p] = __builtin_nontemporal_load(&dcp[i]);
    }
  }
  double* out = MOM ? b.partials + static_cast<int64_t>(row0) * 5 * b.waves +
                           partial_col(w, b.waves)
                     : nullptr;
  const Centre cen = MOM ? centre_of(b.centre) : Centre{0.0, 0.0};
  bool live[P];
#pragma unroll
  for (int p = 0; p < P; ++p) live[p] = first + static_cast<int64_t>(p) * kWave < b.n;
  const bool tail = (w + 1) * static_cast<int64_t>(kWave * P) > b.n;
  auto loop = [&](auto exact, auto shift, auto tail_tile) {
    constexpr bool EXACT = decltype(exact)::value;
    constexpr bool SHIFT = decltype(shift)::value;
    constexpr bool TAIL = decltype(tail_tile)::value;
    for (int t = 0; t < turns; t += kFlushTurns) {
      const int nb = turns - t < kFlushTurns ? turns - t : kFlushTurns;
      for (int j = 0; j < nb; ++j) {
        Sums s;
#pragma unroll
        for (int p = 0; p < P; ++p) {
          turn_f32c<INTEG, EXACT>(zh[p], zc[p], dh[p], dc[p], b.c);
          if constexpr (MOM) {
            const double zv = static_cast<double>(zh[p]) - static_cast<double>(zc[p]);
            const double dv = static_cast<double>(dh[p]) - static_cast<double>(dc[p]);
            add_particle<SHIFT, TAIL>(s, p, zv, dv, cen, live[p]);
          }
        }
        if constexpr (MOM) stage_sums(buf, j, s, lane);
      }
      if constexpr (MOM) {
        wave_sync();
        flush_rows(buf, nb * 5, out + static_cast<int64_t>(t) * 5 * b.waves, b.waves, lane);
        wave_sync();
      }
    }
  };
  // The phase is formed from hi - comp, within |hi| + |comp| of zero.
  double za[P], da[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    za[p] = __builtin_fabs(static_cast<double>(zh[p])) + __builtin_fabs(static_cast<double>(zc[p]));
    da[p] = __builtin_fabs(static_cast<double>(dh[p])) + __builtin_fabs(static_cast<double>(dc[p]));
  }
  auto shifted = [&](auto exact) {
    if (tail)
      loop(exact, std::true_type{}, std::true_type{});
    else
      loop(exact, std::true_type{}, std::false_type{});
  };
  if (in_exact_range<P>(b.c, za, da, turns)) {
    if (is_zero(cen))
      loop(std::true_type{}, std::false_type{}, std::false_type{});
    else
      shifted(std::true_type{});
  } else {
    shifted(std::false_type{});
  }
  if constexpr (INTEG != kMeasureOnly) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int64_t i = first + static_cast<int64_t>(p) * kWave;
      if (i < b.n) {
        __builtin_nontemporal_store(zh[p], &zp[i]);
        __builtin_nontemporal_store(zc[p], &zcp[i]);
        __builtin_nontemporal_store(dh[p], &dpp[i]);
        __builtin_nontemporal_store(dc[p], &dcp[i]);
      }
    }
  }
}

template <int INTEG, int DT, int P>
__device__ __forceinline__ void run_wave(const BunchDev& b, int64_t w, int turns, int row0,
                                         double* buf) {
  if constexpr (DT == kF64) {
    const SingleRf<INTEG, true> exact{b.c};
    const SingleRf<INTEG, false> safe{b.c};
    if (b.partials)
      wave_f64<INTEG, P, true, false>(b, exact, safe, w, turns, row0, buf);
    else
      wave_f64<INTEG, P, false, false>(b, exact, safe, w, turns, row0, buf);
  } else {
    if (b.partials)
      wave_f32c<INTEG, P, true>(b, w, turns, row0, buf);
    else
      wave_f32c<INTEG, P, false>(b, w, turns, row0, buf);
  }
}

// ---------------------------------------------------------------------------
// Kernels

// One bunch; block b covers wave tiles [b * wpb, (b+1) * wpb).
template <int INTEG, int DT, int P>
__global__ __launch_bounds__(kMaxBlock) void k_track_single(BunchDev b, int32_t row0) {
  extern __shared__ double lds[];
  const int wib = threadIdx.x >> 6;
  const int64_t w = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + wib;
  if (w >= b.waves) return;
  run_wave<INTEG, DT, P>(b, w, b.turns, row0, lds + wib * lds_doubles_per_wave(b.turns));
}

// One bunch through the extended map (FP64 state).
// Many bunches, one scheme and precision; block -> tiles[blockIdx.x].
template <int INTEG, int DT, int P>
__global__ __launch_bounds__(kMaxBlock) void k_track_tiles(const BunchDev* __restrict__ bunches,
                                                           const TileDev* __restrict__ tiles,
                                                           int32_t turns, int32_t row0) {
  extern __shared__ double lds[];
  const TileDev t = tiles[blockIdx.x];
  const BunchDev b = bunches[t.bunch];
  const int wib = threadIdx.x >> 6;
  const int64_t w = static_cast<int64_t>(t.wave0) + wib;
  if (w >= b.waves) return;
  run_wave<INTEG, DT, P>(b, w, turns, row0, lds + wib * lds_doubles_per_wave(turns));
}

// Engine step: every bunch carries its own scheme, precision and turn count.
template <int P>
__global__ __launch_bounds__(kMaxBlock) void k_track_mixed(const BunchDev* __restrict__ bunches,
                                                           const TileDev* __restrict__ tiles) {
  extern __shared__ double lds[];
  const TileDev t = tiles[blockIdx.x];
  const BunchDev b = bunches[t.bunch];
  const int wib = threadIdx.x >> 6;
  const int64_t w = static_cast<int64_t>(t.wave0) + wib;
  if (!b.active || w >= b.waves || b.turns <= 0) return;
  double* buf = lds + wib * kLdsDoublesPerWave;
  const int key = b.integrator * 2 + b.dtype;
  switch (key) {
    case kEulerCromer * 2 + kF64: run_wave<kEulerCromer, kF64, P>(b, w, b.turns, 0, buf); break;
    case kEulerCromer * 2 + kF32C: run_wave<kEulerCromer, kF32C, P>(b, w, b.turns, 0, buf); break;
    case kLeapfrog * 2 + kF64: run_wave<kLeapfrog, kF64, P>(b, w, b.turns, 0, buf); break;
    case kLeapfrog * 2 + kF32C: run_wave<kLeapfrog, kF32C, P>(b, w, b.turns, 0, buf); break;
    case kRuth4 * 2 + kF64: run_wave<kRuth4, kF64, P>(b, w, b.turns, 0, buf); break;
    case kRuth4 * 2 + kF32C: run_wave<kRuth4, kF32C, P>(b, w, b.turns, 0, buf); break;
    case kRk4 * 2 + kF64: run_wave<kRk4, kF64, P>(b, w, b.turns, 0, buf); break;
    case kRk4 * 2 + kF32C: run_wave<kRk4, kF32C, P>(b, w, b.turns, 0, buf); break;
    default: break;
  }
}

// Moments of rows of per-wave sums. One wave per row: lane l adds columns
// l, l + 64, ... in order, then a xor butterfly over the 64 lanes (every lane
// ends with the same, fixed-order total). `cols` are wave tiles (one stage)
// or group sums (second stage).
// `p` points at one row's 5 x cols sums, the result goes to *out.
__device__ __forceinline__ void finalize_row(const double* __restrict__ p, int64_t cols,
                                             int64_t n, const double* centre,
                                             ltrk_moments* out) {
  const int lane = threadIdx.x & (kWave - 1);
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t w = lane; w < cols; w += kWave) {
#pragma unroll
    for (int m = 0; m < 5; ++m) s[m] += p[m * cols + w];
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int m = 0; m < 5; ++m) s[m] += __shfl_xor(s[m], off);
  }
  if (lane == 0) {
    // sums of z - c_z and dp - c_dp: the means relative to the centre, then
    // the centre added back
    const double nd = static_cast<double>(n);
    const Centre c = centre_of(centre);
    const double mz = s[0] / nd;
    const double md = s[2] / nd;
    double vz = s[1] / nd - mz * mz;
    double vd = s[3] / nd - md * md;
    const double cov = s[4] / nd - mz * md;
    vz = vz > 0.0 ? vz : 0.0;
    vd = vd > 0.0 ? vd : 0.0;
    const double e2 = vz * vd - cov * cov;
    ltrk_moments o;
    o.mean_z = c.z == 0.0 ? mz : c.z + mz;
    o.rms_z = __builtin_sqrt(vz);
    o.mean_dp = c.d == 0.0 ? md : c.d + md;
    o.rms_dp = __builtin_sqrt(vd);
    o.emit_rms = __builtin_sqrt(e2 > 0.0 ? e2 : 0.0);
    *out = o;
  }
}

// First stage for bunches with more than kGroupWaves wave tiles: a block of
// 256 threads adds the per-wave sums of one (row, group) — thread t takes
// tiles t, t + 256, ... of the group in order, then a xor butterfly per wave
// and the 4 wave totals in a fixed pairwise order.
__device__ __forceinline__ void group_sum(const FinalizeDev& f, int row, int64_t g) {
  __shared__ double red[4][5];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid >> 6;
  const int64_t W = f.waves;
  const double* p = f.partials + static_cast<int64_t>(row) * 5 * planes_of(f) * W;
  const int64_t w0 = g * kGroupWaves;
  const int64_t w1 = w0 + kGroupWaves < W ? w0 + kGroupWaves : W;
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t w = w0 + tid; w < w1; w += 256) {
#pragma unroll
    for (int m = 0; m < 5; ++m) s[m] += p[m * W + w];
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int m = 0; m < 5; ++m) s[m] += __shfl_xor(s[m], off);
  }
  if (lane == 0) {
#pragma unroll
    for (int m = 0; m < 5; ++m) red[wave][m] = s[m];
  }
  __syncthreads();
  if (tid < 5)
    f.stage[(static_cast<int64_t>(row) * 5 + tid) * f.groups + g] =
        (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
}

__global__ __launch_bounds__(256) void k_group_single(FinalizeDev f) {
  group_sum(f, blockIdx.y, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_group_multi(const FinalizeDev* __restrict__ fs,
                                                     int32_t rows) {
  const FinalizeDev f = fs[blockIdx.z];
  const int row = blockIdx.y;
  if (f.out == nullptr || f.groups <= 1 || row >= rows || row >= f.rows ||
      static_cast<int64_t>(blockIdx.x) >= f.groups)
    return;
  group_sum(f, row, blockIdx.x);
}

// Row `row` of one bunch (or plane) into out[row * planes].
__device__ __forceinline__ void finalize_bunch_row(const FinalizeDev& f, ltrk_moments* out,
                                                   int row) {
  const int planes = planes_of(f);
  if (f.groups > 1)
    finalize_row(f.stage + static_cast<int64_t>(row) * 5 * f.groups, f.groups, f.n, f.centre,
                 out + static_cast<int64_t>(row) * planes);
  else
    finalize_row(f.partials + static_cast<int64_t>(row) * 5 * planes * f.waves, f.waves, f.n,
                 f.centre, out + static_cast<int64_t>(row) * planes);
}

__global__ __launch_bounds__(256) void k_finalize_single(FinalizeDev f) {
  const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row < f.rows) finalize_bunch_row(f, f.out, row);
}

// blockIdx.y selects the bunch; rows [0, min(rows, f.rows)) are reduced and
// written to f.out[(out_row0 + row) * planes].
__global__ __launch_bounds__(256) void k_finalize_multi(const FinalizeDev* __restrict__ fs,
                                                        int32_t rows, int64_t out_row0) {
  const FinalizeDev f = fs[blockIdx.y];
  const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (f.out == nullptr || row >= rows || row >= f.rows) return;
  finalize_bunch_row(f, f.out + out_row0 * planes_of(f), row);
}

// ---------------------------------------------------------------------------
// Centre of the moment sums (one block of 256 threads per bunch)

// Block-wide sum of one value per thread in a fixed order: xor butterfly in
// each wave, then the four wave totals pairwise. Every thread gets the total.
__device__ __forceinline__ double block_sum4(double x, double* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x = x + __shfl_xor(x, off);
  const int wave = threadIdx.x >> 6;
  __syncthreads();  // red may still be read from a previous call
  if ((threadIdx.x & (kWave - 1)) == 0) red[wave] = x;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// Mean and variance of an evenly strided sample of S = min(n, kCentreSample)
// particles (sample k is particle floor(k n / S)), two-pass; the centre is the
// sample mean where it lies more than kCentreRatio sample rms from zero, else
// 0 (also for a sample without spread, or a non-finite one). Every thread
// loads all of its samples before the first is used (lanes past S load
// particle 0 and are masked out of the sums), so the loads overlap.
__device__ void centre_block(const CentreDev& c) {
  __shared__ double red[4];
  constexpr int kPer = kCentreSample / 256;
  const int64_t S = c.n < kCentreSample ? c.n : kCentreSample;
  // floor(k n / S) = k q + floor(k r / S) with n = q S + r; k r < S^2 <= 2^20
  const int64_t q = c.n / S;
  const uint32_t r = static_cast<uint32_t>(c.n - q * S);
  const uint32_t s32 = static_cast<uint32_t>(S);
  int64_t idx[kPer];
  bool ok[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const uint32_t k = threadIdx.x + 256u * j;
    ok[j] = k < s32;
    idx[j] = ok[j] ? static_cast<int64_t>(k) * q + (k * r) / s32 : 0;
  }
  double zv[kPer], dv[kPer];
  if (c.dtype == kF64) {
    const double* z = static_cast<const double*>(c.z);
    const double* d = static_cast<const double*>(c.dp);
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      zv[j] = z[idx[j]];
      dv[j] = d[idx[j]];
    }
  } else {
    const float* zh = static_cast<const float*>(c.z);
    const float* zc = static_cast<const float*>(c.z_comp);
    const float* dh = static_cast<const float*>(c.dp);
    const float* dc = static_cast<const float*>(c.dp_comp);
    float a[kPer], b[kPer], e[kPer], f[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      a[j] = zh[idx[j]];
      b[j] = zc[idx[j]];
      e[j] = dh[idx[j]];
      f[j] = dc[idx[j]];
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      zv[j] = static_cast<double>(a[j]) - static_cast<double>(b[j]);
      dv[j] = static_cast<double>(e[j]) - static_cast<double>(f[j]);
    }
  }
  double sz = 0.0, sd = 0.0;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    sz += ok[j] ? zv[j] : 0.0;
    sd += ok[j] ? dv[j] : 0.0;
  }
  const double Sd = static_cast<double>(S);
  const double mz = block_sum4(sz, red) / Sd;
  const double md = block_sum4(sd, red) / Sd;
  double qz = 0.0, qd = 0.0;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    if (ok[j]) {
      qz = __builtin_fma(zv[j] - mz, zv[j] - mz, qz);
      qd = __builtin_fma(dv[j] - md, dv[j] - md, qd);
    }
  }
  const double vz = block_sum4(qz, red) / Sd;
  const double vd = block_sum4(qd, red) / Sd;
  constexpr double r2 = kCentreRatio * kCentreRatio;
  if (threadIdx.x == 0) {
    c.out[0] = (vz > 0.0 && mz * mz > r2 * vz && __builtin_isfinite(mz * mz)) ? mz : 0.0;
    c.out[1] = (vd > 0.0 && md * md > r2 * vd && __builtin_isfinite(md * md)) ? md : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_centre(CentreDev c) { centre_block(c); }

// Block b: the centre of bunches[b] when it computes moments.
__global__ __launch_bounds__(256) void k_centre_bunches(const BunchDev* __restrict__ bunches) {
  const BunchDev b = bunches[blockIdx.x];
  if (!b.partials || !b.centre || b.n <= 0) return;
  centre_block(CentreDev{b.z, b.dp, b.z_comp, b.dp_comp, b.n, b.dtype,
                         const_cast<double*>(b.centre)});
}

__global__ void k_fill_nan(ltrk_moments* out, int64_t rows) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < rows) {
    const double nan = __builtin_nan("");
    out[i] = ltrk_moments{nan, nan, nan, nan, nan};
  }
}

// Deterministic filler for the tuner's scratch particles.
__global__ void k_fill_probe(double* z, double* dp, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    z[i] = 1.0e-3 * static_cast<double>((i * 7919) % 1001 - 500);
    dp[i] = 2.0e-6 * static_cast<double>((i * 104729) % 1001 - 500);
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers

namespace {

using SingleFn = void (*)(BunchDev, int32_t);
using TilesFn = void (*)(const BunchDev*, const TileDev*, int32_t, int32_t);
using MixedFn = void (*)(const BunchDev*, const TileDev*);

// 16 particles per lane only for the FP64 state: its kernels take ~230 VGPRs
// and keep two waves per SIMD; the FP32 + Kahan kernels would take up to 268.
template <int I, int D>
SingleFn single_fn(int pi) {
  switch (pi) {
    case 0: return k_track_single<I, D, 1>;
    case 1: return k_track_single<I, D, 2>;
    case 2: return k_track_single<I, D, 4>;
    case 3: return k_track_single<I, D, 8>;
    case 4: return k_track_single<I, D, 16>;
    default: return nullptr;
  }
}

template <int I, int D>
TilesFn tiles_fn(int pi) {
  switch (pi) {
    case 0: return k_track_tiles<I, D, 1>;
    case 1: return k_track_tiles<I, D, 2>;
    case 2: return k_track_tiles<I, D, 4>;
    case 3: return k_track_tiles<I, D, 8>;
    case 4: return k_track_tiles<I, D, 16>;
    default: return nullptr;
  }
}

SingleFn pick_single(int integ, int dtype, int pi) {
  const bool f = dtype == kF64;
  switch (integ) {
    case kEulerCromer: return f ? single_fn<kEulerCromer, kF64>(pi) : single_fn<kEulerCromer, kF32C>(pi);
    case kLeapfrog: return f ? single_fn<kLeapfrog, kF64>(pi) : single_fn<kLeapfrog, kF32C>(pi);
    case kRuth4: return f ? single_fn<kRuth4, kF64>(pi) : single_fn<kRuth4, kF32C>(pi);
    case kRk4: return f ? single_fn<kRk4, kF64>(pi) : single_fn<kRk4, kF32C>(pi);
    case kMeasureOnly: return f ? single_fn<kMeasureOnly, kF64>(pi) : single_fn<kMeasureOnly, kF32C>(pi);
    default: return nullptr;
  }
}

TilesFn pick_tiles(int integ, int dtype, int pi) {
  const bool f = dtype == kF64;
  switch (integ) {
    case kEulerCromer: return f ? tiles_fn<kEulerCromer, kF64>(pi) : tiles_fn<kEulerCromer, kF32C>(pi);
    case kLeapfrog: return f ? tiles_fn<kLeapfrog, kF64>(pi) : tiles_fn<kLeapfrog, kF32C>(pi);
    case kRuth4: return f ? tiles_fn<kRuth4, kF64>(pi) : tiles_fn<kRuth4, kF32C>(pi);
    case kRk4: return f ? tiles_fn<kRk4, kF64>(pi) : tiles_fn<kRk4, kF32C>(pi);
    default: return nullptr;
  }
}

MixedFn pick_mixed(int pi) {
  switch (pi) {
    case 0: return k_track_mixed<1>;
    case 1: return k_track_mixed<2>;
    case 2: return k_track_mixed<4>;
    case 3: return k_track_mixed<8>;
    default: return nullptr;
  }
}

}  // namespace

hipError_t launch_track_single(const BunchDev& b, int32_t row0, int ppl, int block,
                               hipStream_t s) {
  const int pi = ppl_index(ppl);
  if (pi < 0 || block % kWave != 0 || block > kMaxBlock || block <= 0) return hipErrorInvalidValue;
  SingleFn fn = pick_single(b.integrator, b.dtype, pi);
  if (!fn) return hipErrorInvalidValue;
  const int wpb = block / kWave;
  const int64_t blocks = (b.waves + wpb - 1) / wpb;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(blocks)), dim3(block),
                     lds_bytes(block, b.partials != nullptr, b.turns), s, b, row0);
  return hipGetLastError();
}

hipError_t launch_track_tiles(const BunchDev* bunches, const TileDev* tiles, int64_t ntiles,
                              int integrator, int dtype, int32_t turns, int32_t row0, int ppl,
                              int block, bool moments, hipStream_t s) {
  const int pi = ppl_index(ppl);
  if (pi < 0 || block % kWave != 0 || block > kMaxBlock || block <= 0) return hipErrorInvalidValue;
  TilesFn fn = pick_tiles(integrator, dtype, pi);
  if (!fn) return hipErrorInvalidValue;
  if (ntiles <= 0) return hipSuccess;
  if (ntiles > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(ntiles)), dim3(block),
                     lds_bytes(block, moments, turns), s, bunches, tiles, turns, row0);
  return hipGetLastError();
}

hipError_t launch_track_mixed(const BunchDev* bunches, const TileDev* tiles, int64_t ntiles,
                              int ppl, int block, hipStream_t s) {
  const int pi = ppl_index(ppl);
  if (pi < 0 || block % kWave != 0 || block > kMaxBlock || block <= 0) return hipErrorInvalidValue;
  const MixedFn fn = pick_mixed(pi);
  if (!fn) return hipErrorInvalidValue;
  if (ntiles <= 0) return hipSuccess;
  if (ntiles > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(ntiles)), dim3(block),
                     lds_bytes(block, true, kFlushTurns), s, bunches, tiles);
  return hipGetLastError();
}

hipError_t launch_finalize_single(const FinalizeDev& f, hipStream_t s) {
  if (f.rows <= 0) return hipSuccess;
  if (f.groups > 1) {
    if (f.rows > 65535 || f.groups > 0x7fffffff || !f.stage) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_group_single, dim3(static_cast<unsigned>(f.groups), f.rows), dim3(256),
                       0, s, f);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int blocks = (f.rows + 3) / 4;
  hipLaunchKernelGGL(k_finalize_single, dim3(blocks), dim3(256), 0, s, f);
  return hipGetLastError();
}

hipError_t launch_finalize_multi(const FinalizeDev* fs, int nf, int rows, int64_t out_row0,
                                 int64_t max_groups, hipStream_t s) {
  if (nf <= 0 || rows <= 0) return hipSuccess;
  if (nf > 65535) return hipErrorInvalidValue;
  if (max_groups > 1) {
    if (rows > 65535 || max_groups > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_group_multi, dim3(static_cast<unsigned>(max_groups), rows, nf),
                       dim3(256), 0, s, fs, rows);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int blocks = (rows + 3) / 4;
  hipLaunchKernelGGL(k_finalize_multi, dim3(blocks, nf), dim3(256), 0, s, fs, rows, out_row0);
  return hipGetLastError();
}

hipError_t launch_centre(const CentreDev& c, hipStream_t s) {
  if (c.n <= 0 || !c.out) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_centre, dim3(1), dim3(256), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_centre_bunches(const BunchDev* bunches, int nb, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_centre_bunches, dim3(static_cast<unsigned>(nb)), dim3(256), 0, s, bunches);
  return hipGetLastError();
}

hipError_t launch_fill_nan(ltrk_moments* out, int64_t rows, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  const int64_t blocks = (rows + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fill_nan, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, out, rows);
  return hipGetLastError();
}

hipError_t launch_fill_probe(double* z, double* dp, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fill_probe, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, z, dp, n);
  return hipGetLastError();
}

}  // namespace ltrk
