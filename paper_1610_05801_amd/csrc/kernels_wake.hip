// HIP kernels of libltrk for the longitudinal wake kick (gfx950): the
// collective, memory-bound step that the paper's conclusion (section 3)
// names next after the single-particle tracking.
//
// Every turn needs the line density of the whole bunch after its map step,
// so a turn cannot stay inside one launch the way the single-particle map
// does; it is two launches:
//   k_wake_turn      streams the state once: applies the kick from the
//                    previous turn's potential, adds the moment sums of that
//                    turn, runs one step of the map and bins z into the
//                    block's LDS slice histogram, then adds the non-zero bins
//                    into its copy of the global slice counts (integer adds,
//                    so the counts do not depend on the order of the blocks);
//   k_wake_potential blocks of 32 slices add the copies of the counts into
//                    LDS and form the causal potential V_k = sum_{j >= k}
//                    count_j W_{j-k}, each sum split into 8 consecutive j
//                    ranges added in range order; two count buffers alternate
//                    from turn to turn, so these blocks also zero the other
//                    one for the next map step.
// k_wake_turn runs a grid-stride loop over wave tiles on a fixed grid, so a
// wave's tiles, and with them its moment sums, do not depend on timing.
// The state moves 32 B per particle-turn through HBM: the bound is HBM.

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

#include "kernels.h"
#include "ltrk_device.h"
#include "ltrk_device_ext.h"
#include "turn_ext.h"
#include "wave.h"

namespace ltrk {

// Slice coordinate of z: (z - z_lo) * per_dz, a difference and a product each
// rounded once; slice k holds the coordinates in [k, k + 1).
__device__ __forceinline__ double slice_coord(const WakeDev& w, double z) {
  return (z - w.z_lo) * w.per_dz;
}

// Slice of z, or -1 outside the slices (also for a non-finite z).
__device__ __forceinline__ int slice_of(const WakeDev& w, double z) {
  const double u = slice_coord(w, z);
  if (!(u >= 0.0)) return -1;
  const double f = __builtin_floor(u);
  return f < static_cast<double>(w.n_slices) ? static_cast<int>(f) : -1;
}

// Potential at z by linear interpolation between slice centres (constant
// beyond the first and last centre); pot is the block's LDS copy with one more
// entry, pot[n_slices] = pot[n_slices - 1]. Without branches: the centre
// coordinate is clamped to [0, n_slices - 1] (a NaN to 0), and at either end
// the weight of the neighbour is zero, so the result there is the end value
// itself, as the unclamped definition gives.
__device__ __forceinline__ double potential_at(const WakeDev& w, const double* pot, double z) {
  const double last = static_cast<double>(w.n_slices - 1);
  const double s = __builtin_fmin(__builtin_fmax(slice_coord(w, z) - 0.5, 0.0), last);
  const double k0 = __builtin_floor(s);
  const double f = s - k0;
  const int k = static_cast<int>(k0);
  return (1.0 - f) * pot[k] + f * pot[k + 1];
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x = x + __shfl_xor(x, off);
  return x;
}

// One turn of the wake path over the bunch.
//   KICK: delta -= kappa V(z) with V from w.pot (the previous histogram);
//   MOM:  moment sums of the state after the kick into row `row` of
//         b.partials ([rows][5][waves of this grid]);
//   STEP: one step of the extended map, then the slice histogram of the new
//         z added into w.counts.
template <int INTEG, int H, int P, bool KICK, bool MOM, bool STEP>
__global__ __launch_bounds__(kMaxBlock) void k_wake_turn(BunchDev b, CoeffsRf2 c, WakeDev w,
                                                         int32_t row) {
  extern __shared__ double lds[];
  const int ns = w.n_slices;
  double* pot = lds;                                           // ns + 1 doubles
  uint32_t* hist = reinterpret_cast<uint32_t*>(lds + ns + 1);  // ns + 1 counters, the last
                                                               // for particles outside
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wpb = blockDim.x >> 6;
  const int64_t grid_waves = static_cast<int64_t>(gridDim.x) * wpb;
  const int64_t gw = static_cast<int64_t>(blockIdx.x) * wpb + (tid >> 6);
  for (int k = tid; k <= ns; k += blockDim.x) {
    if constexpr (KICK) pot[k] = w.pot[k < ns ? k : ns - 1];
    if constexpr (STEP) hist[k] = 0u;
  }
  __syncthreads();
  double* __restrict__ zp = static_cast<double*>(b.z);
  double* __restrict__ dpp = static_cast<double*>(b.dp);
  Sums s{0.0, 0.0, 0.0, 0.0, 0.0};
  const Rf2Src src{c};
  const Centre cen = MOM ? centre_of(b.centre) : Centre{0.0, 0.0};
  // One wave tile; FULL: every particle of the tile is in the bunch, so no
  // lane needs a bounds check.
  auto tile_turn = [&](int64_t tile, auto full_tile) {
    constexpr bool FULL = decltype(full_tile)::value;
    const int64_t first = tile * static_cast<int64_t>(kWave * P) + lane;
    double z[P], d[P];
    bool live[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int64_t i = first + static_cast<int64_t>(p) * kWave;
      live[p] = FULL || i < b.n;
      if constexpr (FULL) {
        z[p] = __builtin_nontemporal_load(&zp[i]);
        d[p] = __builtin_nontemporal_load(&dpp[i]);
      } else {
        z[p] = live[p] ? __builtin_nontemporal_load(&zp[i]) : 0.0;
        d[p] = live[p] ? __builtin_nontemporal_load(&dpp[i]) : 0.0;
      }
    }
    if constexpr (KICK) {
      // particles outside the slices keep their momentum (a select, no branch)
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const double kicked = d[p] - w.kappa * potential_at(w, pot, z[p]);
        d[p] = live[p] && slice_of(w, z[p]) >= 0 ? kicked : d[p];
      }
    }
    if constexpr (MOM) {
      // about the call's centre (HBM-bound kernel: the subtractions cost no time)
#pragma unroll
      for (int p = 0; p < P; ++p)
        accumulate(s, live[p] ? z[p] - cen.z : 0.0, live[p] ? d[p] - cen.d : 0.0);
    }
    if constexpr (STEP) {
      turn_ext<INTEG, false, H, P, !FULL>(z, d, live, c, src);
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const int k = live[p] ? slice_of(w, z[p]) : -1;
        atomicAdd(&hist[k >= 0 ? k : ns], 1u);
      }
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int64_t i = first + static_cast<int64_t>(p) * kWave;
      if (FULL || live[p]) {
        if constexpr (STEP) __builtin_nontemporal_store(z[p], &zp[i]);
        if constexpr (KICK || STEP) __builtin_nontemporal_store(d[p], &dpp[i]);
      }
    }
  };
  for (int64_t tile = gw; tile < b.waves; tile += grid_waves) {
    if ((tile + 1) * static_cast<int64_t>(kWave * P) <= b.n)
      tile_turn(tile, std::true_type{});
    else
      tile_turn(tile, std::false_type{});
  }
  if constexpr (MOM) {
    const double t[5] = {wave_sum(s.z), wave_sum(s.zz), wave_sum(s.d), wave_sum(s.dd),
                         wave_sum(s.zd)};
    if (lane == 0) {
      double* out = b.partials + static_cast<int64_t>(row) * 5 * grid_waves + gw;
#pragma unroll
      for (int m = 0; m < 5; ++m) out[static_cast<int64_t>(m) * grid_waves] = t[m];
    }
  }
  if constexpr (STEP) {
    __syncthreads();
    // start each block at its own slice so that blocks finishing together
    // add into different counters
    const int rot = static_cast<int>((static_cast<int64_t>(blockIdx.x) * 61) % w.n_slices);
    uint32_t* counts =
        w.counts + (blockIdx.x % kWakeCountCopies) * kWakeCountStride(w.n_slices);
    for (int i = tid; i < w.n_slices; i += blockDim.x) {
      const int k = i + rot < w.n_slices ? i + rot : i + rot - w.n_slices;
      if (hist[k] != 0u) atomicAdd(&counts[k], hist[k]);
    }
  }
}

// The causal potential V_k = sum_{j >= k} count_j W_{j-k} from the slice
// counts of w.counts (the copies added and staged in LDS); the block of
// slices [k0, k0 + kWakePotSlices) needs the counts of slices k0 and up.
// Each slice's sum is split into 8 consecutive j ranges added by neighbouring
// threads, whose partial sums are then added in range order. The blocks also
// zero w.clear (the other parity's counts) for the next map step: nothing
// reads or writes that buffer while this kernel runs. The wake table is
// staged in LDS when it fits beside the counts.
__global__ __launch_bounds__(kWakePotThreads) void k_wake_potential(WakeDev w) {
  extern __shared__ double sh[];
  constexpr int kParts = kWakePotThreads / kWakePotSlices;  // 8
  const int ns = w.n_slices;
  const int k0 = static_cast<int>(blockIdx.x) * kWakePotSlices;
  const int m = ns - k0;                        // counts and lags this block needs
  const bool stage_w = ns <= kWakeStageSlices;
  double* cnt = sh;                             // counts of slices k0 .. ns - 1
  double* part = sh + m;                        // kWakePotThreads partial sums
  double* wl = part + kWakePotThreads;          // lags 0 .. m - 1 when staged
  const int stride = kWakeCountStride(ns);
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    uint64_t total = 0;
#pragma unroll
    for (int c = 0; c < kWakeCountCopies; ++c) total += w.counts[c * stride + k0 + i];
    cnt[i] = static_cast<double>(total);
    if (stage_w) wl[i] = w.wtab[i];
  }
  const int n_clear = kWakeCountCopies * stride;
  for (int i = static_cast<int>(blockIdx.x) * blockDim.x + threadIdx.x; i < n_clear;
       i += gridDim.x * blockDim.x)
    w.clear[i] = 0u;
  __syncthreads();
  const double* __restrict__ wt = stage_w ? wl : w.wtab;
  const int k = k0 + static_cast<int>(threadIdx.x) / kParts;   // this thread's slice
  const int q = static_cast<int>(threadIdx.x) % kParts;
  double v = 0.0;
  if (k < ns) {
    const int len = (ns - k + kParts - 1) / kParts;
    const int j0 = k + q * len;
    const int j1 = j0 + len < ns ? j0 + len : ns;
    for (int j = j0; j < j1; ++j) v = v + cnt[j - k0] * wt[j - k];
  }
  part[threadIdx.x] = v;
  __syncthreads();
  if (k < ns && q == 0) {
    double sum = part[threadIdx.x];
#pragma unroll
    for (int r = 1; r < kParts; ++r) sum = sum + part[threadIdx.x + r];
    w.pot[k] = sum;
  }
}

__global__ void k_wake_zero(uint32_t* counts, int32_t n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) counts[i] = 0u;
}

// ---------------------------------------------------------------------------
// Host-side launchers

namespace {

using TurnFn = void (*)(BunchDev, CoeffsRf2, WakeDev, int32_t);

template <int I, int H, bool KICK, bool MOM, bool STEP>
TurnFn turn_fn(int ppl) {
  return ppl == 8 ? k_wake_turn<I, H, 8, KICK, MOM, STEP> : k_wake_turn<I, H, 4, KICK, MOM, STEP>;
}

// phase 0: first turn (step only); 1: kick, moments, step; 2: last kick and moments.
template <int I, int H>
TurnFn by_phase(int phase, bool mom, int ppl) {
  if (phase == 0) return turn_fn<I, H, false, false, true>(ppl);
  if (phase == 1)
    return mom ? turn_fn<I, H, true, true, true>(ppl) : turn_fn<I, H, true, false, true>(ppl);
  return mom ? turn_fn<I, H, true, true, false>(ppl) : turn_fn<I, H, true, false, false>(ppl);
}

TurnFn pick_turn(int integ, int harmonics, int phase, bool mom, int ppl) {
  const bool two = harmonics == 2;
  switch (integ) {
    case kEulerCromer: return two ? by_phase<kEulerCromer, 2>(phase, mom, ppl) : by_phase<kEulerCromer, 1>(phase, mom, ppl);
    case kLeapfrog: return two ? by_phase<kLeapfrog, 2>(phase, mom, ppl) : by_phase<kLeapfrog, 1>(phase, mom, ppl);
    case kRuth4: return two ? by_phase<kRuth4, 2>(phase, mom, ppl) : by_phase<kRuth4, 1>(phase, mom, ppl);
    case kRk4: return two ? by_phase<kRk4, 2>(phase, mom, ppl) : by_phase<kRk4, 1>(phase, mom, ppl);
    default: return nullptr;
  }
}

}  // namespace

hipError_t launch_wake_turn(const BunchDev& b, const CoeffsRf2& c, const WakeDev& w, int phase,
                            int32_t row, int ppl, int block, int grid, hipStream_t s) {
  if ((ppl != 4 && ppl != 8) || block <= 0 || block > kMaxBlock || block % kWave != 0 ||
      grid <= 0 || grid > kWakeMaxBlocks || phase < 0 || phase > 2 || w.n_slices < 1 ||
      w.n_slices > kWakeMaxSlices)
    return hipErrorInvalidValue;
  const bool mom = b.partials != nullptr;
  TurnFn fn = pick_turn(b.integrator, c.harmonics, phase, mom, ppl);
  if (!fn) return hipErrorInvalidValue;
  // potential and histogram, each with one more entry (see k_wake_turn)
  const size_t lds = static_cast<size_t>(w.n_slices + 1) * (sizeof(double) + sizeof(uint32_t));
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(grid)), dim3(block), lds, s, b, c, w, row);
  return hipGetLastError();
}

int wake_resident_blocks(int integrator, int harmonics, int ppl, int block, int n_slices) {
  TurnFn fn = pick_turn(integrator, harmonics, 1, true, ppl);
  if (!fn || block <= 0) return 0;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  const size_t lds = static_cast<size_t>(n_slices + 1) * (sizeof(double) + sizeof(uint32_t));
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(fn),
                                                   block, lds) != hipSuccess)
    return 0;
  return cus * per_cu;
}

hipError_t launch_wake_potential(const WakeDev& w, hipStream_t s) {
  if (w.n_slices < 1 || w.n_slices > kWakeMaxSlices || !w.clear) return hipErrorInvalidValue;
  const int blocks = (w.n_slices + kWakePotSlices - 1) / kWakePotSlices;
  // LDS for the block that needs the most: counts and lags of every slice
  const size_t doubles = static_cast<size_t>(w.n_slices) + kWakePotThreads +
                        (w.n_slices <= kWakeStageSlices ? w.n_slices : 0);
  hipLaunchKernelGGL(k_wake_potential, dim3(blocks), dim3(kWakePotThreads),
                     doubles * sizeof(double), s, w);
  return hipGetLastError();
}

hipError_t launch_wake_zero(const WakeDev& w, hipStream_t s) {
  if (w.n_slices < 1 || w.n_slices > kWakeMaxSlices) return hipErrorInvalidValue;
  // both parities' buffers
  const int n = kWakeCountCopies * kWakeCountStride(w.n_slices);
  hipLaunchKernelGGL(k_wake_zero, dim3((n + 255) / 256), dim3(256), 0, s, w.counts, n);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_wake_zero, dim3((n + 255) / 256), dim3(256), 0, s, w.clear, n);
  return hipGetLastError();
}

}  // namespace ltrk
