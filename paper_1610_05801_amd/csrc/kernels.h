// Host-side launchers of the HIP kernels in kernels.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ltrk_device.h"

namespace ltrk {

// One bunch for b.turns turns; moment rows start at row0 of b.partials.
hipError_t launch_track_single(const BunchDev& b, int32_t row0, int ppl, int block,
                               hipStream_t s);
// Tiled launch over device tables of bunches and tiles (one scheme/precision).
hipError_t launch_track_tiles(const BunchDev* bunches, const TileDev* tiles, int64_t ntiles,
                              int integrator, int dtype, int32_t turns, int32_t row0, int ppl,
                              int block, bool moments, hipStream_t s);
// Tiled launch where every bunch has its own scheme, precision and turn count.
hipError_t launch_track_mixed(const BunchDev* bunches, const TileDev* tiles, int64_t ntiles,
                              int ppl, int block, hipStream_t s);
// Moment rows of one bunch (two-stage when f.groups > 1; f.stage then holds
// rows * 5 * groups doubles).
hipError_t launch_finalize_single(const FinalizeDev& f, hipStream_t s);
// Rows [0, rows) of every bunch (bounded by each f.rows) into f.out[out_row0 + row];
// max_groups is the largest f.groups in the table (two-stage reduction when > 1).
hipError_t launch_finalize_multi(const FinalizeDev* fs, int nf, int rows, int64_t out_row0,
                                 int64_t max_groups, hipStream_t s);
hipError_t launch_fill_nan(ltrk_moments* out, int64_t rows, hipStream_t s);
hipError_t launch_fill_probe(double* z, double* dp, int64_t n, hipStream_t s);

}  // namespace ltrk
