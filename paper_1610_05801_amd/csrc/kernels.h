// Host-side launchers of the HIP kernels in kernels.hip and kernels_ext.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ltrk_device.h"
#include "ltrk_device_ext.h"

namespace ltrk {

// One bunch for b.turns turns; moment rows start at row0 of b.partials.
hipError_t launch_track_single(const BunchDev& b, int32_t row0, int ppl, int block,
                               hipStream_t s);
// One bunch (FP64) through the extended map for b.turns turns.
hipError_t launch_track_rf2(const BunchDev& b, const CoeffsRf2& c, int32_t row0, int ppl,
                            int block, hipStream_t s);
// One bunch (FP64) through an RF programme: turn t of the launch uses record
// turn0 + t of `prog` (prog_layout(b.integrator)); accel adds the reference
// momentum step to every kick (not for RK4).
hipError_t launch_track_prog(const BunchDev& b, const CoeffsRf2& c, const double* prog,
                             int32_t turn0, int32_t row0, int ppl, int block, bool accel,
                             hipStream_t s);
// One bunch with a 6-D state for b.turns turns; moment rows (3 planes) start
// at row0 of b.partials.
hipError_t launch_track_6d(const Bunch6Dev& b, const Coeffs6d& c, int32_t row0, int ppl,
                           int block, hipStream_t s);
// One turn of the wake path on a fixed grid of `grid` blocks (<= kWakeMaxBlocks).
// phase 0: map step and histogram; 1: kick from w.pot, moment row `row` (when
// b.partials), step and histogram; 2: kick and moment row only.
hipError_t launch_wake_turn(const BunchDev& b, const CoeffsRf2& c, const WakeDev& w, int phase,
                            int32_t row, int ppl, int block, int grid, hipStream_t s);
// The potential w.pot from the slice counts, which it zeroes (one block).
hipError_t launch_wake_potential(const WakeDev& w, hipStream_t s);
// Blocks of `block` threads of the wake turn kernel that the device holds at
// once (all compute units; 0 if the runtime cannot tell).
int wake_resident_blocks(int integrator, int harmonics, int ppl, int block, int n_slices);
// Zero the slice counts (start of a call; a kernel, not a memset, so a
// captured sequence replays correctly).
hipError_t launch_wake_zero(const WakeDev& w, hipStream_t s);
// Tiled launch over device tables of bunches and tiles (one scheme/precision).
hipError_t launch_track_tiles(const BunchDev* bunches, const TileDev* tiles, int64_t ntiles,
                              int integrator, int dtype, int32_t turns, int32_t row0, int ppl,
                              int block, bool moments, hipStream_t s);
// Tiled launch where every bunch has its own scheme, precision and turn count.
hipError_t launch_track_mixed(const BunchDev* bunches, const TileDev* tiles, int64_t ntiles,
                              int ppl, int block, hipStream_t s);
// Moment rows of one bunch or plane (two-stage when f.groups > 1; f.stage
// then holds rows * 5 * groups doubles); row r goes to f.out[r * planes].
hipError_t launch_finalize_single(const FinalizeDev& f, hipStream_t s);
// Rows [0, rows) of every bunch (bounded by each f.rows) into f.out[out_row0 + row];
// max_groups is the largest f.groups in the table (two-stage reduction when > 1).
hipError_t launch_finalize_multi(const FinalizeDev* fs, int nf, int rows, int64_t out_row0,
                                 int64_t max_groups, hipStream_t s);
// The centre of a bunch's moment sums (kCentreSample) into c.out[0..1].
hipError_t launch_centre(const CentreDev& c, hipStream_t s);
// The same for every bunch of a device table that computes moments (into
// its b.centre).
hipError_t launch_centre_bunches(const BunchDev* bunches, int nb, hipStream_t s);
hipError_t launch_fill_nan(ltrk_moments* out, int64_t rows, hipStream_t s);
hipError_t launch_fill_probe(double* z, double* dp, int64_t n, hipStream_t s);

}  // namespace ltrk
