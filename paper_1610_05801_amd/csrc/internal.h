// Host-side internals of libltrk shared by runtime.hip and engine.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/ltrk.h"
#include "ltrk_device.h"

namespace ltrk {

// Thread-local error state; returns `code` so call sites can `return fail(...)`.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail_hip(hipError_t e, const char* what);
void clear_error();

// Ring validation and FP64 derivation (section 1.1.2 map; textbook relations).
int validate_ring(const ltrk_ring* r);
void derive(const ltrk_ring& r, ltrk_derived* out);
// Kernel coefficients of `integrator` for ring r.
void make_coeffs(const ltrk_ring& r, int integrator, Coeffs* c);

bool valid_integrator(int integ);
bool valid_dtype(int dtype);

// EINVAL unless [p, p + bytes) lies inside one device allocation.
int check_device_range(const void* p, size_t bytes, const char* name);

int64_t waves_for(int64_t n, int ppl);
// Moment scratch doubles per (row, moment) for W wave tiles (two-stage aware).
int64_t scratch_cols(int64_t W);

// Current device (for per-device contexts).
int current_device(int* dev);

// Plans: forced plan, tuned cache, built-in default (see runtime.hip).
// is_default (optional) tells whether the built-in default was chosen.
ltrk_plan choose_plan(int integrator, int dtype, int64_t n, bool batched,
                      bool* is_default = nullptr);
// Turns per launch of a default plan that computes moments, given the bytes
// of one turn's moment partials (see tune.hip).
int64_t default_turns_for_partials(int64_t turns_per_launch, int64_t bytes_per_row);

// Launch timing hooks (no-ops unless ltrk_timing_enable(1)).
bool timing_on();
void timing_begin(hipStream_t s, int kind, void** token);
void timing_end(hipStream_t s, void* token);
enum { kTimeTrack = 0, kTimeFinalize = 1 };

}  // namespace ltrk
