// Stage block products for up to 16 right-hand sides on the matrix cores (FP32).
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace mbf {

// Stage s of part P (forward, or adjoint when adj) in passes of 16
// right-hand sides (v_mfma_f32_16x16x4_f32); meant for 1 <= nrhs <= 16.
Error launch_stage_r16(const DevPart& P, int s, bool adj, const BlockDesc* blk, const void* W, const void* in,
                       int64_t ld_in, void* out, int64_t ld_out, int nrhs, const float* scale, hipStream_t st);

}  // namespace mbf
