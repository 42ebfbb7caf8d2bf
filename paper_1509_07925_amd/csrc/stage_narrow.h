// Stage block products for few right-hand sides (FP32, streaming the blocks).
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace mbf {

// Stage s of part P (forward, or adjoint when adj) for 1 <= nrhs, in passes
// of 8, 16 or 32 right-hand sides; meant for nrhs <= 32, where the stage is
// bound by reading its FP32 blocks.
Error launch_stage_narrow(const DevPart& P, int s, bool adj, const BlockDesc* blk, const void* W, const void* in,
                          int64_t ld_in, void* out, int64_t ld_out, int nrhs, const float* scale, hipStream_t st);

}  // namespace mbf
