// Stage block products for up to 32 right-hand sides on the matrix cores (FP32).
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace mbf {

// Stage s of part P (forward, or adjoint when adj) on the 16 x 16 matrix-core
// tile (v_mfma_f32_16x16x4_f32): one 16-RHS tile per workgroup for
// nrhs <= 16, two for larger nrhs (the FP32 path uses it up to 32 RHS; any
// nrhs >= 1 is accepted, in workgroups of 32 right-hand sides).
Error launch_stage_r16(const DevPart& P, int s, bool adj, const BlockDesc* blk, const void* W, const void* in,
                       int64_t ld_in, void* out, int64_t ld_out, int nrhs, const float* scale, hipStream_t st);

}  // namespace mbf
