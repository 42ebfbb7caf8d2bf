// Matrix-core (MFMA) stage kernels for many right-hand sides.
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace mbf {

// True when stage s of part P at this RHS count runs on the MFMA kernels
// (always true for the split-BF16 precision, whose blocks exist only in
// the split layout).
bool use_mfma(const DevPart& P, int s, int64_t nrhs, int prec);

Error launch_stage_mfma(const DevPart& P, int s, int prec, bool adjoint, const BlockDesc* blk,
                        const void* W, const void* in, int64_t ld_in, void* out, int64_t ld_out,
                        int nrhs, const float* scale, hipStream_t st);

}  // namespace mbf
