// Matrix-core (MFMA) stage kernels for many right-hand sides.
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace mbf {

// True when stage s of part P at this RHS count runs on the MFMA kernels
// (always true for the split-BF16 precision, whose blocks exist only in
// the split layout).
bool use_mfma(const DevPart& P, int s, int64_t nrhs, int prec);

// Stage kernel variants (tile shape, register prefetch, LDS buffering):
// 11 for the FP32 kernels (8 on the real embedding, 3 with three real
// products), 7 for the split-BF16 kernels.
inline int num_variants(int prec) { return prec == MBF_C64 ? 11 : 7; }

// force_variant >= 0 bypasses the tuned choice.
Error launch_stage_mfma(const DevPart& P, int s, int prec, bool adjoint, const BlockDesc* blk,
                        const void* W, const void* in, int64_t ld_in, void* out, int64_t ld_out,
                        int nrhs, const float* scale, hipStream_t st, int force_variant = -1);

// Variant used for a stage shape (tuned, else MBF_STAGE_VARIANT, else a default).
int tuned_variant(int prec, bool adj, int R, int Q, int nrhs);

// Time every variant on stage s (2 launches each after one warm-up launch,
// on scratch data in / out) and record the fastest for the shape.
Error autotune_stage(const DevPart& P, int s, int prec, bool adj, const BlockDesc* blk, const void* W,
                     const void* in, int64_t ld_in, void* out, int64_t ld_out, int nrhs, hipStream_t st,
                     int* chosen, float* best_ms);

}  // namespace mbf
