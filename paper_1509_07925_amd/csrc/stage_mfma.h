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
// products), 7 for the split-BF16 kernels of FP32 input states and 4 for
// those of split input states (in_split).
inline int num_variants(int prec, bool in_split = false) {
  return prec == MBF_C64 ? 11 : in_split ? 4 : 7;
}

// force_variant >= 0 bypasses the tuned choice.  in_split / out_split (split
// BF16 precision only): the input / output state is split, i.e. each complex
// entry is held as the BF16 words hi = Re_hi | Im_hi << 16 and
// lo = Re_lo | Im_lo << 16, side by side in the 8 bytes of the entry (hi at
// 32-bit word 2 (ld n + row), lo at the next word, for the column stride ld);
// interior stages pass the state on in that form.  in_split needs
// ld_in < 2^23.
Error launch_stage_mfma(const DevPart& P, int s, int prec, bool adjoint, const BlockDesc* blk,
                        const void* W, const void* in, int64_t ld_in, void* out, int64_t ld_out,
                        int nrhs, const float* scale, hipStream_t st, bool in_split = false,
                        bool out_split = false, int force_variant = -1);

// Variant used for a stage shape (tuned, else MBF_STAGE_VARIANT modulo the
// family's variant count, else a default).
int tuned_variant(int prec, bool in_split, bool adj, int R, int Q, int nrhs);

// Split-BF16 states between stages: the faster of split states (the split-
// input kernels) and FP32 states (every stage splits its input itself), as
// timed by the autotuner, per (precision, widest state bucket, RHS bucket):
// 1 split, 0 FP32, -1 not tuned.  Both give identical results.
int split_choice(int prec, int64_t rows, int nrhs);
void set_split_choice(int prec, int64_t rows, int nrhs, bool on);

// Time every variant of the family (prec, in_split) on stage s (2 launches
// each after one warm-up launch, on scratch data in / out) and record the
// fastest for the shape.
Error autotune_stage(const DevPart& P, int s, int prec, bool in_split, bool adj, const BlockDesc* blk,
                     const void* W, const void* in, int64_t ld_in, void* out, int64_t ld_out, int nrhs,
                     hipStream_t st, int* chosen, float* best_ms);

}  // namespace mbf
