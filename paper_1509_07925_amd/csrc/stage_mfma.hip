// Matrix-core (MFMA) stage kernels; see stage_mfma.h.
#include "stage_mfma.h"

namespace mbf {

bool use_mfma(const DevPart&, int, int64_t, int prec) { return prec == MBF_C64_SPLIT_BF16; }

Error launch_stage_mfma(const DevPart&, int, int, bool, const BlockDesc*, const void*, const void*,
                        int64_t, void*, int64_t, int, const float*, hipStream_t) {
  return {MBF_ERR_UNSUPPORTED, "split-BF16 stage kernel not available"};
}

}  // namespace mbf
