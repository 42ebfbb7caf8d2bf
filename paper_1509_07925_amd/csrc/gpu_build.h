// FP64 builder on the GPU (Section 2, case (ii)): the same steps as the host
// builder, with the kernel entries evaluated on the device.
#pragma once

#include <cstdint>
#include <vector>

#include "device.h"
#include "factor.h"

namespace mbf {

// Kernels whose entries the device evaluates: the 2D DFT and the Example-1
// FIO (the ready-made callbacks mbf_kernel_dft / mbf_kernel_fio).
struct DeviceKernel {
  int kind = 0;          // 0 = DFT, 1 = FIO
  int64_t n = 0;         // grid side
  double c_scale = 1.0;  // FIO only
  const double* x = nullptr;   // X points as given to mbf_build (caller order)
  const double* xi = nullptr;  // Omega points
  int64_t nx = 0, nxi = 0;
};

// Build one part (trees over X and over an Omega subset) on the current
// device and fill P (layout + factors in every precision of prec_mask).
// xs / os map tree point indices to caller indices (os: the part's Omega
// indices in the caller's order, or the identity).
Error build_part_device(const Tree& xt, const Tree& ot, const std::vector<int64_t>& xs,
                        const std::vector<int64_t>& os, const DeviceKernel& K, const mbf_opts& o,
                        uint32_t prec_mask, DevPart& P);

// Dense center K_C of the multiscale split evaluated on the device
// (nx x |idx|, column-major) in every precision of prec_mask.
Error build_center_device(const DeviceKernel& K, const std::vector<int64_t>& idx, uint32_t prec_mask,
                          DevFactor& F);

}  // namespace mbf
