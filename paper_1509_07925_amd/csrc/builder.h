// Host FP64 builder of the butterfly factorization from a kernel-entry
// callback (Section 2, case (ii)); polar (Section 3.2) and multiscale
// (Section 4.2) splits.
#pragma once

#include <stdexcept>
#include <string>

#include "device.h"
#include "factor.h"

namespace mbf {

struct CallbackError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

bool validate_opts(const mbf_opts& o, std::string& why);

Error build_factor(int64_t nx, const double* x, int64_t nxi, const double* xi, mbf_entry_cb cb,
                   void* user, const mbf_opts& o, DevFactor& out);

// Build one plain factorization on given trees (exposed for tests of the
// host builder).  xs / os map tree point indices to callback indices.
HostFactor build_host(const Tree& xt, const Tree& ot, const std::vector<int64_t>& xs,
                      const std::vector<int64_t>& os, mbf_entry_cb cb, void* user, const mbf_opts& o);

}  // namespace mbf
