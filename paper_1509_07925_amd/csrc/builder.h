// Host FP64 builder of the butterfly factorization from a kernel-entry
// callback (Section 2, case (ii)) or from fast products with K and K^*
// (case (i)); polar (Section 3.2) and multiscale (Section 4.2) splits.
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

// Case (i) of Section 2.3: the black box of K and K^* and the Gaussian
// probes C (nxi x q) and R (nx x q), column-major complex128.
struct MatvecSource {
  mbf_matvec_cb mv;
  void* user;
  const std::complex<double>* C;
  const std::complex<double>* R;
  int64_t q, nx, nxi;
};

// With src, every middle-level block is factored from products with the
// black box (case (i)) and cb / user are not used; otherwise from entries
// (case (ii)).
Error build_factor(int64_t nx, const double* x, int64_t nxi, const double* xi, mbf_entry_cb cb,
                   void* user, const mbf_opts& o, DevFactor& out, const MatvecSource* src = nullptr);

// Build one plain factorization on given trees (exposed for tests of the
// host builder).  xs / os map tree point indices to callback indices.
HostFactor build_host(const Tree& xt, const Tree& ot, const std::vector<int64_t>& xs,
                      const std::vector<int64_t>& os, mbf_entry_cb cb, void* user, const mbf_opts& o);

}  // namespace mbf
