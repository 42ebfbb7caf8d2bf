// C ABI of libmbf (declarations and contracts in include/mbf.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <exception>
#include <new>
#include <random>
#include <string>

#include "builder.h"
#include "device.h"
#include "factor.h"


namespace mbf {
namespace {
thread_local std::string g_last_error;
}
void set_error(const std::string& s) { g_last_error = s; }
const char* last_error_cstr() { return g_last_error.c_str(); }
}  // namespace mbf

using namespace mbf;

namespace {

mbf_status fail(mbf_status st, const std::string& msg) {
  set_error(msg);
  return st;
}
mbf_status from(const Error& e) {
  if (e.st != MBF_OK) set_error(e.msg);
  return e.st;
}

template <typename F>
mbf_status guarded(F&& fn) {
  try {
    return fn();
  } catch (const std::bad_alloc&) {
    return fail(MBF_ERR_OOM, "host allocation failed");
  } catch (const CallbackError& e) {
    return fail(MBF_ERR_CALLBACK, e.what());
  } catch (const std::exception& e) {
    return fail(MBF_ERR_INVALID_ARG, e.what());
  } catch (...) {
    return fail(MBF_ERR_INVALID_ARG, "unknown error");
  }
}

bool valid_prec(int p) { return p >= 0 && p < kNumPrec; }

}  // namespace

extern "C" {

const char* mbf_last_error(void) { return last_error_cstr(); }

mbf_status mbf_import(const mbf_import_desc* d, uint32_t prec_mask, void* stream, mbf_factor* out) {
  (void)stream;
  return guarded([&]() -> mbf_status {
    if (!d || !out) return fail(MBF_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    if (d->depth < 0 || d->depth > 15 || d->nx <= 0 || d->nxi <= 0 || !d->x_leaf_code ||
        !d->xi_leaf_code || !d->ranks || !d->v_leaf || !d->s_mid || !d->u_leaf)
      return fail(MBF_ERR_INVALID_ARG, "invalid import descriptor");
    if ((prec_mask & ((1u << kNumPrec) - 1)) == 0) return fail(MBF_ERR_INVALID_ARG, "empty precision mask");
    const int L = d->depth;
    const int64_t maxc = (int64_t)1 << (2 * L);
    for (int64_t i = 0; i < d->nx; ++i)
      if (d->x_leaf_code[i] < 0 || d->x_leaf_code[i] >= maxc) return fail(MBF_ERR_INVALID_ARG, "bad X leaf code");
    for (int64_t i = 0; i < d->nxi; ++i)
      if (d->xi_leaf_code[i] < 0 || d->xi_leaf_code[i] >= maxc)
        return fail(MBF_ERR_INVALID_ARG, "bad Omega leaf code");
    HostFactor f;
    f.L = L;
    f.m = L / 2;
    f.xt = tree_from_leaf_codes(L, d->nx, d->x_leaf_code);
    f.ot = tree_from_leaf_codes(L, d->nxi, d->xi_leaf_code);
    f.rank.resize(L + 1);
    const int32_t* rk = d->ranks;
    for (int s = 0; s <= L; ++s) {
      const int64_t np = (int64_t)f.xt.nn(s) * f.ot.nn(L - s);
      f.rank[s].assign(rk, rk + np);
      for (auto v : f.rank[s])
        if (v < 0) return fail(MBF_ERR_INVALID_ARG, "negative rank");
      rk += np;
    }
    if (f.m > 0 && !d->h_blocks) return fail(MBF_ERR_INVALID_ARG, "missing H blocks");
    if (f.m < L && !d->g_blocks) return fail(MBF_ERR_INVALID_ARG, "missing G blocks");
    const cd* V = reinterpret_cast<const cd*>(d->v_leaf);
    for (int32_t ib = 0; ib < f.ot.nn(L); ++ib) {
      const int64_t n = f.ot.size(L, ib) * f.rank[0][f.pair(0, 0, ib)];
      f.V0.emplace_back(V, V + n);
      V += n;
    }
    const cd* U = reinterpret_cast<const cd*>(d->u_leaf);
    for (int32_t ia = 0; ia < f.xt.nn(L); ++ia) {
      const int64_t n = f.xt.size(L, ia) * f.rank[L][f.pair(L, ia, 0)];
      f.UL.emplace_back(U, U + n);
      U += n;
    }
    int64_t ns = 0;
    for (auto v : f.rank[f.m]) ns += v;
    f.S.assign(d->s_mid, d->s_mid + ns);
    assemble_blocks(f, d->h_blocks, d->g_blocks);
    auto* h = new mbf_factor_s();
    h->dev.nx = d->nx;
    h->dev.nxi = d->nxi;
    h->dev.prec_mask = prec_mask & ((1u << kNumPrec) - 1);
    h->dev.parts.emplace_back();
    Error e = upload_part(f, nullptr, h->dev.prec_mask, h->dev.parts[0]);
    if (e.st != MBF_OK) {
      free_factor(h->dev);
      delete h;
      return from(e);
    }
    h->dev.nnz = h->dev.parts[0].nnz;
    for (auto& p : h->dev.parts[0].prec) h->dev.device_bytes += p.bytes;
    *out = h;
    return MBF_OK;
  });
}

// Owns a factor under construction: released (device memory included) when
// the build fails or throws before the handle is given out.
struct FactorGuard {
  mbf_factor_s* h = new mbf_factor_s();
  ~FactorGuard() {
    if (h) {
      free_factor(h->dev);
      delete h;
    }
  }
  mbf_factor_s* release() {
    mbf_factor_s* p = h;
    h = nullptr;
    return p;
  }
};

mbf_status mbf_build(int32_t dim, int64_t nx, const double* x, int64_t nxi, const double* xi,
                     mbf_entry_cb cb, void* user, const mbf_opts* opts, void* stream, mbf_factor* out) {
  (void)stream;
  return guarded([&]() -> mbf_status {
    if (!out) return fail(MBF_ERR_INVALID_ARG, "null output handle");
    *out = nullptr;
    if (dim != 2) return fail(MBF_ERR_UNSUPPORTED, "only dim = 2 is supported");
    if (!x || !xi || !cb || !opts || nx <= 0 || nxi <= 0) return fail(MBF_ERR_INVALID_ARG, "null or empty input");
    std::string why;
    if (!validate_opts(*opts, why)) return fail(MBF_ERR_INVALID_ARG, why);
    FactorGuard g;
    Error e = build_factor(nx, x, nxi, xi, cb, user, *opts, g.h->dev);
    if (e.st != MBF_OK) return from(e);
    *out = g.release();
    return MBF_OK;
  });
}

mbf_status mbf_build_matvec(int32_t dim, int64_t nx, const double* x, int64_t nxi, const double* xi,
                            mbf_matvec_cb mv, void* user, const mbf_opts* opts, const double* probes,
                            void* stream, mbf_factor* out) {
  (void)stream;
  return guarded([&]() -> mbf_status {
    if (!out) return fail(MBF_ERR_INVALID_ARG, "null output handle");
    *out = nullptr;
    if (dim != 2) return fail(MBF_ERR_UNSUPPORTED, "only dim = 2 is supported");
    if (!x || !xi || !mv || !opts || nx <= 0 || nxi <= 0) return fail(MBF_ERR_INVALID_ARG, "null or empty input");
    std::string why;
    if (!validate_opts(*opts, why)) return fail(MBF_ERR_INVALID_ARG, why);
    if (opts->oversample < 1) return fail(MBF_ERR_INVALID_ARG, "the matvec build needs oversample >= 1");
    if (opts->builder != MBF_BUILD_HOST) return fail(MBF_ERR_UNSUPPORTED, "the matvec build runs on the host builder");
    const int64_t q = (int64_t)opts->max_rank + opts->oversample;
    std::vector<cd> C, R;
    if (probes) {
      const cd* p = reinterpret_cast<const cd*>(probes);
      C.assign(p, p + nxi * q);
      R.assign(p + nxi * q, p + (nxi + nx) * q);
    } else {  // complex Gaussian entries, E|z|^2 = 1
      std::mt19937_64 rng(opts->seed ^ 0x5eed0f9a11ull);
      std::normal_distribution<double> nd(0.0, std::sqrt(0.5));
      C.resize((size_t)(nxi * q));
      R.resize((size_t)(nx * q));
      for (auto& z : C) z = cd(nd(rng), nd(rng));
      for (auto& z : R) z = cd(nd(rng), nd(rng));
    }
    MatvecSource src{mv, user, C.data(), R.data(), q, nx, nxi};
    FactorGuard g;
    Error e = build_factor(nx, x, nxi, xi, nullptr, nullptr, *opts, g.h->dev, &src);
    if (e.st != MBF_OK) return from(e);
    *out = g.release();
    return MBF_OK;
  });
}

mbf_status mbf_multiscale_assemble(int32_t nparts, mbf_factor* parts, const int64_t* const* part_idx,
                                   const int64_t* part_n, int64_t nxi, int64_t n_center,
                                   const int64_t* center_idx, const double* center, uint32_t prec_mask,
                                   void* stream, mbf_factor* out) {
  (void)stream;
  return guarded([&]() -> mbf_status {
    auto release = [&]() {
      for (int32_t t = 0; t < nparts; ++t)
        if (parts && parts[t]) {
          free_factor(parts[t]->dev);
          delete parts[t];
          parts[t] = nullptr;
        }
    };
    if (!out || nparts <= 0 || !parts || !part_idx || !part_n || nxi <= 0 || n_center < 0 ||
        (n_center > 0 && (!center_idx || !center))) {
      release();
      return fail(MBF_ERR_INVALID_ARG, "invalid multiscale arguments");
    }
    *out = nullptr;
    const int64_t nx = parts[0]->dev.nx;
    prec_mask &= (1u << kNumPrec) - 1;
    // Every Omega index of a part and of the center must name a point of
    // Omega: the apply gathers and scatters through them.
    for (int32_t t = 0; t < nparts; ++t) {
      if (part_n[t] < 0 || (part_n[t] > 0 && !part_idx[t])) {
        release();
        return fail(MBF_ERR_INVALID_ARG, "invalid multiscale part index list");
      }
      for (int64_t k = 0; k < part_n[t]; ++k)
        if (part_idx[t][k] < 0 || part_idx[t][k] >= nxi) {
          release();
          return fail(MBF_ERR_INVALID_ARG, "multiscale part index outside [0, nxi)");
        }
    }
    for (int64_t k = 0; k < n_center; ++k)
      if (center_idx[k] < 0 || center_idx[k] >= nxi) {
        release();
        return fail(MBF_ERR_INVALID_ARG, "center index outside [0, nxi)");
      }
    for (int32_t t = 0; t < nparts; ++t) {
      if (!parts[t] || parts[t]->dev.parts.size() != 1 || parts[t]->dev.nx != nx ||
          parts[t]->dev.nxi != part_n[t] || (parts[t]->dev.prec_mask & prec_mask) != prec_mask) {
        release();
        return fail(MBF_ERR_INVALID_ARG, "multiscale part mismatch");
      }
    }
    auto* h = new mbf_factor_s();
    h->dev.nx = nx;
    h->dev.nxi = nxi;
    h->dev.prec_mask = prec_mask;
    // Re-map every part's Omega indices to the caller's order.
    for (int32_t t = 0; t < nparts; ++t) {
      DevPart& P = parts[t]->dev.parts[0];
      std::vector<int32_t> idx(P.nxi);
      (void)hipMemcpy(idx.data(), P.d_vidx, idx.size() * 4, hipMemcpyDeviceToHost);
      for (auto& v : idx) {
        if (v < 0 || v >= part_n[t]) {
          free_factor(h->dev);
          delete h;
          release();
          return fail(MBF_ERR_INVALID_ARG, "bad part index");
        }
        v = (int32_t)part_idx[t][v];
      }
      (void)hipMemcpy(P.d_vidx, idx.data(), idx.size() * 4, hipMemcpyHostToDevice);
      h->dev.parts.push_back(P);
      h->dev.nnz += P.nnz;
      for (auto& p : P.prec) h->dev.device_bytes += p.bytes;
      parts[t]->dev.parts.clear();
      delete parts[t];
      parts[t] = nullptr;
    }
    if (n_center > 0) {
      std::vector<cd> KC(reinterpret_cast<const cd*>(center), reinterpret_cast<const cd*>(center) + nx * n_center);
      std::vector<int64_t> ci(center_idx, center_idx + n_center);
      Error e = upload_center(h->dev, KC, ci, prec_mask);
      if (e.st != MBF_OK) {
        free_factor(h->dev);
        delete h;
        return from(e);
      }
      h->dev.nnz += nx * n_center;
      for (auto& p : h->dev.center) h->dev.device_bytes += p.bytes;
    }
    *out = h;
    return MBF_OK;
  });
}

mbf_status mbf_autotune(mbf_factor f, mbf_prec p, int64_t nrhs, void* workspace, size_t ws_bytes, void* stream,
                        int32_t* tuned) {
  if (!f || !valid_prec(p) || nrhs <= 0 || !workspace) return fail(MBF_ERR_INVALID_ARG, "invalid argument");
  if (!(f->dev.prec_mask & (1u << p))) return fail(MBF_ERR_UNSUPPORTED, "precision not built for this factor");
  int n = 0;
  mbf_status st = from(autotune_factor(f->dev, p, nrhs, workspace, ws_bytes, (hipStream_t)stream, &n));
  if (tuned) *tuned = n;
  return st;
}

mbf_status mbf_save(mbf_factor f, uint32_t prec_mask, const char* path) {
  if (!f || !path) return fail(MBF_ERR_INVALID_ARG, "invalid argument");
  prec_mask &= (1u << kNumPrec) - 1;
  if (prec_mask == 0) prec_mask = f->dev.prec_mask;
  if ((prec_mask & f->dev.prec_mask) != prec_mask) return fail(MBF_ERR_UNSUPPORTED, "precision not held by the factor");
  return guarded([&]() -> mbf_status { return from(save_factor(f->dev, prec_mask, path)); });
}

mbf_status mbf_load(const char* path, uint32_t prec_mask, void* stream, mbf_factor* out) {
  (void)stream;
  if (!path || !out) return fail(MBF_ERR_INVALID_ARG, "invalid argument");
  *out = nullptr;
  return guarded([&]() -> mbf_status {
    auto* h = new mbf_factor_s();
    Error e = load_factor(path, prec_mask & ((1u << kNumPrec) - 1), h->dev);
    if (e.st != MBF_OK) {
      free_factor(h->dev);
      delete h;
      return from(e);
    }
    *out = h;
    return MBF_OK;
  });
}

mbf_status mbf_workspace_size(mbf_factor f, mbf_prec p, int64_t nrhs, size_t* bytes) {
  if (!f || !bytes || nrhs < 0 || !valid_prec(p)) return fail(MBF_ERR_INVALID_ARG, "invalid argument");
  *bytes = workspace_bytes(f->dev, p, nrhs);
  return MBF_OK;
}

static mbf_status apply_common(mbf_factor f, mbf_prec p, bool adj, int64_t nrhs, const void* in,
                               int64_t ldin, void* out, int64_t ldout, void* ws, size_t wsb, void* stream) {
  if (!f || !valid_prec(p) || nrhs < 0) return fail(MBF_ERR_INVALID_ARG, "invalid argument");
  if (!(f->dev.prec_mask & (1u << p))) return fail(MBF_ERR_UNSUPPORTED, "precision not built for this factor");
  if (nrhs == 0) return MBF_OK;
  if (nrhs > 65535 * 32) return fail(MBF_ERR_INVALID_ARG, "too many right-hand sides");
  const int64_t nin = adj ? f->dev.nx : f->dev.nxi;
  const int64_t nout = adj ? f->dev.nxi : f->dev.nx;
  if (!in || !out || !ws) return fail(MBF_ERR_INVALID_ARG, "null device pointer");
  if (ldin < nin || ldout < nout) return fail(MBF_ERR_INVALID_ARG, "leading dimension too small");
  return from(launch_apply(f->dev, p, adj, nrhs, in, ldin, out, ldout, ws, wsb, (hipStream_t)stream));
}

mbf_status mbf_apply(mbf_factor f, mbf_prec p, int64_t nrhs, const void* g, int64_t ldg, void* u, int64_t ldu,
                     void* workspace, size_t ws_bytes, void* stream) {
  return apply_common(f, p, false, nrhs, g, ldg, u, ldu, workspace, ws_bytes, stream);
}

mbf_status mbf_apply_scratch(mbf_factor f, mbf_prec p, int64_t nrhs, const void* g, int64_t ldg, void* u,
                             int64_t ldu, void* stream) {
  if (!f || !valid_prec(p) || nrhs < 0) return fail(MBF_ERR_INVALID_ARG, "invalid argument");
  if (!(f->dev.prec_mask & (1u << p))) return fail(MBF_ERR_UNSUPPORTED, "precision not built for this factor");
  if (nrhs == 0) return MBF_OK;
  if (nrhs > 65535 * 32) return fail(MBF_ERR_INVALID_ARG, "too many right-hand sides");
  if (!g || !u) return fail(MBF_ERR_INVALID_ARG, "null device pointer");
  if (ldg < f->dev.nxi || ldu < f->dev.nx) return fail(MBF_ERR_INVALID_ARG, "leading dimension too small");
  return from(launch_apply_scratch(f->dev, p, nrhs, g, ldg, u, ldu, (hipStream_t)stream));
}

size_t mbf_scratch_bytes(void) { return scratch_bytes(); }

mbf_status mbf_apply_adjoint(mbf_factor f, mbf_prec p, int64_t nrhs, const void* h, int64_t ldh, void* v,
                             int64_t ldv, void* workspace, size_t ws_bytes, void* stream) {
  return apply_common(f, p, true, nrhs, h, ldh, v, ldv, workspace, ws_bytes, stream);
}

mbf_status mbf_info(mbf_factor f, mbf_info_t* out) {
  if (!f || !out) return fail(MBF_ERR_INVALID_ARG, "invalid argument");
  std::memset(out, 0, sizeof(*out));
  const auto& F = f->dev;
  out->nparts = (int32_t)F.parts.size();
  if (!F.parts.empty()) {
    const auto& P = F.parts[0];
    out->depth = F.parts.size() == 1 ? P.L : 0;
    out->mid = P.m;
    for (int s = 0; s <= P.L && s < 33; ++s) out->max_rank[s] = P.max_rank[s];
  }
  for (const auto& P : F.parts) {
    for (int s = 0; s < P.L; ++s) {
      const int64_t w = (s + 1 < (int)P.w_stage_off.size() ? P.w_stage_off[s + 1] : P.w_elems) - P.w_stage_off[s];
      out->nnz_stage_max = std::max(out->nnz_stage_max, w);
    }
    for (auto r : P.rows) out->state_rows_max = std::max(out->state_rows_max, r);
  }
  out->nx = F.nx;
  out->nxi = F.nxi;
  out->nnz = F.nnz;
  out->prec_mask = F.prec_mask;
  out->device_bytes = F.device_bytes;
  return MBF_OK;
}

static void profile_release(Profiler& p) {
  for (auto e : p.ev) (void)hipEventDestroy(e);
  p = Profiler{};
}

mbf_status mbf_profile_begin(mbf_factor f, int32_t max_launches) {
  if (!f || max_launches <= 0 || max_launches > (1 << 20)) return fail(MBF_ERR_INVALID_ARG, "invalid argument");
  Profiler& p = f->dev.prof;
  profile_release(p);
  p.ev.resize(2 * (size_t)max_launches);
  for (auto& e : p.ev) {
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) {
      e = nullptr;
      profile_release(p);
      return fail(MBF_ERR_HIP, std::string("hipEventCreate: ") + hipGetErrorString(r));
    }
  }
  p.rec.resize(max_launches);
  p.cap = max_launches;
  p.used = 0;
  p.on = true;
  return MBF_OK;
}

mbf_status mbf_profile_end(mbf_factor f, mbf_launch_record* out, int32_t cap, int32_t* count) {
  if (!f || !count || (cap > 0 && !out)) return fail(MBF_ERR_INVALID_ARG, "invalid argument");
  Profiler& p = f->dev.prof;
  int32_t n = 0;
  for (int32_t i = 0; i < p.used; ++i) {
    hipError_t r = hipEventSynchronize(p.ev[2 * i + 1]);
    float ms = 0.f;
    if (r == hipSuccess) r = hipEventElapsedTime(&ms, p.ev[2 * i], p.ev[2 * i + 1]);
    if (r != hipSuccess) {
      profile_release(p);
      return fail(MBF_ERR_HIP, std::string("event timing: ") + hipGetErrorString(r));
    }
    p.rec[i].ms = ms;
    if (n < cap) out[n++] = p.rec[i];
  }
  *count = n;
  profile_release(p);
  return MBF_OK;
}

void mbf_destroy(mbf_factor f) {
  if (!f) return;
  profile_release(f->dev.prof);
  free_factor(f->dev);
  delete f;
}

}  // extern "C"
