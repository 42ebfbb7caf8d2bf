// Host FP64 builder (see builder.h).
//
// Order of work: the recursive factorization of U^h is independent for
// every middle-level node A of T_X, and that of V^h for every middle-level
// node B of T_Omega.  The builder runs one task per middle-level node:
//   U task (A):  for every B, factor K_{A,B} at the middle level (SVD via
//                random sampling, form eq. (lowrank1)); keep V_{B,A} for the
//                V pass; then recurse down the subtree of A with U_{A,.}
//                (split, merge, truncate in form eq. (lowrank2), assemble G).
//   V task (B):  take V_{B,.} and recurse down the subtree of B, producing H.
// U^h is held one subtree per thread; V^h is held whole between the passes.
#include "builder.h"

#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <numeric>
#include <random>
#include <thread>
#include <sched.h>
#include <cstdlib>

#include "gpu_build.h"
#include "linalg.h"

namespace mbf {

using la::Mat;

namespace {

struct Ctx {
  mbf_entry_cb cb;
  void* user;
  const std::vector<int64_t>* xs;  // tree point -> callback row index
  const std::vector<int64_t>* os;  // tree point -> callback column index
};

// Entries K(rows, cols) where rows / cols are callback indices.
Mat entries(const Ctx& c, const std::vector<int64_t>& rows, const std::vector<int64_t>& cols) {
  Mat Z((int64_t)rows.size(), (int64_t)cols.size());
  if (Z.m == 0 || Z.n == 0) return Z;
  const int rc = c.cb(c.user, Z.m, rows.data(), Z.n, cols.data(), reinterpret_cast<double*>(Z.a.data()));
  if (rc != 0) throw CallbackError("entry callback returned " + std::to_string(rc));
  return Z;
}

uint64_t mix(uint64_t a, uint64_t b) {
  uint64_t z = a * 0x9E3779B97F4A7C15ull + b + 0x632BE59BD9B4E019ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

std::vector<int64_t> sample(std::mt19937_64& rng, int64_t n, int64_t k) {
  k = std::min(k, n);
  std::vector<int64_t> all(n);
  std::iota(all.begin(), all.end(), 0);
  for (int64_t i = 0; i < k; ++i) {
    std::uniform_int_distribution<int64_t> d(i, n - 1);
    std::swap(all[i], all[d(rng)]);
  }
  all.resize(k);
  std::sort(all.begin(), all.end());
  return all;
}

std::vector<int64_t> merge_sorted(const std::vector<int64_t>& a, const std::vector<int64_t>& b) {
  std::vector<int64_t> out;
  std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(out));
  return out;
}

struct Low {
  Mat U0, V0;
  std::vector<double> s;
};

// SVD via random sampling (Section 2.1, case ii) of Z = K(ra, cb) where ra
// and cb list callback indices of the rows / columns.  Steps, in the
// paper's order:
//   (1) representative columns: pivoted QR of q randomly selected rows;
//       the representative rows are those q random rows (reading of the
//       paper's iteration, see the design notes: one selection round);
//   (2) orthonormal bases Q_col of the representative columns and Q_row of
//       the representative rows (Householder QR);
//   (3) M = pinv(Q_col[I_row]) Z(I_row, I_col) pinv(Q_row[I_col]^*) on index
//       sets that contain the representatives plus q fresh random indices;
//   (4) SVD of M:  Z ~ (Q_col U_M) S_M (Q_row V_M)^*.
Low sampled_svd(const Ctx& c, const std::vector<int64_t>& ra, const std::vector<int64_t>& cb, double tol,
                int64_t rmax, int64_t os, int64_t q, std::mt19937_64& rng) {
  const int64_t m = (int64_t)ra.size(), n = (int64_t)cb.size();
  auto sub = [](const std::vector<int64_t>& base, const std::vector<int64_t>& idx) {
    std::vector<int64_t> o(idx.size());
    for (size_t i = 0; i < idx.size(); ++i) o[i] = base[idx[i]];
    return o;
  };
  const double qtol = tol * 1e-2;
  Low out;
  // (1) representatives
  std::vector<int64_t> reps_r = sample(rng, m, q);
  Mat Zr = entries(c, sub(ra, reps_r), cb);  // |reps_r| x n
  la::QRP qr1 = la::pivoted_qr(Zr, qtol, std::min<int64_t>(rmax + os, n));
  std::vector<int64_t> reps_c(qr1.piv.begin(), qr1.piv.begin() + qr1.k);
  std::sort(reps_c.begin(), reps_c.end());
  if (reps_c.empty()) {
    out.U0 = Mat(m, 0);
    out.V0 = Mat(n, 0);
    return out;
  }
  // (2) bases.  Q_col from the representative columns; the representative
  // rows are then refined by a pivoted QR over the rows of those columns
  // (the paper's alternation between columns and rows), and Q_row is the
  // basis of the selected rows.
  Mat Zcr = entries(c, ra, sub(cb, reps_c));  // m x kc
  la::QRP qc = la::pivoted_qr(Zcr, qtol * 1e-2, (int64_t)reps_c.size(), false);
  la::QRP qsel = la::pivoted_qr(la::adjoint(Zcr), qtol, std::min<int64_t>((int64_t)reps_c.size(), m));
  std::vector<int64_t> rows2(qsel.piv.begin(), qsel.piv.begin() + qsel.k);
  std::sort(rows2.begin(), rows2.end());
  reps_r = merge_sorted(rows2, reps_r);
  la::QRP qrr = la::pivoted_qr(la::adjoint(entries(c, sub(ra, reps_r), cb)), qtol, (int64_t)reps_r.size(), true);
  const Mat& Qc = qc.Q;   // m x kc
  const Mat& Qr = qrr.Q;  // n x kr
  // (3) middle matrix on index sets containing the representatives
  // Least-squares systems stay overdetermined by at least q rows / columns.
  const std::vector<int64_t> Irow = merge_sorted(reps_r, sample(rng, m, Qc.n + q));
  const std::vector<int64_t> Icol = merge_sorted(reps_c, sample(rng, n, Qr.n + q));
  Mat Zs = entries(c, sub(ra, Irow), sub(cb, Icol));
  Mat Qci((int64_t)Irow.size(), Qc.n), Qri((int64_t)Icol.size(), Qr.n);
  for (int64_t j = 0; j < Qc.n; ++j)
    for (size_t i = 0; i < Irow.size(); ++i) Qci((int64_t)i, j) = Qc(Irow[i], j);
  for (int64_t j = 0; j < Qr.n; ++j)
    for (size_t i = 0; i < Icol.size(); ++i) Qri((int64_t)i, j) = Qr(Icol[i], j);
  // M = pinv(Qc[Irow]) Z pinv(Qr[Icol])^*, both pseudo-inverses as least-squares solves
  Mat T = la::lstsq(Qci, Zs);                           // kc x |Icol|
  Mat M = la::adjoint(la::lstsq(Qri, la::adjoint(T)));  // kc x kr
  // (4) SVD of M
  la::SVD d = la::svd(M);
  const int64_t r = la::trunc_rank(d.s, tol, rmax);
  Mat UM(M.m, r), VM(M.n, r);
  for (int64_t j = 0; j < r; ++j) {
    for (int64_t i = 0; i < M.m; ++i) UM(i, j) = d.U(i, j);
    for (int64_t i = 0; i < M.n; ++i) VM(i, j) = d.V(i, j);
  }
  out.U0 = la::matmul(Qc, UM);
  out.V0 = la::matmul(Qr, VM);
  out.s.assign(d.s.begin(), d.s.begin() + r);
  return out;
}

// Middle-level factorization of pair (ia, ib).  The sample size starts at
// q0 and doubles while the rank found reaches q - oversample; the random
// stream depends only on (seed, ia, ib, q), so the U and V passes obtain
// identical factors for the same pair.
std::atomic<int64_t> g_mid_us{0}, g_rec_us{0}, g_t_ent{0}, g_t_round{0}, g_t_basis{0}, g_t_solve{0}, g_t_svd{0};
struct ScopedUs;
struct ScopedUs {
  std::atomic<int64_t>& acc;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  explicit ScopedUs(std::atomic<int64_t>& a) : acc(a) {}
  ~ScopedUs() {
    acc += std::chrono::duration_cast<std::chrono::microseconds>(std::chrono::steady_clock::now() - t0).count();
  }
};

Low middle_pair(const Ctx& c, const Tree& xt, const Tree& ot, int m, int32_t ia, int32_t ib,
                const mbf_opts& o, int64_t q0, int64_t* rank_out = nullptr) {
  ScopedUs timer(g_mid_us);
  const int L = xt.L;
  std::vector<int64_t> ra, cb;
  for (int64_t p = xt.off[m][ia]; p < xt.off[m][ia + 1]; ++p) ra.push_back((*c.xs)[xt.perm[p]]);
  for (int64_t p = ot.off[L - m][ib]; p < ot.off[L - m][ib + 1]; ++p) cb.push_back((*c.os)[ot.perm[p]]);
  const int64_t mn = std::min<int64_t>(ra.size(), cb.size());
  int64_t q = std::max<int64_t>(16, q0);
  for (;;) {
    std::mt19937_64 rng(mix(mix(o.seed, (uint64_t)ia), (uint64_t)ib) ^ (uint64_t)q);
    Low lw = sampled_svd(c, ra, cb, o.tol, o.max_rank, o.oversample, q, rng);
    const int64_t r = (int64_t)lw.s.size();
    if (r + o.oversample <= q || q >= mn || r >= o.max_rank) {
      if (rank_out) *rank_out = r;
      return lw;
    }
    q *= 2;
  }
}

// Restrict rows [r0, r1) of a column block set and merge side by side.
Mat merge_rows(const std::vector<const Mat*>& parts, int64_t r0, int64_t r1) {
  int64_t cols = 0;
  for (auto* p : parts) cols += p->n;
  Mat W(r1 - r0, cols);
  int64_t c0 = 0;
  for (auto* p : parts) {
    for (int64_t j = 0; j < p->n; ++j) std::copy(p->col(j) + r0, p->col(j) + r1, W.col(c0 + j));
    c0 += p->n;
  }
  return W;
}

// SVD via random matrix-vector products (Section 2.1, first option) of one
// middle-level block Z, known only through its products with Gaussian
// probes: ZC = Z C (m x q) and ZsR = Z^* R (n x q), with C (n x q) and R
// (m x q), q = rank cap r + oversampling.  Steps, in the paper's order:
//   (1) orthonormal bases Q_col of ZC and Q_row of Z^* R by pivoted QR, at
//       most r columns each (the extra probe columns keep the solves of
//       step 2 overdetermined);
//   (2) M = pinv(R^* Q_col) (R^* ZC) pinv(Q_row^* C), as two least-squares
//       solves;
//   (3) SVD of M:  Z ~ (Q_col U_M) S_M (Q_row V_M)^*, truncated.
Low matvec_svd(const Mat& ZC, const Mat& ZsR, const Mat& C, const Mat& R, double tol, int64_t rmax) {
  Low out;
  const int64_t m = ZC.m, n = ZsR.m;
  if (m == 0 || n == 0) {
    out.U0 = Mat(m, 0);
    out.V0 = Mat(n, 0);
    return out;
  }
  const double qtol = tol * 1e-2;
  const int64_t r = std::min<int64_t>(rmax, ZC.n);
  la::QRP qc = la::pivoted_qr(ZC, qtol, r);
  la::QRP qr = la::pivoted_qr(ZsR, qtol, r);
  if (qc.k == 0 || qr.k == 0) {  // Z C = 0 or Z^* R = 0: Z = 0 to the probes
    out.U0 = Mat(m, 0);
    out.V0 = Mat(n, 0);
    return out;
  }
  const Mat& Qc = qc.Q;  // m x kc
  const Mat& Qr = qr.Q;  // n x kr
  // (2) T = pinv(R^* Q_col) (R^* ZC), then M = T pinv(Q_row^* C) via M^* = lstsq((Q_row^* C)^*, T^*)
  Mat T = la::lstsq(la::matmul_ah(R, Qc), la::matmul_ah(R, ZC));     // kc x q
  Mat M = la::adjoint(la::lstsq(la::matmul_ah(C, Qr), la::adjoint(T)));  // kc x kr
  // (3) SVD of M
  la::SVD d = la::svd(M);
  const int64_t rk = la::trunc_rank(d.s, tol, rmax);
  Mat UM(M.m, rk), VM(M.n, rk);
  for (int64_t j = 0; j < rk; ++j) {
    for (int64_t i = 0; i < M.m; ++i) UM(i, j) = d.U(i, j);
    for (int64_t i = 0; i < M.n; ++i) VM(i, j) = d.V(i, j);
  }
  out.U0 = la::matmul(Qc, UM);
  out.V0 = la::matmul(Qr, VM);
  out.s.assign(d.s.begin(), d.s.begin() + rk);
  return out;
}

// Products of case (i) for one part (Section 2.3): K applied to the
// zero-padded probe C^P_B of every Omega node B at level L - m (rows: all of
// X, callback order) and K^* applied to R^P_A of every X node A at level m
// (rows: the part's Omega points, tree point order).  The black box is
// called on blocks of at most about 1 GiB.
struct MidProducts {
  std::vector<Mat> KC;   // per B: nx x q
  std::vector<Mat> KsR;  // per A: |part Omega points| x q
};

MidProducts mid_products(const Tree& xt, const Tree& ot, const std::vector<int64_t>& xs,
                         const std::vector<int64_t>& os, const MatvecSource& src) {
  const int L = xt.L, m = L / 2;
  const int64_t q = src.q, nx = src.nx, nxi = src.nxi;
  MidProducts P;
  const int64_t per_call = std::max<int64_t>(1, ((int64_t)1 << 26) / (std::max(nx, nxi) * q));
  auto call = [&](int adjoint, int64_t ncols, const std::vector<la::cd>& in, std::vector<la::cd>& out) {
    const int rc = src.mv(src.user, adjoint, ncols, reinterpret_cast<const double*>(in.data()),
                          reinterpret_cast<double*>(out.data()));
    if (rc != 0) throw CallbackError("matvec callback returned " + std::to_string(rc));
  };
  const int lb = L - m;
  P.KC.resize(ot.nn(lb));
  for (int32_t b0 = 0; b0 < ot.nn(lb); b0 += (int32_t)per_call) {
    const int32_t b1 = (int32_t)std::min<int64_t>(ot.nn(lb), b0 + per_call);
    const int64_t nc = (int64_t)(b1 - b0) * q;
    std::vector<la::cd> in((size_t)(nxi * nc)), out((size_t)(nx * nc));
    for (int32_t b = b0; b < b1; ++b)
      for (int64_t p = ot.off[lb][b]; p < ot.off[lb][b + 1]; ++p) {
        const int64_t g = os[ot.perm[p]];
        for (int64_t c = 0; c < q; ++c) in[(size_t)(g + ((b - b0) * q + c) * nxi)] = src.C[(size_t)(g + c * nxi)];
      }
    call(0, nc, in, out);
    for (int32_t b = b0; b < b1; ++b) {
      Mat Y(nx, q);
      std::copy(out.begin() + (size_t)((b - b0) * q * nx), out.begin() + (size_t)((b - b0 + 1) * q * nx), Y.a.begin());
      P.KC[b] = std::move(Y);
    }
  }
  const int64_t npart = (int64_t)os.size();
  P.KsR.resize(xt.nn(m));
  for (int32_t a0 = 0; a0 < xt.nn(m); a0 += (int32_t)per_call) {
    const int32_t a1 = (int32_t)std::min<int64_t>(xt.nn(m), a0 + per_call);
    const int64_t nc = (int64_t)(a1 - a0) * q;
    std::vector<la::cd> in((size_t)(nx * nc)), out((size_t)(nxi * nc));
    for (int32_t a = a0; a < a1; ++a)
      for (int64_t p = xt.off[m][a]; p < xt.off[m][a + 1]; ++p) {
        const int64_t g = xs[xt.perm[p]];
        for (int64_t c = 0; c < q; ++c) in[(size_t)(g + ((a - a0) * q + c) * nx)] = src.R[(size_t)(g + c * nx)];
      }
    call(1, nc, in, out);
    for (int32_t a = a0; a < a1; ++a) {
      Mat W(npart, q);
      for (int64_t c = 0; c < q; ++c)
        for (int64_t j = 0; j < npart; ++j) W(j, c) = out[(size_t)(os[j] + ((a - a0) * q + c) * nxi)];
      P.KsR[a] = std::move(W);
    }
  }
  return P;
}

// Middle-level factorization of pair (ia, ib) from the products of case (i).
Low matvec_pair(const MidProducts& P, const Tree& xt, const Tree& ot, const std::vector<int64_t>& xs,
                const std::vector<int64_t>& os, const MatvecSource& src, int32_t ia, int32_t ib, const mbf_opts& o) {
  ScopedUs timer(g_mid_us);
  const int L = xt.L, m = L / 2;
  const int64_t q = src.q;
  const int64_t ma = xt.size(m, ia), nb = ot.size(L - m, ib);
  Mat ZC(ma, q), Ra(ma, q), ZsR(nb, q), Cb(nb, q);
  for (int64_t i = 0; i < ma; ++i) {
    const int64_t g = xs[xt.perm[xt.off[m][ia] + i]];
    for (int64_t c = 0; c < q; ++c) {
      ZC(i, c) = P.KC[ib](g, c);
      Ra(i, c) = src.R[(size_t)(g + c * src.nx)];
    }
  }
  for (int64_t j = 0; j < nb; ++j) {
    const int64_t t = ot.perm[ot.off[L - m][ib] + j];
    for (int64_t c = 0; c < q; ++c) {
      ZsR(j, c) = P.KsR[ia](t, c);
      Cb(j, c) = src.C[(size_t)(os[t] + c * src.nxi)];
    }
  }
  return matvec_svd(ZC, ZsR, Cb, Ra, o.tol, o.max_rank);
}

// Progress lines on stderr when MBF_VERBOSE is set (long builds).
struct Progress {
  const char* what;
  int64_t total;
  std::atomic<int64_t> done{0};
  std::mutex mu;
  std::chrono::steady_clock::time_point last = std::chrono::steady_clock::now();
  bool on = std::getenv("MBF_VERBOSE") != nullptr;
  Progress(const char* w, int64_t t) : what(w), total(t) {}
  void tick() {
    const int64_t d = ++done;
    if (!on) return;
    std::lock_guard<std::mutex> g(mu);
    auto now = std::chrono::steady_clock::now();
    if (d == total || std::chrono::duration<double>(now - last).count() > 10.0) {
      last = now;
      std::fprintf(stderr, "[mbf build] %s %lld/%lld\n", what, (long long)d, (long long)total);
      std::fflush(stderr);
    }
  }
};

template <typename F>
void parallel_for(int64_t n, int threads, F&& fn) {
  std::atomic<int64_t> next{0};
  std::exception_ptr err;
  std::mutex mu;
  auto work = [&]() {
    for (;;) {
      const int64_t i = next.fetch_add(1);
      if (i >= n) return;
      {
        std::lock_guard<std::mutex> g(mu);
        if (err) return;
      }
      try {
        fn(i);
      } catch (...) {
        std::lock_guard<std::mutex> g(mu);
        if (!err) err = std::current_exception();
        return;
      }
    }
  };
  const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(threads, n));
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
  if (err) std::rethrow_exception(err);
}

}  // namespace

bool validate_opts(const mbf_opts& o, std::string& why) {
  if (!(o.tol >= 0.0) || o.tol >= 1.0) return why = "tol must be in [0, 1)", false;
  if (o.max_rank < 1) return why = "max_rank must be >= 1", false;
  if (o.depth < 0 || o.depth > 14) return why = "depth must be in [0, 14]", false;
  if (o.depth == 0 && (o.leaf_side < 1 || (o.leaf_side & (o.leaf_side - 1))))
    return why = "leaf_side must be a power of two", false;
  if (o.grid_n == 0) {  // general point sets
    if (o.depth < 1) return why = "general point sets (grid_n = 0) need depth >= 1", false;
    if (o.split == MBF_SPLIT_MULTISCALE) return why = "the multiscale split needs grid points (grid_n > 0)", false;
  } else if (o.grid_n < 2 || (o.grid_n & (o.grid_n - 1))) {
    return why = "grid_n must be a power of two >= 2, or 0 for general point sets", false;
  }
  if (o.split < MBF_SPLIT_NONE || o.split > MBF_SPLIT_MULTISCALE) return why = "unknown split", false;
  if (o.split == MBF_SPLIT_MULTISCALE && (o.center_side < 2 || (o.center_side & (o.center_side - 1))))
    return why = "center_side must be a power of two >= 2", false;
  if (o.oversample < 0) return why = "oversample must be >= 0", false;
  if ((o.prec_mask & 7u) == 0) return why = "empty precision mask", false;
  if (o.builder != MBF_BUILD_HOST && o.builder != MBF_BUILD_DEVICE) return why = "unknown builder", false;
  if (o.device_mem_gb < 0) return why = "device_mem_gb must be >= 0", false;
  return true;
}

// Build threads when the caller leaves the count open: OMP_NUM_THREADS when
// set (the usual cap on shared machines), else the CPUs this process may run
// on, else the hardware concurrency.
static int default_threads() {
  if (const char* e = std::getenv("OMP_NUM_THREADS")) {
    const int v = std::atoi(e);
    if (v > 0) return v;
  }
  cpu_set_t set;
  if (sched_getaffinity(0, sizeof(set), &set) == 0) {
    const int c = CPU_COUNT(&set);
    if (c > 0) return c;
  }
  return (int)std::max(1u, std::thread::hardware_concurrency());
}

namespace {
// The build of Section 2 on given trees; the middle level comes from the
// entry callback (case (ii)) or, with `src`, from products with the black
// box (case (i)).
HostFactor build_host_impl(const Tree& xt, const Tree& ot, const std::vector<int64_t>& xs,
                           const std::vector<int64_t>& os, mbf_entry_cb cb, void* user, const mbf_opts& o,
                           const MatvecSource* src) {
  HostFactor f;
  const int L = xt.L;
  const int m = L / 2;
  f.L = L;
  f.m = m;
  f.xt = xt;
  f.ot = ot;
  Ctx c{cb, user, &xs, &os};
  const int threads = o.threads > 0 ? o.threads : default_threads();
  f.rank.resize(L + 1);
  for (int s = 0; s <= L; ++s) f.rank[s].assign((size_t)xt.nn(s) * ot.nn(L - s), -1);
  // per-block outputs, filled by the owning task
  std::vector<std::vector<std::vector<la::cd>>> blk(L);
  for (int s = 0; s < L; ++s) blk[s].resize((size_t)xt.nn(s) * ot.nn(L - s - 1));
  std::vector<std::vector<double>> Smid((size_t)xt.nn(m) * ot.nn(L - m));
  f.UL.resize(xt.nn(L));
  f.V0.resize(ot.nn(L));
  // V^m of every middle-level pair, produced by the U pass (form eq. (lowrank1))
  // and consumed by the V pass: each pair is factored once.
  std::vector<Mat> Vmid((size_t)xt.nn(m) * ot.nn(L - m));

  // Descendants of node i at level l0 found at level l (contiguous range).
  auto desc = [](const Tree& t, int l0, int32_t i, int l) {
    int32_t a = i, b = i + 1;
    for (int q = l0; q < l; ++q) {
      a = t.cfirst[q][a];
      b = t.cfirst[q][b];
    }
    return std::make_pair(a, b);
  };

  // Case (i): every product with the black box up front.  Case (ii): the
  // sample size of the middle level from one probe pair.
  MidProducts mp;
  int64_t q0 = 32;
  if (src) {
    mp = mid_products(xt, ot, xs, os, *src);
  } else {
    int64_t r = 0;
    (void)middle_pair(c, xt, ot, m, 0, 0, o, 32, &r);
    q0 = std::max<int64_t>(32, r + 2 * o.oversample);
  }

  // ---------------- U tasks: one per middle-level X node
  Progress pu("U pass", xt.nn(m)), pv("V pass", ot.nn(L - m));
  Progress pm("middle-level pairs", (int64_t)xt.nn(m) * ot.nn(L - m));
  parallel_for(xt.nn(m), threads, [&](int64_t ia_m) {
    std::map<std::pair<int32_t, int32_t>, Mat> U;  // (ia, ib) at current stage
    for (int32_t ib = 0; ib < ot.nn(L - m); ++ib) {
      Low lw = src ? matvec_pair(mp, xt, ot, xs, os, *src, (int32_t)ia_m, ib, o)
                   : middle_pair(c, xt, ot, m, (int32_t)ia_m, ib, o, q0);
      pm.tick();
      const int64_t r = (int64_t)lw.s.size();
      Mat Uf = lw.U0;
      for (int64_t j = 0; j < r; ++j)
        for (int64_t i = 0; i < Uf.m; ++i) Uf(i, j) *= lw.s[j];
      std::vector<double> sinv(r);
      for (int64_t j = 0; j < r; ++j) sinv[j] = 1.0 / lw.s[j];
      const int64_t p = (int64_t)ia_m * ot.nn(L - m) + ib;
      f.rank[m][p] = (int32_t)r;
      Smid[p] = std::move(sinv);
      U[{(int32_t)ia_m, ib}] = std::move(Uf);
      Mat Vf = std::move(lw.V0);
      for (int64_t j = 0; j < r; ++j)
        for (int64_t i = 0; i < Vf.m; ++i) Vf(i, j) *= lw.s[j];
      Vmid[p] = std::move(Vf);
    }
    for (int s = m; s < L; ++s) {
      std::map<std::pair<int32_t, int32_t>, Mat> Un;
      const int lo = L - s - 1;
      auto [a0, a1] = desc(xt, m, (int32_t)ia_m, s);
      for (int32_t ia = a0; ia < a1; ++ia) {
        for (int32_t ibp = 0; ibp < ot.nn(lo); ++ibp) {
          std::vector<const Mat*> parts;
          for (int32_t ib = ot.cfirst[lo][ibp]; ib < ot.cfirst[lo][ibp + 1]; ++ib) parts.push_back(&U.at({ia, ib}));
          int64_t K = 0;
          for (auto* p : parts) K += p->n;
          std::vector<Mat> Gs;
          int64_t M = 0;
          for (int32_t it = xt.cfirst[s][ia]; it < xt.cfirst[s][ia + 1]; ++it) {
            const int64_t r0 = xt.off[s + 1][it] - xt.off[s][ia];
            const int64_t r1 = xt.off[s + 1][it + 1] - xt.off[s][ia];
            la::Trunc t;
            {
              ScopedUs timer(g_rec_us);
              t = la::truncated_svd(merge_rows(parts, r0, r1), o.tol, o.max_rank);
            }
            const int64_t r = (int64_t)t.s.size();
            Mat Uf = t.U0;
            for (int64_t j = 0; j < r; ++j)
              for (int64_t i = 0; i < Uf.m; ++i) Uf(i, j) *= t.s[j];
            f.rank[s + 1][(int64_t)it * ot.nn(lo) + ibp] = (int32_t)r;
            Un[{it, ibp}] = std::move(Uf);
            Gs.push_back(la::adjoint(t.V0));  // r x K
            M += r;
          }
          // G-side block: rows grouped by the children of ia
          std::vector<la::cd>& Wb = blk[s][(size_t)ia * ot.nn(lo) + ibp];
          Wb.assign((size_t)(M * K), la::cd(0, 0));
          int64_t m0 = 0;
          for (auto& G : Gs) {
            for (int64_t j = 0; j < K; ++j)
              for (int64_t i = 0; i < G.m; ++i) Wb[(size_t)(j * M + m0 + i)] = G(i, j);
            m0 += G.m;
          }
        }
      }
      U = std::move(Un);
    }
    auto [l0, l1] = desc(xt, m, (int32_t)ia_m, L);
    for (int32_t ia = l0; ia < l1; ++ia) {
      Mat& Uf = U.at({ia, 0});
      f.UL[ia] = std::move(Uf.a);
    }
    pu.tick();
  });

  // ---------------- V tasks: one per middle-level Omega node
  parallel_for(ot.nn(L - m), threads, [&](int64_t ib_m) {
    std::map<std::pair<int32_t, int32_t>, Mat> V;  // (ia, ib) at current stage
    for (int32_t ia = 0; ia < xt.nn(m); ++ia) {
      Mat& Vf = Vmid[(size_t)ia * ot.nn(L - m) + ib_m];
      V[{ia, (int32_t)ib_m}] = std::move(Vf);
      Vf = Mat();
    }
    for (int s = m; s >= 1; --s) {
      std::map<std::pair<int32_t, int32_t>, Mat> Vn;
      const int lb = L - s;  // Omega level of the current B nodes
      auto [b0, b1] = desc(ot, L - m, (int32_t)ib_m, lb);
      for (int32_t ib = b0; ib < b1; ++ib) {
        // H blocks of the children of ib, for every X node iap at level s-1
        for (int32_t iap = 0; iap < xt.nn(s - 1); ++iap) {
          std::vector<const Mat*> parts;
          for (int32_t ia = xt.cfirst[s - 1][iap]; ia < xt.cfirst[s - 1][iap + 1]; ++ia) parts.push_back(&V.at({ia, ib}));
          int64_t M = 0;
          for (auto* p : parts) M += p->n;
          std::vector<Mat> Hs;
          int64_t K = 0;
          for (int32_t ibc = ot.cfirst[lb][ib]; ibc < ot.cfirst[lb][ib + 1]; ++ibc) {
            const int64_t r0 = ot.off[lb + 1][ibc] - ot.off[lb][ib];
            const int64_t r1 = ot.off[lb + 1][ibc + 1] - ot.off[lb][ib];
            la::Trunc t;
            {
              ScopedUs timer(g_rec_us);
              t = la::truncated_svd(merge_rows(parts, r0, r1), o.tol, o.max_rank);
            }
            const int64_t r = (int64_t)t.s.size();
            Mat Vf = t.U0;
            for (int64_t j = 0; j < r; ++j)
              for (int64_t i = 0; i < Vf.m; ++i) Vf(i, j) *= t.s[j];
            f.rank[s - 1][(int64_t)iap * ot.nn(lb + 1) + ibc] = (int32_t)r;
            Vn[{iap, ibc}] = std::move(Vf);
            Hs.push_back(la::adjoint(t.V0));  // r x M
            K += r;
          }
          // H-side block of stage s-1 for (iap, ib): columns grouped by children of ib,
          // group sigma holds H_sigma^* (M x r_sigma)
          std::vector<la::cd>& Wb = blk[s - 1][(size_t)iap * ot.nn(lb) + ib];
          Wb.assign((size_t)(M * K), la::cd(0, 0));
          int64_t k0 = 0;
          for (auto& H : Hs) {
            for (int64_t j = 0; j < H.m; ++j)
              for (int64_t i = 0; i < M; ++i) Wb[(size_t)((k0 + j) * M + i)] = std::conj(H(j, i));
            k0 += H.m;
          }
        }
      }
      V = std::move(Vn);
    }
    auto [l0, l1] = desc(ot, L - m, (int32_t)ib_m, L);
    for (int32_t ib = l0; ib < l1; ++ib) {
      Mat& Vf = V.at({0, ib});
      f.V0[ib] = std::move(Vf.a);
    }
    pv.tick();
  });

  if (std::getenv("MBF_VERBOSE"))
    std::fprintf(stderr, "[mbf build] thread-seconds: middle level %.1f, recursion %.1f\n", g_mid_us * 1e-6,
                 g_rec_us * 1e-6);
  for (int s = 0; s <= L; ++s)
    for (auto v : f.rank[s])
      if (v < 0) throw std::runtime_error("missing rank");
  for (auto& v : Smid) f.S.insert(f.S.end(), v.begin(), v.end());
  f.W.assign(L, {});
  f.Woff.assign(L, {});
  for (int s = 0; s < L; ++s) {
    f.Woff[s].push_back(0);
    for (auto& b : blk[s]) f.Woff[s].push_back(f.Woff[s].back() + (int64_t)b.size());
    f.W[s].reserve((size_t)f.Woff[s].back());
    for (auto& b : blk[s]) {
      f.W[s].insert(f.W[s].end(), b.begin(), b.end());
      std::vector<la::cd>().swap(b);
    }
  }
  return f;
}
}  // namespace

HostFactor build_host(const Tree& xt, const Tree& ot, const std::vector<int64_t>& xs,
                      const std::vector<int64_t>& os, mbf_entry_cb cb, void* user, const mbf_opts& o) {
  return build_host_impl(xt, ot, xs, os, cb, user, o, nullptr);
}

namespace {

// Grid index of each point along both axes (points on a uniform grid of
// side n with spacing h): i = round((p - min) / h).
std::vector<int64_t> grid_index(int64_t npts, const double* p, int64_t n, int axis) {
  double lo = p[axis], hi = p[axis];
  for (int64_t i = 0; i < npts; ++i) {
    lo = std::min(lo, p[2 * i + axis]);
    hi = std::max(hi, p[2 * i + axis]);
  }
  const double h = (hi - lo) / (double)(n - 1);
  std::vector<int64_t> out(npts);
  for (int64_t i = 0; i < npts; ++i) {
    const int64_t v = h > 0 ? (int64_t)std::llround((p[2 * i + axis] - lo) / h) : 0;
    out[i] = std::min<int64_t>(std::max<int64_t>(v, 0), n - 1);
  }
  return out;
}

std::vector<int64_t> grid_leaf_codes(const std::vector<int64_t>& i1, const std::vector<int64_t>& i2, int64_t side,
                                     int L) {
  // cells of side / 2^L grid points
  const int64_t cell = side >> L;
  std::vector<int64_t> code(i1.size());
  for (size_t i = 0; i < i1.size(); ++i) code[i] = morton2(i1[i] / cell, i2[i] / cell, L);
  return code;
}

int ilog2(int64_t v) {
  int l = 0;
  while ((1ll << l) < v) ++l;
  return l;
}

Error finish_part(const HostFactor& f, const int64_t* idx_map, uint32_t mask, DevFactor& F) {
  F.parts.emplace_back();
  Error e = upload_part(f, idx_map, mask, F.parts.back());
  if (e.st != MBF_OK) return e;
  F.nnz += F.parts.back().nnz;
  for (auto& p : F.parts.back().prec) F.device_bytes += p.bytes;
  return {MBF_OK, ""};
}

Error finish_device_part(const Tree& xt, const Tree& ot, const std::vector<int64_t>& xs,
                         const std::vector<int64_t>& os, const DeviceKernel& K, const mbf_opts& o, DevFactor& F) {
  F.parts.emplace_back();
  Error e = build_part_device(xt, ot, xs, os, K, o, F.prec_mask, F.parts.back());
  if (e.st != MBF_OK) return e;
  F.nnz += F.parts.back().nnz;
  for (auto& p : F.parts.back().prec) F.device_bytes += p.bytes;
  return {MBF_OK, ""};
}

}  // namespace

namespace {
// Leaf codes of points in a square: cell (floor((p - lo) / side * 2^L)),
// the last cell closed, Morton-ordered (Fig. 1).
std::vector<int64_t> square_leaf_codes(int64_t np, const double* p, double lo0, double lo1, double side, int L) {
  const int64_t nl = (int64_t)1 << L;
  const double sc = (double)nl / side;
  std::vector<int64_t> c(np);
  for (int64_t i = 0; i < np; ++i) {
    const int64_t c1 = std::min<int64_t>(std::max<int64_t>((int64_t)std::floor((p[2 * i] - lo0) * sc), 0), nl - 1);
    const int64_t c2 = std::min<int64_t>(std::max<int64_t>((int64_t)std::floor((p[2 * i + 1] - lo1) * sc), 0), nl - 1);
    c[i] = morton2(c1, c2, L);
  }
  return c;
}

// Smallest axis-aligned square holding every point (false on a non-finite coordinate).
bool bounding_square(int64_t np, const double* p, double& lo0, double& lo1, double& side) {
  double a0 = INFINITY, a1 = INFINITY, b0 = -INFINITY, b1 = -INFINITY;
  for (int64_t i = 0; i < np; ++i) {
    const double u = p[2 * i], v = p[2 * i + 1];
    if (!std::isfinite(u) || !std::isfinite(v)) return false;
    a0 = std::min(a0, u), b0 = std::max(b0, u), a1 = std::min(a1, v), b1 = std::max(b1, v);
  }
  lo0 = a0, lo1 = a1;
  side = std::max(b0 - a0, b1 - a1);
  if (!(side > 0)) side = 1.0;
  return true;
}

// General point sets (Section 2.6: the trees follow the points and drop
// empty nodes): X and Omega in their bounding squares, or Omega through the
// polar map p = (|xi| / R, angle / 2 pi mod 1) with R = max |xi| (Section
// 3.2), both of depth opts.depth; one part, built on the host.
Error build_general(int64_t nx, const double* x, int64_t nxi, const double* xi, mbf_entry_cb cb, void* user,
                    const mbf_opts& o, DevFactor& F, const MatvecSource* src) {
  if (o.builder != MBF_BUILD_HOST) return {MBF_ERR_UNSUPPORTED, "general point sets build on the host"};
  const int L = o.depth;
  double lo0, lo1, side;
  if (!bounding_square(nx, x, lo0, lo1, side)) return {MBF_ERR_INVALID_ARG, "non-finite X coordinate"};
  std::vector<int64_t> xc = square_leaf_codes(nx, x, lo0, lo1, side, L);
  std::vector<int64_t> oc;
  if (o.split == MBF_SPLIT_POLAR) {
    double R = 0.0;
    for (int64_t i = 0; i < nxi; ++i) {
      const double r = std::hypot(xi[2 * i], xi[2 * i + 1]);
      if (!std::isfinite(r)) return {MBF_ERR_INVALID_ARG, "non-finite Omega coordinate"};
      R = std::max(R, r);
    }
    if (!(R > 0)) R = 1.0;
    std::vector<double> pp((size_t)(2 * nxi));
    for (int64_t i = 0; i < nxi; ++i) {
      const double a = xi[2 * i], b = xi[2 * i + 1];
      double p2 = (a == 0.0 && b == 0.0) ? 0.0 : std::atan2(b, a) / (2.0 * M_PI);
      pp[2 * i] = std::hypot(a, b) / R;
      pp[2 * i + 1] = p2 - std::floor(p2);
    }
    oc = square_leaf_codes(nxi, pp.data(), 0.0, 0.0, 1.0, L);
  } else {
    if (!bounding_square(nxi, xi, lo0, lo1, side)) return {MBF_ERR_INVALID_ARG, "non-finite Omega coordinate"};
    oc = square_leaf_codes(nxi, xi, lo0, lo1, side, L);
  }
  std::vector<int64_t> xs(nx), os(nxi);
  std::iota(xs.begin(), xs.end(), 0);
  std::iota(os.begin(), os.end(), 0);
  Tree xt = tree_from_leaf_codes(L, nx, xc.data());
  Tree ot = tree_from_leaf_codes(L, nxi, oc.data());
  HostFactor f = build_host_impl(xt, ot, xs, os, cb, user, o, src);
  return finish_part(f, nullptr, F.prec_mask, F);
}
}  // namespace

Error build_factor(int64_t nx, const double* x, int64_t nxi, const double* xi, mbf_entry_cb cb, void* user,
                   const mbf_opts& o, DevFactor& F, const MatvecSource* src) {
  const int64_t n = o.grid_n;
  if (n == 0) {
    F.nx = nx;
    F.nxi = nxi;
    F.prec_mask = o.prec_mask & 7u;
    return build_general(nx, x, nxi, xi, cb, user, o, F, src);
  }
  if (nx != n * n || nxi != n * n) return {MBF_ERR_INVALID_ARG, "points must form n x n grids (grid_n)"};
  if (src && o.builder != MBF_BUILD_HOST) return {MBF_ERR_UNSUPPORTED, "the matvec build runs on the host builder"};
  // Device builder: the entries are evaluated on the GPU, so the kernel must
  // be one the device knows (the ready-made callbacks).
  const bool dev = o.builder == MBF_BUILD_DEVICE;
  DeviceKernel DK;
  if (dev) {
    const auto* kp = static_cast<const mbf_kernel_params*>(user);
    if (cb == mbf_kernel_dft)
      DK.kind = 0;
    else if (cb == mbf_kernel_fio)
      DK.kind = 1;
    else
      return {MBF_ERR_UNSUPPORTED, "the device builder evaluates only mbf_kernel_dft / mbf_kernel_fio"};
    if (!kp || !kp->x || !kp->xi || kp->n <= 0) return {MBF_ERR_INVALID_ARG, "missing kernel parameters"};
    if (!(o.tol >= 1e-7)) return {MBF_ERR_UNSUPPORTED, "the device builder needs tol >= 1e-7"};
    DK.n = kp->n;
    DK.c_scale = kp->c_scale;
    DK.x = kp->x;
    DK.xi = kp->xi;
    DK.nx = nx;
    DK.nxi = nxi;
  }
  F.nx = nx;
  F.nxi = nxi;
  F.prec_mask = o.prec_mask & 7u;
  const std::vector<int64_t> x1 = grid_index(nx, x, n, 0), x2 = grid_index(nx, x, n, 1);
  const std::vector<int64_t> w1 = grid_index(nxi, xi, n, 0), w2 = grid_index(nxi, xi, n, 1);
  std::vector<int64_t> xs(nx), os(nxi);
  std::iota(xs.begin(), xs.end(), 0);
  std::iota(os.begin(), os.end(), 0);
  const int Lfull = ilog2(n / std::max(1, o.leaf_side));
  if (o.split == MBF_SPLIT_NONE || o.split == MBF_SPLIT_POLAR) {
    const int L = o.depth > 0 ? o.depth : Lfull;
    if ((1ll << L) > n) return {MBF_ERR_INVALID_ARG, "depth too large for the grid"};
    std::vector<int64_t> xc = grid_leaf_codes(x1, x2, n, L);
    std::vector<int64_t> oc;
    if (o.split == MBF_SPLIT_NONE) {
      oc = grid_leaf_codes(w1, w2, n, L);
    } else {
      // polar map of eq. (polar): p1 = |xi| / R, p2 = atan2(xi2, xi1) / 2pi mod 1, R = sqrt(2)/2 n
      oc.resize(nxi);
      const double R = std::sqrt(2.0) / 2.0 * (double)n;
      const int64_t nl = 1ll << L;
      for (int64_t i = 0; i < nxi; ++i) {
        const double a = xi[2 * i], b = xi[2 * i + 1];
        double p1 = std::hypot(a, b) / R;
        double p2 = (a == 0.0 && b == 0.0) ? 0.0 : std::atan2(b, a) / (2.0 * M_PI);
        p2 -= std::floor(p2);
        p1 = std::min(std::max(p1, 0.0), 1.0);
        const int64_t c1 = std::min<int64_t>((int64_t)std::floor(p1 * nl), nl - 1);
        const int64_t c2 = std::min<int64_t>((int64_t)std::floor(p2 * nl), nl - 1);
        oc[i] = morton2(c1, c2, L);
      }
    }
    Tree xt = tree_from_leaf_codes(L, nx, xc.data());
    Tree ot = tree_from_leaf_codes(L, nxi, oc.data());
    if (dev) return finish_device_part(xt, ot, xs, os, DK, o, F);
    HostFactor f = build_host_impl(xt, ot, xs, os, cb, user, o, src);
    return finish_part(f, nullptr, F.prec_mask, F);
  }
  // Multiscale (Section 4.1 corona split, half-open reading):
  // Omega_t = [-a_t, a_t)^2 minus [-a_t/2, a_t/2)^2 in centered grid
  // coordinates, a_t = n / 2^(t+1), down to the center [-c/2, c/2)^2.
  const int64_t half = n / 2;
  std::vector<int64_t> cen_idx;
  int t = 0;
  for (int64_t a = n / 2; a / 2 >= o.center_side / 2 && a > o.center_side / 2; a /= 2, ++t) {
    std::vector<int64_t> idx;
    for (int64_t i = 0; i < nxi; ++i) {
      const int64_t c1 = w1[i] - half, c2 = w2[i] - half;
      const bool in_a = c1 >= -a && c1 < a && c2 >= -a && c2 < a;
      const bool in_h = c1 >= -a / 2 && c1 < a / 2 && c2 >= -a / 2 && c2 < a / 2;
      if (in_a && !in_h) idx.push_back(i);
    }
    // L_t = 2 floor((L - t) / 2) (Section 4.2) with L = log2(n / leaf_side)
    const int Lt = std::max(0, 2 * ((Lfull - t) / 2));
    std::vector<int64_t> xc = grid_leaf_codes(x1, x2, n, Lt);
    std::vector<int64_t> b1(idx.size()), b2(idx.size());
    for (size_t k = 0; k < idx.size(); ++k) {
      b1[k] = w1[idx[k]] - half + a;
      b2[k] = w2[idx[k]] - half + a;
    }
    std::vector<int64_t> oc = grid_leaf_codes(b1, b2, 2 * a, Lt);
    Tree xt = tree_from_leaf_codes(Lt, nx, xc.data());
    Tree ot = tree_from_leaf_codes(Lt, (int64_t)idx.size(), oc.data());
    if (dev) {
      Error e = finish_device_part(xt, ot, xs, idx, DK, o, F);
      if (e.st != MBF_OK) return e;
      continue;
    }
    HostFactor f = build_host_impl(xt, ot, xs, idx, cb, user, o, src);
    Error e = finish_part(f, idx.data(), F.prec_mask, F);
    if (e.st != MBF_OK) return e;
  }
  const int64_t a_c = o.center_side / 2;
  for (int64_t i = 0; i < nxi; ++i) {
    const int64_t c1 = w1[i] - half, c2 = w2[i] - half;
    if (c1 >= -a_c && c1 < a_c && c2 >= -a_c && c2 < a_c) cen_idx.push_back(i);
  }
  if (!cen_idx.empty() && dev) {
    Error e = build_center_device(DK, cen_idx, F.prec_mask, F);
    if (e.st != MBF_OK) return e;
    F.nnz += nx * (int64_t)cen_idx.size();
    for (auto& p : F.center) F.device_bytes += p.bytes;
  } else if (!cen_idx.empty()) {
    std::vector<int64_t> rows(nx);
    std::iota(rows.begin(), rows.end(), 0);
    const int64_t nc = (int64_t)cen_idx.size();
    std::vector<cd> KC((size_t)(nx * nc));
    int rc;
    if (src) {  // case (i): K applied to the unit vectors of the center
      std::vector<cd> E((size_t)(nxi * nc));
      for (int64_t j = 0; j < nc; ++j) E[(size_t)(cen_idx[j] + j * nxi)] = cd(1, 0);
      rc = src->mv(src->user, 0, nc, reinterpret_cast<const double*>(E.data()), reinterpret_cast<double*>(KC.data()));
      if (rc != 0) throw CallbackError("matvec callback returned " + std::to_string(rc));
    } else {
      rc = cb(user, nx, rows.data(), nc, cen_idx.data(), reinterpret_cast<double*>(KC.data()));
      if (rc != 0) throw CallbackError("entry callback returned " + std::to_string(rc));
    }
    Error e = upload_center(F, KC, cen_idx, F.prec_mask);
    if (e.st != MBF_OK) return e;
    F.nnz += (int64_t)KC.size();
    for (auto& p : F.center) F.device_bytes += p.bytes;
  }
  return {MBF_OK, ""};
}

}  // namespace mbf

// ------------------------------------------------------------ ready-made kernels
extern "C" int mbf_kernel_dft(void* user, int64_t m, const int64_t* rows, int64_t k, const int64_t* cols,
                              double* out) {
  const auto* p = static_cast<const mbf_kernel_params*>(user);
  if (!p || !p->x || !p->xi || p->n <= 0) return 1;
  const int64_t n = p->n;
  for (int64_t b = 0; b < k; ++b) {
    const int64_t w1 = std::llround(p->xi[2 * cols[b]]), w2 = std::llround(p->xi[2 * cols[b] + 1]);
    for (int64_t a = 0; a < m; ++a) {
      const int64_t x1 = std::llround(p->x[2 * rows[a]]), x2 = std::llround(p->x[2 * rows[a] + 1]);
      int64_t q = (x1 * w1 + x2 * w2) % n;
      if (q < 0) q += n;
      const double ph = -2.0 * M_PI * ((double)q / (double)n);
      out[2 * (a + b * m)] = std::cos(ph);
      out[2 * (a + b * m) + 1] = std::sin(ph);
    }
  }
  return 0;
}

extern "C" int mbf_kernel_fio_points(void* user, int64_t m, const int64_t* rows, int64_t k, const int64_t* cols,
                                     double* out) {
  const auto* p = static_cast<const mbf_kernel_params*>(user);
  if (!p || !p->x || !p->xi) return 1;
  std::vector<double> c1(m), c2(m), y1(m), y2(m);
  for (int64_t a = 0; a < m; ++a) {
    const double x1 = p->x[2 * rows[a]], x2 = p->x[2 * rows[a] + 1];
    c1[a] = p->c_scale * (2.0 + std::sin(2.0 * M_PI * x1) * std::sin(2.0 * M_PI * x2)) / 16.0;
    c2[a] = p->c_scale * (2.0 + std::cos(2.0 * M_PI * x1) * std::cos(2.0 * M_PI * x2)) / 16.0;
    y1[a] = x1;
    y2[a] = x2;
  }
  for (int64_t b = 0; b < k; ++b) {
    const double w1 = p->xi[2 * cols[b]], w2 = p->xi[2 * cols[b] + 1];
    for (int64_t a = 0; a < m; ++a) {
      const double ph = y1[a] * w1 + y2[a] * w2 + std::sqrt(c1[a] * c1[a] * w1 * w1 + c2[a] * c2[a] * w2 * w2);
      const double arg = 2.0 * M_PI * (ph - std::floor(ph));
      out[2 * (a + b * m)] = std::cos(arg);
      out[2 * (a + b * m) + 1] = std::sin(arg);
    }
  }
  return 0;
}

extern "C" int mbf_kernel_fio(void* user, int64_t m, const int64_t* rows, int64_t k, const int64_t* cols,
                              double* out) {
  const auto* p = static_cast<const mbf_kernel_params*>(user);
  if (!p || !p->x || !p->xi || p->n <= 0) return 1;
  const int64_t n = p->n;
  std::vector<double> c1(m), c2(m);
  std::vector<int64_t> n1(m), n2(m);
  for (int64_t a = 0; a < m; ++a) {
    const double x1 = p->x[2 * rows[a]], x2 = p->x[2 * rows[a] + 1];
    c1[a] = p->c_scale * (2.0 + std::sin(2.0 * M_PI * x1) * std::sin(2.0 * M_PI * x2)) / 16.0;
    c2[a] = p->c_scale * (2.0 + std::cos(2.0 * M_PI * x1) * std::cos(2.0 * M_PI * x2)) / 16.0;
    n1[a] = std::llround(x1 * (double)n);
    n2[a] = std::llround(x2 * (double)n);
  }
  for (int64_t b = 0; b < k; ++b) {
    const double w1 = p->xi[2 * cols[b]], w2 = p->xi[2 * cols[b] + 1];
    const int64_t i1 = std::llround(w1), i2 = std::llround(w2);
    for (int64_t a = 0; a < m; ++a) {
      // x.xi = (n1 xi1 + n2 xi2) / n, integer part reduced exactly
      int64_t q = (n1[a] * i1 + n2[a] * i2) % n;
      if (q < 0) q += n;
      const double ph = (double)q / (double)n + std::sqrt(c1[a] * c1[a] * w1 * w1 + c2[a] * c2[a] * w2 * w2);
      const double arg = 2.0 * M_PI * (ph - std::floor(ph));
      out[2 * (a + b * m)] = std::cos(arg);
      out[2 * (a + b * m) + 1] = std::sin(arg);
    }
  }
  return 0;
}
