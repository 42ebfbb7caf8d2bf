// Host-side tree construction and block assembly (see factor.h).
#include <algorithm>
#include <numeric>
#include <stdexcept>

#include "factor.h"

namespace mbf {

int64_t morton2(int64_t c1, int64_t c2, int level) {
  int64_t code = 0;
  for (int b = 0; b < level; ++b) {
    code |= ((c1 >> b) & 1) << (2 * b + 1);
    code |= ((c2 >> b) & 1) << (2 * b);
  }
  return code;
}

Tree tree_from_leaf_codes(int L, int64_t npts, const int64_t* leaf_code) {
  Tree t;
  t.L = L;
  t.npts = npts;
  t.perm.resize(npts);
  std::iota(t.perm.begin(), t.perm.end(), 0);
  std::stable_sort(t.perm.begin(), t.perm.end(),
                   [&](int64_t a, int64_t b) { return leaf_code[a] < leaf_code[b]; });
  t.code.resize(L + 1);
  t.off.resize(L + 1);
  t.cfirst.resize(L);
  for (int l = 0; l <= L; ++l) {
    const int sh = 2 * (L - l);
    auto& c = t.code[l];
    auto& o = t.off[l];
    for (int64_t i = 0; i < npts; ++i) {
      int64_t cc = leaf_code[t.perm[i]] >> sh;
      if (c.empty() || c.back() != cc) {
        c.push_back(cc);
        o.push_back(i);
      }
    }
    o.push_back(npts);
  }
  for (int l = 0; l < L; ++l) {
    auto& cf = t.cfirst[l];
    cf.resize(t.nn(l) + 1);
    int32_t j = 0;
    for (int32_t i = 0; i < t.nn(l); ++i) {
      cf[i] = j;
      while (j < t.nn(l + 1) && (t.code[l + 1][j] >> 2) == t.code[l][i]) ++j;
    }
    cf[t.nn(l)] = j;
    if (j != t.nn(l + 1)) throw std::runtime_error("tree children are inconsistent");
  }
  return t;
}

int64_t host_nnz(const HostFactor& f) {
  int64_t t = 0;
  for (auto& v : f.V0) t += (int64_t)v.size();
  for (auto& v : f.UL) t += (int64_t)v.size();
  for (auto& w : f.W) t += (int64_t)w.size();
  t += (int64_t)f.S.size();
  t += (int64_t)f.center.size();
  return t;
}

// Row counts per block side.  For stage s and block (ia, ib'):
//   K = sum over Omega children ib of ib' of rank_s(ia, ib)
//   M = sum over X children ia_t of ia of rank_{s+1}(ia_t, ib')
void assemble_blocks(HostFactor& f, const double* h_blocks, const double* g_blocks) {
  const int L = f.L, m = f.m;
  const cd* H = reinterpret_cast<const cd*>(h_blocks);
  const cd* G = reinterpret_cast<const cd*>(g_blocks);
  f.W.assign(L, {});
  f.Woff.assign(L, {});
  for (int s = 0; s < L; ++s) {
    const Tree& xt = f.xt;
    const Tree& ot = f.ot;
    const int lo = L - s - 1;  // Omega level of B'
    auto& Woff = f.Woff[s];
    Woff.push_back(0);
    // first pass: sizes
    for (int32_t ia = 0; ia < xt.nn(s); ++ia)
      for (int32_t ibp = 0; ibp < ot.nn(lo); ++ibp) {
        int64_t K = 0, M = 0;
        for (int32_t ib = ot.cfirst[lo][ibp]; ib < ot.cfirst[lo][ibp + 1]; ++ib)
          K += f.rank[s][f.pair(s, ia, ib)];
        for (int32_t it = xt.cfirst[s][ia]; it < xt.cfirst[s][ia + 1]; ++it)
          M += f.rank[s + 1][f.pair(s + 1, it, ibp)];
        Woff.push_back(Woff.back() + M * K);
      }
    auto& W = f.W[s];
    W.assign(Woff.back(), cd(0, 0));
    int64_t blk = 0;
    for (int32_t ia = 0; ia < xt.nn(s); ++ia)
      for (int32_t ibp = 0; ibp < ot.nn(lo); ++ibp, ++blk) {
        std::vector<int64_t> kr, mr;  // ranks of the inputs / outputs
        for (int32_t ib = ot.cfirst[lo][ibp]; ib < ot.cfirst[lo][ibp + 1]; ++ib)
          kr.push_back(f.rank[s][f.pair(s, ia, ib)]);
        for (int32_t it = xt.cfirst[s][ia]; it < xt.cfirst[s][ia + 1]; ++it)
          mr.push_back(f.rank[s + 1][f.pair(s + 1, it, ibp)]);
        int64_t K = 0, M = 0;
        for (auto v : kr) K += v;
        for (auto v : mr) M += v;
        cd* Wb = W.data() + Woff[blk];
        if (s < m) {
          // H-side: columns k of group sigma come from H_{child_sigma B', A}^*
          int64_t k0 = 0;
          for (size_t sg = 0; sg < kr.size(); ++sg) {
            const int64_t r = kr[sg];  // rows of H block
            for (int64_t j = 0; j < r; ++j)
              for (int64_t i = 0; i < M; ++i) Wb[(k0 + j) * M + i] = std::conj(H[j + i * r]);
            H += r * M;
            k0 += r;
          }
        } else {
          // G-side: rows of group tau come from G_{child_tau A, B'} (r_tau x K)
          int64_t m0 = 0;
          for (size_t tg = 0; tg < mr.size(); ++tg) {
            const int64_t r = mr[tg];
            for (int64_t j = 0; j < K; ++j)
              for (int64_t i = 0; i < r; ++i) Wb[j * M + m0 + i] = G[i + j * r];
            G += r * K;
            m0 += r;
          }
        }
      }
  }
}

}  // namespace mbf
