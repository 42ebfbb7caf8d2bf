// Upload of host factorizations to HBM in the apply layout (see device.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>

#include "device.h"

namespace mbf {

namespace {

struct bf16x4 {
  uint16_t v[4];
};

template <typename T>
Error dev_alloc_copy(void** dst, const T* src, size_t count, size_t& bytes) {
  *dst = nullptr;
  if (count == 0) return {MBF_OK, ""};
  size_t nb = count * sizeof(T);
  hipError_t e = hipMalloc(dst, nb);
  if (e != hipSuccess) {
    *dst = nullptr;
    return {e == hipErrorOutOfMemory ? MBF_ERR_OOM : MBF_ERR_HIP,
            std::string("hipMalloc failed: ") + hipGetErrorString(e)};
  }
  e = hipMemcpy(*dst, src, nb, hipMemcpyHostToDevice);
  if (e != hipSuccess) return {MBF_ERR_HIP, std::string("hipMemcpy failed: ") + hipGetErrorString(e)};
  bytes += nb;
  return {MBF_OK, ""};
}

// Round-to-nearest-even FP32 -> BF16 (bit manipulation; NaN kept quiet).
inline uint16_t f2bf(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
inline float bf2f(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// Convert complex128 data to the storage type of precision p.
Error upload_complex(int p, const cd* src, size_t count, void** dst, size_t& bytes) {
  if (p == MBF_C128) return dev_alloc_copy(dst, reinterpret_cast<const double*>(src), 2 * count, bytes);
  std::vector<float> tmp(2 * count);
  for (size_t i = 0; i < count; ++i) {
    tmp[2 * i] = (float)src[i].real();
    tmp[2 * i + 1] = (float)src[i].imag();
  }
  return dev_alloc_copy(dst, tmp.data(), tmp.size(), bytes);
}

// Stage blocks for the split-BF16 path: per complex entry (re_hi, im_hi,
// re_lo, im_lo) with hi = bf16(x), lo = bf16(x - hi).
Error upload_split(const cd* src, size_t count, void** dst, size_t& bytes) {
  std::vector<bf16x4> tmp(count);
  for (size_t i = 0; i < count; ++i) {
    float re = (float)src[i].real(), im = (float)src[i].imag();
    uint16_t rh = f2bf(re), ih = f2bf(im);
    tmp[i].v[0] = rh;
    tmp[i].v[1] = ih;
    tmp[i].v[2] = f2bf(re - bf2f(rh));
    tmp[i].v[3] = f2bf(im - bf2f(ih));
  }
  return dev_alloc_copy(dst, tmp.data(), tmp.size(), bytes);
}

// Convert `count` complex128 entries to the storage of precision p and copy
// them to dst (device), in chunks.
Error copy_blocks(int p, const cd* src, size_t count, void* dst) {
  const size_t chunk = (size_t)1 << 24;
  for (size_t o = 0; o < count; o += chunk) {
    const size_t c = std::min(chunk, count - o);
    hipError_t e;
    if (p == MBF_C128) {
      e = hipMemcpy((char*)dst + o * 16, src + o, c * 16, hipMemcpyHostToDevice);
    } else if (p == MBF_C64) {
      std::vector<float> t(2 * c);
      for (size_t i = 0; i < c; ++i) {
        t[2 * i] = (float)src[o + i].real();
        t[2 * i + 1] = (float)src[o + i].imag();
      }
      e = hipMemcpy((char*)dst + o * 8, t.data(), c * 8, hipMemcpyHostToDevice);
    } else {
      std::vector<bf16x4> t(c);
      for (size_t i = 0; i < c; ++i) {
        float re = (float)src[o + i].real(), im = (float)src[o + i].imag();
        uint16_t rh = f2bf(re), ih = f2bf(im);
        t[i].v[0] = rh;
        t[i].v[1] = ih;
        t[i].v[2] = f2bf(re - bf2f(rh));
        t[i].v[3] = f2bf(im - bf2f(ih));
      }
      e = hipMemcpy((char*)dst + o * 8, t.data(), c * 8, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return {MBF_ERR_HIP, std::string("hipMemcpy failed: ") + hipGetErrorString(e)};
  }
  return {MBF_OK, ""};
}

Error upload_real(int p, const double* src, size_t count, void** dst, size_t& bytes) {
  if (p == MBF_C128) return dev_alloc_copy(dst, src, count, bytes);
  std::vector<float> tmp(count);
  for (size_t i = 0; i < count; ++i) tmp[i] = (float)src[i];
  return dev_alloc_copy(dst, tmp.data(), count, bytes);
}

#define MBF_TRY(expr)                   \
  do {                                  \
    Error _e = (expr);                  \
    if (_e.st != MBF_OK) return _e;     \
  } while (0)

}  // namespace

Error layout_part(const Tree& xt, const Tree& ot, int L, int m, const std::vector<std::vector<int32_t>>& rank,
                  const int64_t* idx_map, DevPart& P, std::vector<int64_t>* blk_off) {
  auto pair = [&](int s, int32_t ia, int32_t ib) { return (int64_t)ia * ot.nn(L - s) + ib; };
  P.L = L;
  P.m = m;
  P.nx = xt.npts;
  P.nxi = ot.npts;
  std::vector<std::vector<int64_t>> roff(L + 1);
  P.rows.assign(L + 1, 0);
  P.ld.assign(L + 1, 0);
  P.max_rank.assign(L + 1, 0);
  for (int s = 0; s <= L; ++s) {
    const auto& rk = rank[s];
    if ((int64_t)rk.size() != (int64_t)xt.nn(s) * ot.nn(L - s)) return {MBF_ERR_INVALID_ARG, "rank table size"};
    roff[s].resize(rk.size() + 1);
    int64_t acc = 0;
    for (size_t p = 0; p < rk.size(); ++p) {
      if (rk[p] < 0) return {MBF_ERR_INVALID_ARG, "negative rank"};
      roff[s][p] = acc;
      acc += rk[p];
      P.max_rank[s] = std::max(P.max_rank[s], rk[p]);
    }
    roff[s][rk.size()] = acc;
    if (acc > INT32_MAX) return {MBF_ERR_UNSUPPORTED, "stage state exceeds 2^31 rows"};
    P.rows[s] = acc;
    P.ld[s] = std::max<int64_t>(4, (acc + 3) / 4 * 4);
  }
  // Stage block descriptors; blocks are stored in block order, so a block's
  // offset inside its stage is the sum of M * K over the blocks before it.
  std::vector<BlockDesc> blks;
  P.nblk.assign(L, 0);
  P.blk_first.assign(L, 0);
  P.w_stage_off.assign(L, 0);
  P.max_M.assign(L, 0);
  P.max_K.assign(L, 0);
  if (blk_off) blk_off->clear();
  int64_t woff = 0;
  for (int s = 0; s < L; ++s) {
    const int lo = L - s - 1;
    P.blk_first[s] = (int64_t)blks.size();
    P.w_stage_off[s] = woff;
    int64_t b = 0, soff = 0;
    for (int32_t ia = 0; ia < xt.nn(s); ++ia)
      for (int32_t ibp = 0; ibp < ot.nn(lo); ++ibp, ++b) {
        BlockDesc d{};
        d.w_off = soff;
        const int32_t ib0 = ot.cfirst[lo][ibp], ib1 = ot.cfirst[lo][ibp + 1];
        d.in_row = (int32_t)roff[s][pair(s, ia, ib0)];
        d.K = (int32_t)(roff[s][pair(s, ia, ib1 - 1) + 1] - d.in_row);
        int32_t M = 0, t = 0;
        for (int32_t it = xt.cfirst[s][ia]; it < xt.cfirst[s][ia + 1]; ++it, ++t) {
          const int64_t p = pair(s + 1, it, ibp);
          d.ms[t] = M;
          d.orow[t] = (int32_t)roff[s + 1][p];
          M += rank[s + 1][p];
        }
        for (; t < 4; ++t) {
          d.ms[t] = M;
          d.orow[t] = 0;
        }
        d.M = M;
        P.max_M[s] = std::max(P.max_M[s], d.M);
        P.max_K[s] = std::max(P.max_K[s], d.K);
        if (blk_off) blk_off->push_back(soff);
        soff += (int64_t)d.M * d.K;
        blks.push_back(d);
      }
    P.nblk[s] = b;
    woff += soff;
  }
  P.w_elems = woff;
  // Leaves.
  std::vector<LeafDesc> vl, ul;
  int64_t fo = 0;
  for (int32_t ib = 0; ib < ot.nn(L); ++ib) {
    LeafDesc d{};
    d.f_off = fo;
    d.p_off = (int32_t)ot.off[L][ib];
    d.np = (int32_t)ot.size(L, ib);
    d.r = rank[0][pair(0, 0, ib)];
    d.row = (int32_t)roff[0][pair(0, 0, ib)];
    fo += (int64_t)d.np * d.r;
    P.max_vnp = std::max(P.max_vnp, d.np);
    P.max_vr = std::max(P.max_vr, d.r);
    vl.push_back(d);
  }
  P.v_elems = fo;
  fo = 0;
  for (int32_t ia = 0; ia < xt.nn(L); ++ia) {
    LeafDesc d{};
    d.f_off = fo;
    d.p_off = (int32_t)xt.off[L][ia];
    d.np = (int32_t)xt.size(L, ia);
    d.r = rank[L][pair(L, ia, 0)];
    d.row = (int32_t)roff[L][pair(L, ia, 0)];
    fo += (int64_t)d.np * d.r;
    P.max_unp = std::max(P.max_unp, d.np);
    P.max_ur = std::max(P.max_ur, d.r);
    ul.push_back(d);
  }
  P.u_elems = fo;
  P.n_vleaf = (int32_t)vl.size();
  P.n_uleaf = (int32_t)ul.size();
  P.s_elems = P.rows[m];
  P.nnz = P.w_elems + P.v_elems + P.u_elems + P.s_elems;

  std::vector<int32_t> vidx(ot.npts), uidx(xt.npts);
  for (int64_t i = 0; i < ot.npts; ++i) vidx[i] = (int32_t)(idx_map ? idx_map[ot.perm[i]] : ot.perm[i]);
  for (int64_t i = 0; i < xt.npts; ++i) uidx[i] = (int32_t)xt.perm[i];

  size_t meta = 0;
  MBF_TRY(dev_alloc_copy((void**)&P.d_blk, blks.data(), blks.size(), meta));
  MBF_TRY(dev_alloc_copy((void**)&P.d_vleaf, vl.data(), vl.size(), meta));
  MBF_TRY(dev_alloc_copy((void**)&P.d_uleaf, ul.data(), ul.size(), meta));
  MBF_TRY(dev_alloc_copy((void**)&P.d_vidx, vidx.data(), vidx.size(), meta));
  MBF_TRY(dev_alloc_copy((void**)&P.d_uidx, uidx.data(), uidx.size(), meta));
  return {MBF_OK, ""};
}

Error upload_part(const HostFactor& f, const int64_t* idx_map, uint32_t prec_mask, DevPart& P) {
  const int L = f.L;
  MBF_TRY(layout_part(f.xt, f.ot, L, f.m, f.rank, idx_map, P, nullptr));
  for (int s = 0; s < L; ++s) {
    const int64_t e = (s + 1 < L ? P.w_stage_off[s + 1] : P.w_elems) - P.w_stage_off[s];
    if (e != (int64_t)f.W[s].size()) return {MBF_ERR_INVALID_ARG, "block size mismatch at stage " + std::to_string(s)};
  }
  for (int32_t ib = 0; ib < f.ot.nn(L); ++ib)
    if (f.ot.size(L, ib) * f.rank[0][f.pair(0, 0, ib)] != (int64_t)f.V0[ib].size())
      return {MBF_ERR_INVALID_ARG, "Omega leaf factor size mismatch"};
  for (int32_t ia = 0; ia < f.xt.nn(L); ++ia)
    if (f.xt.size(L, ia) * f.rank[L][f.pair(L, ia, 0)] != (int64_t)f.UL[ia].size())
      return {MBF_ERR_INVALID_ARG, "X leaf factor size mismatch"};
  if ((int64_t)f.S.size() != P.rows[f.m]) return {MBF_ERR_INVALID_ARG, "middle scaling size mismatch"};
  P.nnz = host_nnz(f);
  const int64_t woff = P.w_elems;

  // Upload stage by stage (no host copy of the whole factorization).
  for (int p = 0; p < kNumPrec; ++p) {
    if (!(prec_mask & (1u << p))) continue;
    PrecData& d = P.prec[p];
    d.present = true;
    const int leafp = (p == MBF_C128) ? MBF_C128 : MBF_C64;
    const size_t esz = (p == MBF_C128) ? 16 : 8;
    d.Wst.assign(L, nullptr);
    if (woff > 0) {
      void* W = nullptr;
      hipError_t e = hipMalloc(&W, (size_t)woff * esz);
      if (e != hipSuccess)
        return {e == hipErrorOutOfMemory ? MBF_ERR_OOM : MBF_ERR_HIP,
                std::string("hipMalloc (stage blocks) failed: ") + hipGetErrorString(e)};
      d.Walloc.push_back(W);
      d.bytes += (size_t)woff * esz;
      for (int s = 0; s < L; ++s) {
        d.Wst[s] = (char*)W + (size_t)P.w_stage_off[s] * esz;
        MBF_TRY(copy_blocks(p, f.W[s].data(), f.W[s].size(), d.Wst[s]));
      }
    }
    std::vector<cd> tmp;
    tmp.reserve((size_t)std::max(P.v_elems, P.u_elems));
    for (auto& v : f.V0) tmp.insert(tmp.end(), v.begin(), v.end());
    MBF_TRY(upload_complex(leafp, tmp.data(), tmp.size(), &d.V0, d.bytes));
    tmp.clear();
    for (auto& v : f.UL) tmp.insert(tmp.end(), v.begin(), v.end());
    MBF_TRY(upload_complex(leafp, tmp.data(), tmp.size(), &d.UL, d.bytes));
    MBF_TRY(upload_real(leafp, f.S.data(), f.S.size(), &d.S, d.bytes));
  }
  return {MBF_OK, ""};
}

Error upload_center(DevFactor& F, const std::vector<cd>& KC, const std::vector<int64_t>& idx,
                    uint32_t prec_mask) {
  F.n_center = (int64_t)idx.size();
  std::vector<int32_t> ci(idx.begin(), idx.end());
  size_t meta = 0;
  MBF_TRY(dev_alloc_copy((void**)&F.d_center_idx, ci.data(), ci.size(), meta));
  for (int p = 0; p < kNumPrec; ++p) {
    if (!(prec_mask & (1u << p))) continue;
    PrecData& d = F.center[p];
    d.present = true;
    MBF_TRY(upload_complex(p == MBF_C128 ? MBF_C128 : MBF_C64, KC.data(), KC.size(), &d.center, d.bytes));
  }
  return {MBF_OK, ""};
}

static void free_prec(PrecData& d) {
  for (void* w : d.Walloc) (void)hipFree(w);
  (void)hipFree(d.V0);
  (void)hipFree(d.UL);
  (void)hipFree(d.S);
  (void)hipFree(d.center);
  d = PrecData{};
}

void free_factor(DevFactor& F) {
  for (auto& P : F.parts) {
    (void)hipFree(P.d_blk);
    (void)hipFree(P.d_vleaf);
    (void)hipFree(P.d_uleaf);
    (void)hipFree(P.d_vidx);
    (void)hipFree(P.d_uidx);
    for (auto& d : P.prec) free_prec(d);
  }
  F.parts.clear();
  (void)hipFree(F.d_center_idx);
  F.d_center_idx = nullptr;
  for (auto& d : F.center) free_prec(d);
}

}  // namespace mbf
