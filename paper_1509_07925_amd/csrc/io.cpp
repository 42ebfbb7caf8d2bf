// Versioned binary files of device-resident factorizations (mbf_save /
// mbf_load): builds take minutes at N = 512^2, so a factorization is kept
// on disk and reloaded to HBM instead of rebuilt.
//
// Layout (little endian):
//   "MBFFACT1" | u32 version | u32 prec_mask | i64 nx | i64 nxi | i64 n_center
//   | u32 nparts | parts... | center... | "MBFEND01" | u64 payload bytes
//   | u64 checksum
// Each part: scalars, per-stage vectors, block and leaf descriptors, point
// indices, then for every precision in the mask its stage blocks (stage by
// stage) and V0 / UL / S arrays.  The checksum is a multiply-xor hash of
// the payload bytes.  A file is loaded only when every descriptor and index
// addresses memory inside its arrays (checked on the host before upload).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "device.h"

namespace mbf {
namespace {

constexpr uint32_t kVersion = 2;
const char kMagic[9] = "MBFFACT1";
const char kEnd[9] = "MBFEND01";

struct File {
  FILE* f = nullptr;
  uint64_t bytes = 0;
  uint64_t hash = 0x84222325cbf29ce4ull;
  bool ok = true;
  ~File() {
    if (f) std::fclose(f);
  }
  // Payload hash over the byte stream: little-endian 8-byte words (the last
  // one zero-padded), h = rotl29((h ^ word) * 0x100000001b3).  Bytes are
  // carried across calls, so the hash does not depend on how the stream was
  // cut into reads or writes.
  uint64_t pend = 0;
  int npend = 0;
  void absorb(uint64_t w) {
    hash = (hash ^ w) * 0x100000001b3ull;
    hash = (hash << 29) | (hash >> 35);
  }
  void mix(const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    size_t i = 0;
    while (i < n && npend > 0) {
      pend |= (uint64_t)c[i++] << (8 * npend);
      if (++npend == 8) {
        absorb(pend);
        pend = 0;
        npend = 0;
      }
    }
    for (; i + 8 <= n; i += 8) {
      uint64_t w;
      std::memcpy(&w, c + i, 8);
      absorb(w);
    }
    for (; i < n; ++i) pend |= (uint64_t)c[i] << (8 * npend++);
  }
  uint64_t digest() {
    uint64_t h = hash;
    if (npend > 0) {
      h = (h ^ pend) * 0x100000001b3ull;
      h = (h << 29) | (h >> 35);
    }
    return h;
  }
  void w(const void* p, size_t n) {
    if (ok && n && std::fwrite(p, 1, n, f) != n) ok = false;
    if (n) mix(p, n);
    bytes += n;
  }
  void r(void* p, size_t n) {
    if (ok && n && std::fread(p, 1, n, f) != n) ok = false;
    if (ok && n) mix(p, n);
    bytes += n;
  }
  template <typename T>
  void wv(const std::vector<T>& v) {
    const uint64_t n = v.size();
    w(&n, 8);
    w(v.data(), n * sizeof(T));
  }
  template <typename T>
  void rv(std::vector<T>& v, uint64_t cap) {
    uint64_t n = 0;
    r(&n, 8);
    if (!ok || n > cap) {
      ok = false;
      return;
    }
    v.resize(n);
    r(v.data(), n * sizeof(T));
  }
};

// device -> file in chunks
bool dev_to_file(File& F, const void* d, size_t bytes) {
  const size_t chunk = (size_t)1 << 28;
  std::vector<char> buf(std::min(bytes, chunk));
  for (size_t o = 0; o < bytes; o += chunk) {
    const size_t c = std::min(chunk, bytes - o);
    if (hipMemcpy(buf.data(), (const char*)d + o, c, hipMemcpyDeviceToHost) != hipSuccess) return false;
    F.w(buf.data(), c);
  }
  return F.ok;
}

// file -> new device allocation
Error file_to_dev(File& F, void** d, size_t bytes, size_t& total) {
  *d = nullptr;
  if (bytes == 0) return {MBF_OK, ""};
  if (hipMalloc(d, bytes) != hipSuccess) {
    *d = nullptr;
    return {MBF_ERR_OOM, "hipMalloc failed while loading"};
  }
  total += bytes;
  const size_t chunk = (size_t)1 << 28;
  std::vector<char> buf(std::min(bytes, chunk));
  for (size_t o = 0; o < bytes; o += chunk) {
    const size_t c = std::min(chunk, bytes - o);
    F.r(buf.data(), c);
    if (!F.ok) return {MBF_ERR_IO, "truncated factor file"};
    if (hipMemcpy((char*)*d + o, buf.data(), c, hipMemcpyHostToDevice) != hipSuccess)
      return {MBF_ERR_HIP, "hipMemcpy failed while loading"};
  }
  return {MBF_OK, ""};
}

// file -> host vector (descriptors and indices are checked before upload)
template <typename T>
bool file_to_host(File& F, std::vector<T>& v, int64_t count) {
  if (count < 0 || count > ((int64_t)1 << 40) / (int64_t)sizeof(T)) return false;
  v.resize((size_t)count);
  F.r(v.data(), (size_t)count * sizeof(T));
  return F.ok;
}

template <typename T>
Error host_to_dev(void** d, const std::vector<T>& v, size_t& total) {
  *d = nullptr;
  if (v.empty()) return {MBF_OK, ""};
  const size_t bytes = v.size() * sizeof(T);
  if (hipMalloc(d, bytes) != hipSuccess) {
    *d = nullptr;
    return {MBF_ERR_OOM, "hipMalloc failed while loading"};
  }
  total += bytes;
  if (hipMemcpy(*d, v.data(), bytes, hipMemcpyHostToDevice) != hipSuccess)
    return {MBF_ERR_HIP, "hipMemcpy failed while loading"};
  return {MBF_OK, ""};
}

size_t elem(int p) { return p == MBF_C128 ? 16 : 8; }
size_t leaf_elem(int p) { return p == MBF_C128 ? 16 : 8; }
size_t real_elem(int p) { return p == MBF_C128 ? 8 : 4; }

#define IO_TRY(expr)                \
  do {                              \
    Error _e = (expr);              \
    if (_e.st != MBF_OK) return _e; \
  } while (0)

}  // namespace

namespace {

int64_t stage_elems(const DevPart& P, int s) {
  return ((s + 1 < P.L) ? P.w_stage_off[s + 1] : P.w_elems) - P.w_stage_off[s];
}

// Every field the apply indexes with must stay inside its arrays: stage
// vectors of the right length, state rows within int32, block descriptors
// inside their stage's elements and the state rows of stages s and s+1,
// leaf descriptors inside the leaf arrays, the point-index slices and the
// state rows of stage 0 / L, point indices inside [0, nx) / [0, nxi).
bool check_part(const DevPart& P, int64_t nxi_total, const std::vector<BlockDesc>& blk,
                const std::vector<LeafDesc>& vl, const std::vector<LeafDesc>& ul, const std::vector<int32_t>& vidx,
                const std::vector<int32_t>& uidx, std::string& why) {
  const int L = P.L;
  auto bad = [&](const std::string& w) {
    why = w;
    return false;
  };
  if (P.m < 0 || P.m > L) return bad("middle level out of range");
  if (P.rows.size() != (size_t)L + 1 || P.ld.size() != (size_t)L + 1 || P.max_rank.size() != (size_t)L + 1 ||
      P.nblk.size() != (size_t)L || P.blk_first.size() != (size_t)L || P.w_stage_off.size() != (size_t)L ||
      P.max_M.size() != (size_t)L || P.max_K.size() != (size_t)L)
    return bad("stage vectors of the wrong length");
  for (int s = 0; s <= L; ++s) {
    if (P.rows[s] < 0 || P.rows[s] > INT32_MAX || P.ld[s] < P.rows[s] || P.ld[s] < 1) return bad("state rows");
    if (P.max_rank[s] < 0 || P.max_rank[s] > P.rows[s]) return bad("max rank");
  }
  int64_t nb = 0;
  for (int s = 0; s < L; ++s) {
    if (P.nblk[s] < 0 || P.blk_first[s] != nb) return bad("block counts");
    nb += P.nblk[s];
    const int64_t lo = P.w_stage_off[s], hi = (s + 1 < L) ? P.w_stage_off[s + 1] : P.w_elems;
    if (lo < 0 || hi < lo || hi > P.w_elems || (s == 0 && lo != 0)) return bad("stage offsets");
  }
  if ((int64_t)blk.size() != nb) return bad("block descriptor count");
  for (int s = 0; s < L; ++s) {
    const int64_t se = stage_elems(P, s);
    int32_t mM = 0, mK = 0;
    for (int64_t b = P.blk_first[s]; b < P.blk_first[s] + P.nblk[s]; ++b) {
      const BlockDesc& d = blk[(size_t)b];
      if (d.M < 0 || d.K < 0 || d.w_off < 0 || d.w_off + (int64_t)d.M * d.K > se) return bad("block outside its stage");
      if (d.in_row < 0 || (int64_t)d.in_row + d.K > P.rows[s]) return bad("block input rows");
      if (d.ms[0] != 0) return bad("block output groups");
      for (int t = 0; t < 4; ++t) {
        const int32_t end = t < 3 ? d.ms[t + 1] : d.M;
        if (d.ms[t] < 0 || end < d.ms[t] || end > d.M) return bad("block output groups");
        if (end > d.ms[t] && (d.orow[t] < 0 || (int64_t)d.orow[t] + (end - d.ms[t]) > P.rows[s + 1]))
          return bad("block output rows");
      }
      mM = std::max(mM, d.M);
      mK = std::max(mK, d.K);
    }
    if (mM != P.max_M[s] || mK != P.max_K[s]) return bad("block size maxima");
  }
  auto leaves = [&](const std::vector<LeafDesc>& lv, int32_t n, int64_t elems, int64_t npts, int64_t rows,
                    int32_t mnp, int32_t mr) {
    if ((int64_t)lv.size() != n) return false;
    int32_t gnp = 0, gr = 0;
    for (const LeafDesc& d : lv) {
      if (d.np < 0 || d.r < 0 || d.f_off < 0 || d.f_off + (int64_t)d.np * d.r > elems) return false;
      if (d.p_off < 0 || (int64_t)d.p_off + d.np > npts) return false;
      if (d.row < 0 || (int64_t)d.row + d.r > rows) return false;
      gnp = std::max(gnp, d.np);
      gr = std::max(gr, d.r);
    }
    return gnp == mnp && gr == mr;
  };
  if (!leaves(vl, P.n_vleaf, P.v_elems, P.nxi, P.rows[0], P.max_vnp, P.max_vr)) return bad("Omega leaf descriptors");
  if (!leaves(ul, P.n_uleaf, P.u_elems, P.nx, P.rows[L], P.max_unp, P.max_ur)) return bad("X leaf descriptors");
  if (P.s_elems != P.rows[P.m]) return bad("middle scaling length");
  for (int32_t v : vidx)
    if (v < 0 || v >= nxi_total) return bad("Omega point index");
  for (int32_t v : uidx)
    if (v < 0 || v >= P.nx) return bad("X point index");
  return true;
}

}  // namespace

Error save_factor(const DevFactor& D, uint32_t mask, const char* path) {
  File F;
  F.f = std::fopen(path, "wb");
  if (!F.f) return {MBF_ERR_IO, std::string("cannot open ") + path};
  F.w(kMagic, 8);
  F.w(&kVersion, 4);
  F.w(&mask, 4);
  F.w(&D.nx, 8);
  F.w(&D.nxi, 8);
  F.w(&D.n_center, 8);
  const uint32_t np = (uint32_t)D.parts.size();
  F.w(&np, 4);
  for (const DevPart& P : D.parts) {
    const int32_t hdr[8] = {P.L, P.m, P.n_vleaf, P.n_uleaf, P.max_vnp, P.max_unp, P.max_vr, P.max_ur};
    F.w(hdr, sizeof(hdr));
    const int64_t sc[7] = {P.nx, P.nxi, P.nnz, P.w_elems, P.v_elems, P.u_elems, P.s_elems};
    F.w(sc, sizeof(sc));
    F.wv(P.rows);
    F.wv(P.ld);
    F.wv(P.nblk);
    F.wv(P.blk_first);
    F.wv(P.w_stage_off);
    F.wv(P.max_rank);
    F.wv(P.max_M);
    F.wv(P.max_K);
    int64_t nb = 0;
    for (auto v : P.nblk) nb += v;
    if (!dev_to_file(F, P.d_blk, nb * sizeof(BlockDesc)) ||
        !dev_to_file(F, P.d_vleaf, P.n_vleaf * sizeof(LeafDesc)) ||
        !dev_to_file(F, P.d_uleaf, P.n_uleaf * sizeof(LeafDesc)) || !dev_to_file(F, P.d_vidx, P.nxi * 4) ||
        !dev_to_file(F, P.d_uidx, P.nx * 4))
      return {MBF_ERR_IO, "write failed"};
    for (int p = 0; p < kNumPrec; ++p) {
      if (!(mask & (1u << p))) continue;
      const PrecData& d = P.prec[p];
      for (int s = 0; s < P.L; ++s)
        if (!dev_to_file(F, d.Wst[s], stage_elems(P, s) * elem(p))) return {MBF_ERR_IO, "write failed"};
      if (!dev_to_file(F, d.V0, P.v_elems * leaf_elem(p)) || !dev_to_file(F, d.UL, P.u_elems * leaf_elem(p)) ||
          !dev_to_file(F, d.S, P.s_elems * real_elem(p)))
        return {MBF_ERR_IO, "write failed"};
    }
  }
  if (D.n_center > 0) {
    if (!dev_to_file(F, D.d_center_idx, D.n_center * 4)) return {MBF_ERR_IO, "write failed"};
    for (int p = 0; p < kNumPrec; ++p)
      if (mask & (1u << p))
        if (!dev_to_file(F, D.center[p].center, (size_t)D.nx * D.n_center * leaf_elem(p)))
          return {MBF_ERR_IO, "write failed"};
  }
  const uint64_t payload = F.bytes;
  const uint64_t hash = F.digest();
  F.w(kEnd, 8);
  F.w(&payload, 8);
  F.w(&hash, 8);
  if (!F.ok || std::fflush(F.f) != 0) return {MBF_ERR_IO, "write failed"};
  return {MBF_OK, ""};
}

Error load_factor(const char* path, uint32_t want, DevFactor& D) {
  File F;
  F.f = std::fopen(path, "rb");
  if (!F.f) return {MBF_ERR_IO, std::string("cannot open ") + path};
  char magic[8];
  uint32_t ver = 0, mask = 0, np = 0;
  F.r(magic, 8);
  F.r(&ver, 4);
  if (!F.ok || std::memcmp(magic, kMagic, 8) != 0) return {MBF_ERR_IO, "not a factor file"};
  if (ver != kVersion) return {MBF_ERR_IO, "unsupported factor file version " + std::to_string(ver)};
  F.r(&mask, 4);
  F.r(&D.nx, 8);
  F.r(&D.nxi, 8);
  F.r(&D.n_center, 8);
  F.r(&np, 4);
  if (!F.ok || np == 0 || np > 64 || D.nx <= 0 || D.nxi <= 0 || D.nx > INT32_MAX || D.nxi > INT32_MAX ||
      D.n_center < 0 || D.n_center > D.nxi || (mask & ~((1u << kNumPrec) - 1)) != 0)
    return {MBF_ERR_IO, "corrupted factor header"};
  if (want == 0) want = mask;
  if ((want & mask) != want) return {MBF_ERR_UNSUPPORTED, "precision not stored in the file"};
  D.prec_mask = want;
  for (uint32_t i = 0; i < np; ++i) {
    D.parts.emplace_back();
    DevPart& P = D.parts.back();
    int32_t hdr[8];
    F.r(hdr, sizeof(hdr));
    P.L = hdr[0];
    P.m = hdr[1];
    P.n_vleaf = hdr[2];
    P.n_uleaf = hdr[3];
    P.max_vnp = hdr[4];
    P.max_unp = hdr[5];
    P.max_vr = hdr[6];
    P.max_ur = hdr[7];
    int64_t sc[7];
    F.r(sc, sizeof(sc));
    P.nx = sc[0];
    P.nxi = sc[1];
    P.nnz = sc[2];
    P.w_elems = sc[3];
    P.v_elems = sc[4];
    P.u_elems = sc[5];
    P.s_elems = sc[6];
    const int64_t cap_elems = (int64_t)1 << 40;
    if (!F.ok || P.L < 0 || P.L > 30 || P.n_vleaf < 0 || P.n_uleaf < 0 || P.nx != D.nx || P.nxi <= 0 ||
        P.nxi > D.nxi || P.w_elems < 0 || P.v_elems < 0 || P.u_elems < 0 || P.s_elems < 0 || P.nnz < 0 ||
        P.w_elems > cap_elems || P.v_elems > cap_elems || P.u_elems > cap_elems || P.s_elems > cap_elems)
      return {MBF_ERR_IO, "corrupted part header"};
    const uint64_t cap = (uint64_t)P.L + 1;
    F.rv(P.rows, cap);
    F.rv(P.ld, cap);
    F.rv(P.nblk, cap);
    F.rv(P.blk_first, cap);
    F.rv(P.w_stage_off, cap);
    F.rv(P.max_rank, cap);
    F.rv(P.max_M, cap);
    F.rv(P.max_K, cap);
    if (!F.ok || P.nblk.size() != (size_t)P.L) return {MBF_ERR_IO, "corrupted part"};
    int64_t nb = 0;
    for (auto v : P.nblk) {
      if (v < 0 || v > ((int64_t)1 << 31)) return {MBF_ERR_IO, "corrupted part"};
      nb += v;
    }
    std::vector<BlockDesc> blk;
    std::vector<LeafDesc> vl, ul;
    std::vector<int32_t> vidx, uidx;
    if (!file_to_host(F, blk, nb) || !file_to_host(F, vl, P.n_vleaf) || !file_to_host(F, ul, P.n_uleaf) ||
        !file_to_host(F, vidx, P.nxi) || !file_to_host(F, uidx, P.nx))
      return {MBF_ERR_IO, "truncated factor file"};
    std::string why;
    if (!check_part(P, D.nxi, blk, vl, ul, vidx, uidx, why)) return {MBF_ERR_IO, "corrupted factor file: " + why};
    size_t meta = 0;
    IO_TRY(host_to_dev((void**)&P.d_blk, blk, meta));
    IO_TRY(host_to_dev((void**)&P.d_vleaf, vl, meta));
    IO_TRY(host_to_dev((void**)&P.d_uleaf, ul, meta));
    IO_TRY(host_to_dev((void**)&P.d_vidx, vidx, meta));
    IO_TRY(host_to_dev((void**)&P.d_uidx, uidx, meta));
    for (int p = 0; p < kNumPrec; ++p) {
      if (!(mask & (1u << p))) continue;
      PrecData& d = P.prec[p];
      const size_t sizes[4] = {P.w_elems * elem(p), P.v_elems * leaf_elem(p), P.u_elems * leaf_elem(p),
                               P.s_elems * real_elem(p)};
      if (want & (1u << p)) {
        d.present = true;
        void* W = nullptr;
        IO_TRY(file_to_dev(F, &W, sizes[0], d.bytes));
        if (W) d.Walloc.push_back(W);
        d.Wst.assign(P.L, nullptr);
        for (int s = 0; s < P.L; ++s) d.Wst[s] = W ? (char*)W + (size_t)P.w_stage_off[s] * elem(p) : nullptr;
        IO_TRY(file_to_dev(F, &d.V0, sizes[1], d.bytes));
        IO_TRY(file_to_dev(F, &d.UL, sizes[2], d.bytes));
        IO_TRY(file_to_dev(F, &d.S, sizes[3], d.bytes));
        D.device_bytes += d.bytes;
      } else {
        // skipped precisions still enter the checksum
        std::vector<char> buf;
        for (size_t k = 0; k < 4; ++k) {
          for (size_t o = 0; o < sizes[k]; o += ((size_t)1 << 28)) {
            const size_t c = std::min(sizes[k] - o, (size_t)1 << 28);
            buf.resize(c);
            F.r(buf.data(), c);
            if (!F.ok) return {MBF_ERR_IO, "truncated factor file"};
          }
        }
      }
    }
    D.nnz += P.nnz;
  }
  if (D.n_center > 0) {
    std::vector<int32_t> cidx;
    if (!file_to_host(F, cidx, D.n_center)) return {MBF_ERR_IO, "truncated factor file"};
    for (int32_t v : cidx)
      if (v < 0 || v >= D.nxi) return {MBF_ERR_IO, "corrupted factor file: center index"};
    size_t meta = 0;
    IO_TRY(host_to_dev((void**)&D.d_center_idx, cidx, meta));
    for (int p = 0; p < kNumPrec; ++p) {
      if (!(mask & (1u << p))) continue;
      const size_t sz = (size_t)D.nx * D.n_center * leaf_elem(p);
      if (want & (1u << p)) {
        D.center[p].present = true;
        IO_TRY(file_to_dev(F, &D.center[p].center, sz, D.center[p].bytes));
        D.device_bytes += D.center[p].bytes;
      } else {
        std::vector<char> buf;
        for (size_t o = 0; o < sz; o += ((size_t)1 << 28)) {
          const size_t c = std::min(sz - o, (size_t)1 << 28);
          buf.resize(c);
          F.r(buf.data(), c);
          if (!F.ok) return {MBF_ERR_IO, "truncated factor file"};
        }
      }
    }
    D.nnz += D.nx * D.n_center;
  }
  const uint64_t payload = F.bytes;
  const uint64_t hash = F.digest();
  char end[8];
  uint64_t stored = 0, stored_hash = 0;
  F.r(end, 8);
  F.r(&stored, 8);
  F.r(&stored_hash, 8);
  if (!F.ok || std::memcmp(end, kEnd, 8) != 0 || stored != payload)
    return {MBF_ERR_IO, "corrupted or truncated factor file"};
  if (stored_hash != hash) return {MBF_ERR_IO, "factor file checksum mismatch"};
  return {MBF_OK, ""};
}

}  // namespace mbf
