// Versioned binary files of device-resident factorizations (mbf_save /
// mbf_load): builds take minutes at N = 512^2, so a factorization is kept
// on disk and reloaded to HBM instead of rebuilt.
//
// Layout (little endian):
//   "MBFFACT1" | u32 version | u32 prec_mask | i64 nx | i64 nxi | i64 n_center
//   | u32 nparts | parts... | center... | "MBFEND01" | u64 payload bytes
// Each part: scalars, per-stage vectors, block and leaf descriptors, point
// indices, then for every precision in the mask its W / V0 / UL / S arrays.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "device.h"

namespace mbf {
namespace {

constexpr uint32_t kVersion = 1;
const char kMagic[9] = "MBFFACT1";
const char kEnd[9] = "MBFEND01";

struct File {
  FILE* f = nullptr;
  uint64_t bytes = 0;
  bool ok = true;
  ~File() {
    if (f) std::fclose(f);
  }
  void w(const void* p, size_t n) {
    if (ok && n && std::fwrite(p, 1, n, f) != n) ok = false;
    bytes += n;
  }
  void r(void* p, size_t n) {
    if (ok && n && std::fread(p, 1, n, f) != n) ok = false;
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

size_t elem(int p) { return p == MBF_C128 ? 16 : 8; }
size_t leaf_elem(int p) { return p == MBF_C128 ? 16 : 8; }
size_t real_elem(int p) { return p == MBF_C128 ? 8 : 4; }

#define IO_TRY(expr)                \
  do {                              \
    Error _e = (expr);              \
    if (_e.st != MBF_OK) return _e; \
  } while (0)

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
      if (!dev_to_file(F, d.W, P.w_elems * elem(p)) || !dev_to_file(F, d.V0, P.v_elems * leaf_elem(p)) ||
          !dev_to_file(F, d.UL, P.u_elems * leaf_elem(p)) || !dev_to_file(F, d.S, P.s_elems * real_elem(p)))
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
  F.w(kEnd, 8);
  F.w(&payload, 8);
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
  if (!F.ok || np == 0 || np > 64 || D.nx <= 0 || D.nxi <= 0 || D.n_center < 0 || D.n_center > D.nxi)
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
    if (!F.ok || P.L < 0 || P.L > 30 || P.n_vleaf < 0 || P.n_uleaf < 0 || P.nx != D.nx || P.nxi <= 0 ||
        P.nxi > D.nxi || P.w_elems < 0 || P.v_elems < 0 || P.u_elems < 0 || P.s_elems < 0)
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
    if (!F.ok || P.rows.size() != cap || P.nblk.size() != (size_t)P.L) return {MBF_ERR_IO, "corrupted part"};
    int64_t nb = 0;
    for (auto v : P.nblk) nb += v;
    size_t meta = 0;
    IO_TRY(file_to_dev(F, (void**)&P.d_blk, nb * sizeof(BlockDesc), meta));
    IO_TRY(file_to_dev(F, (void**)&P.d_vleaf, P.n_vleaf * sizeof(LeafDesc), meta));
    IO_TRY(file_to_dev(F, (void**)&P.d_uleaf, P.n_uleaf * sizeof(LeafDesc), meta));
    IO_TRY(file_to_dev(F, (void**)&P.d_vidx, P.nxi * 4, meta));
    IO_TRY(file_to_dev(F, (void**)&P.d_uidx, P.nx * 4, meta));
    for (int p = 0; p < kNumPrec; ++p) {
      if (!(mask & (1u << p))) continue;
      PrecData& d = P.prec[p];
      const size_t sizes[4] = {P.w_elems * elem(p), P.v_elems * leaf_elem(p), P.u_elems * leaf_elem(p),
                               P.s_elems * real_elem(p)};
      if (want & (1u << p)) {
        d.present = true;
        IO_TRY(file_to_dev(F, &d.W, sizes[0], d.bytes));
        IO_TRY(file_to_dev(F, &d.V0, sizes[1], d.bytes));
        IO_TRY(file_to_dev(F, &d.UL, sizes[2], d.bytes));
        IO_TRY(file_to_dev(F, &d.S, sizes[3], d.bytes));
        D.device_bytes += d.bytes;
      } else {
        const size_t skip = sizes[0] + sizes[1] + sizes[2] + sizes[3];
        if (std::fseek(F.f, (long)skip, SEEK_CUR) != 0) return {MBF_ERR_IO, "truncated factor file"};
        F.bytes += skip;
      }
    }
    D.nnz += P.nnz;
  }
  if (D.n_center > 0) {
    size_t meta = 0;
    IO_TRY(file_to_dev(F, (void**)&D.d_center_idx, D.n_center * 4, meta));
    for (int p = 0; p < kNumPrec; ++p) {
      if (!(mask & (1u << p))) continue;
      const size_t sz = (size_t)D.nx * D.n_center * leaf_elem(p);
      if (want & (1u << p)) {
        D.center[p].present = true;
        IO_TRY(file_to_dev(F, &D.center[p].center, sz, D.center[p].bytes));
        D.device_bytes += D.center[p].bytes;
      } else {
        if (std::fseek(F.f, (long)sz, SEEK_CUR) != 0) return {MBF_ERR_IO, "truncated factor file"};
        F.bytes += sz;
      }
    }
    D.nnz += D.nx * D.n_center;
  }
  const uint64_t payload = F.bytes;
  char end[8];
  uint64_t stored = 0;
  F.r(end, 8);
  F.r(&stored, 8);
  if (!F.ok || std::memcmp(end, kEnd, 8) != 0 || stored != payload)
    return {MBF_ERR_IO, "corrupted or truncated factor file"};
  return {MBF_OK, ""};
}

}  // namespace mbf
