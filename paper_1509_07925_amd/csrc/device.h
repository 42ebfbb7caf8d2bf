// Device-resident factorization and apply launchers (see kernels.hip).
//
// Layout in HBM.  The state of stage s (one vector per pair, Section 2.5) is
// a column-major complex matrix of rows_s x nrhs with leading dimension
// ld_s: the rows of pair p are [row_off(p), row_off(p) + rank(p)), pairs in
// A-major / B-minor order.  With this order the four inputs of a stage
// block, (A, child_sigma B'), are one contiguous row range, and its four
// outputs, (child_tau A, B'), are four row ranges of stage s+1: the
// quadtree permutation between levels is folded into the block's output
// addressing.  Stage blocks are stored column-major (M x K), one after the
// other in block order.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>

#include <cstdint>
#include <vector>

#include "factor.h"

namespace mbf {

struct BlockDesc {
  int64_t w_off;   // element offset of the block's M x K matrix from the start of its stage
  int32_t M, K;    // output rows / input rows (forward direction)
  int32_t in_row;  // first stage-s row of the contiguous input side
  int32_t ms[4];   // start of output group t inside [0, M); unused groups = M
  int32_t orow[4]; // first stage-(s+1) row of output group t
  int32_t pad;
};
static_assert(sizeof(BlockDesc) == 56, "BlockDesc layout");

struct LeafDesc {
  int64_t f_off;  // element offset of the |leaf| x r factor (column-major)
  int32_t p_off;  // offset into the point-index array
  int32_t np;     // points in the leaf
  int32_t r;      // rank
  int32_t row;    // first state row of the leaf's pair
};
static_assert(sizeof(LeafDesc) == 24, "LeafDesc layout");

constexpr int kNumPrec = 3;

struct PrecData {
  bool present = false;
  // Stage blocks (element type depends on precision): Wst[s] is the start of
  // stage s; block descriptors address their matrix relative to it.  The
  // stages live in the allocations listed in Walloc (one for all stages, or
  // one per stage when a builder writes stages as they complete).
  std::vector<void*> Wst;
  std::vector<void*> Walloc;
  void* V0 = nullptr;     // Omega-leaf factors
  void* UL = nullptr;     // X-leaf factors
  void* S = nullptr;      // middle scaling, real, state-h rows
  void* center = nullptr; // dense center (multiscale)
  size_t bytes = 0;
};

struct DevPart {
  int L = 0, m = 0;
  int64_t nx = 0, nxi = 0;
  std::vector<int64_t> rows, ld;         // per stage 0..L
  std::vector<int64_t> nblk;             // per stage 0..L-1
  std::vector<int64_t> blk_first;        // per stage: first descriptor index
  std::vector<int64_t> w_stage_off;      // per stage: element offset into W
  std::vector<int32_t> max_rank;         // per stage
  std::vector<int32_t> max_M, max_K;     // per stage 0..L-1
  int64_t nnz = 0, w_elems = 0, v_elems = 0, u_elems = 0, s_elems = 0;
  BlockDesc* d_blk = nullptr;
  LeafDesc* d_vleaf = nullptr;
  LeafDesc* d_uleaf = nullptr;
  int32_t n_vleaf = 0, n_uleaf = 0;
  int32_t max_vnp = 0, max_unp = 0, max_vr = 0, max_ur = 0;
  int32_t* d_vidx = nullptr;  // Omega point indices (caller's order), tree order
  int32_t* d_uidx = nullptr;  // X point indices, tree order
  PrecData prec[kNumPrec];
};

struct Profiler {
  bool on = false;
  int32_t cap = 0, used = 0;
  std::vector<hipEvent_t> ev;
  std::vector<mbf_launch_record> rec;
};

struct DevFactor {
  int64_t nx = 0, nxi = 0;
  uint32_t prec_mask = 0;
  std::vector<DevPart> parts;
  // multiscale center: u += K_C g[center_idx]
  int64_t n_center = 0;
  int32_t* d_center_idx = nullptr;
  PrecData center[kNumPrec];
  int64_t nnz = 0;
  size_t device_bytes = 0;
  mutable Profiler prof;
};

// Layout of a part from its trees and ranks alone (Section 2.5 bookkeeping):
// state rows, stage block and leaf descriptors, and the point-index arrays,
// uploaded to the device; no factor data.  blk_off (optional) receives the
// offset of every block inside its stage, in block order.
Error layout_part(const Tree& xt, const Tree& ot, int L, int m, const std::vector<std::vector<int32_t>>& rank,
                  const int64_t* idx_map, DevPart& P, std::vector<int64_t>* blk_off);
// Upload a host factorization as one part.  idx_map (optional, nxi
// entries) maps the part's Omega column order to the caller's order.
Error upload_part(const HostFactor& f, const int64_t* idx_map, uint32_t prec_mask, DevPart& out);
Error upload_center(DevFactor& F, const std::vector<cd>& KC, const std::vector<int64_t>& idx,
                    uint32_t prec_mask);
void free_factor(DevFactor& F);

Error save_factor(const DevFactor& F, uint32_t prec_mask, const char* path);
Error load_factor(const char* path, uint32_t prec_mask, DevFactor& F);

size_t workspace_bytes(const DevFactor& F, int prec, int64_t nrhs);
Error autotune_factor(const DevFactor& F, int prec, int64_t nrhs, void* ws, size_t ws_bytes, hipStream_t st,
                      int* ntuned);
Error launch_apply(const DevFactor& F, int prec, bool adjoint, int64_t nrhs, const void* in,
                   int64_t ldin, void* out, int64_t ldout, void* ws, size_t ws_bytes,
                   hipStream_t stream);
// u = K g with the workspace in the library's fixed device scratch (no
// allocation); fails when the apply needs more than scratch_bytes().
Error launch_apply_scratch(const DevFactor& F, int prec, int64_t nrhs, const void* in, int64_t ldin, void* out,
                           int64_t ldout, hipStream_t stream);
size_t scratch_bytes();
// Destroy the side streams that multiscale applies created for the caller
// stream `caller` on the current device (after they drain); a caller that
// destroys its stream calls this first.
void release_side_streams(hipStream_t caller);

}  // namespace mbf

namespace mbf {
// Process-wide serial numbers of factor handles (never reused, unlike
// addresses): the server keys its captured graphs by them.
inline std::atomic<uint64_t> g_factor_serial{1};
}  // namespace mbf

// The opaque handle of the C ABI.
struct mbf_factor_s {
  mbf::DevFactor dev;
  uint64_t serial = mbf::g_factor_serial.fetch_add(1);
};
