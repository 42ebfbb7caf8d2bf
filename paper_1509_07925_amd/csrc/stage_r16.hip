// Stage block products for up to 32 right-hand sides on the matrix cores
// (FP32, v_mfma_f32_16x16x4_f32).
//
// With few right-hand sides a stage streams its blocks from HBM; on the
// vector ALUs the 4 real FMAs of every complex multiply-add then cost about
// as much time as the bytes.  The 16 x 16 matrix-core tile fits 16
// right-hand sides exactly, so the arithmetic moves to the matrix cores and
// the kernel is left with the block stream.  A workgroup takes NTN tiles of
// 16 right-hand sides (NTN = 1 up to 16 RHS, 2 up to 32), so every chunk of
// the block is read from HBM once for all of them.
//
// Same real embedding as the wide kernels, Out^T = In^T W^T:
//   A(n, 2k+c)    = (Re, Im)_c x(n, k)                   16 RHS x 32 real k per chunk
//   B(2k+c, 2m+d) = [[Wr, Wi], [-Wi, Wr]]_{c,d}          forward (conj(W) for the adjoint)
// One instruction consumes 4 real k = 2 complex k: lane group g = lane / 16
// supplies complex k = 2 j + g / 2 (j-th instruction of a group of 8), part
// c = g % 2.  In LDS the complex index is stored even-first
// (word = (k & 1) * 8 + k / 2 within a chunk of 16), so the 4 instructions of
// a group read one 16-byte word per lane.
// Workgroup: 16 NTN RHS x 64 complex output rows, 4 waves of 16 NTN RHS x 32
// real columns (NTN x 2 tiles of 16 x 16).  Two-level sums as in the other
// FP32 kernels.
#include "stage_r16.h"

namespace mbf {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int RT = 16;   // right-hand sides per matrix-core tile
constexpr int RM = 64;   // complex output rows per workgroup
constexpr int RK = 16;   // complex reduction entries per chunk
constexpr int RP = 20;   // LDS row pitch (words)
constexpr int kXcdR = 8;  // XCDs per device

__device__ __forceinline__ int32_t r16_group_row(const BlockDesc& d, int32_t i) {
  int32_t base = d.orow[0] - d.ms[0];
  base = i >= d.ms[1] ? d.orow[1] - d.ms[1] : base;
  base = i >= d.ms[2] ? d.orow[2] - d.ms[2] : base;
  base = i >= d.ms[3] ? d.orow[3] - d.ms[3] : base;
  return base + i;
}

__device__ __forceinline__ int perm(int k) { return (k & 1) * (RK / 2) + (k >> 1); }

template <bool ADJ, int NTN>
__global__ __launch_bounds__(256) void k_stage_r16(const BlockDesc* __restrict__ blk, const float2* __restrict__ W,
                                                   const float2* __restrict__ in, int64_t ld_in,
                                                   float2* __restrict__ out, int64_t ld_out, int nrhs,
                                                   const float* __restrict__ scale, int mtiles, int64_t total) {
  constexpr int RN = RT * NTN;  // right-hand sides per workgroup
  __shared__ __attribute__((aligned(16))) float As[2][RN * RP];      // [c][n][perm(k)]
  __shared__ __attribute__((aligned(16))) float Bs[2][2 * RM * RP];  // [c][real col][perm(k)]
  // XCD-aware tile order: consecutive output tiles of a block on one XCD
  const int64_t per = (total + kXcdR - 1) / kXcdR;
  const int64_t t = (int64_t)(blockIdx.x % kXcdR) * per + blockIdx.x / kXcdR;
  if (t >= total) return;
  const int b = (int)(t / mtiles), mt = (int)(t % mtiles);
  const BlockDesc d = blk[b];
  const int R = ADJ ? d.K : d.M;
  const int Q = ADJ ? d.M : d.K;
  const int r0 = mt * RM;
  if (r0 >= R) return;
  if (Q <= 0) {  // empty reduction: the outputs are zero
    for (int e = threadIdx.x; e < RN * RM; e += 256) {
      const int n = blockIdx.y * RN + e / RM, m = r0 + e % RM;
      if (n < nrhs && m < R) out[(int64_t)n * ld_out + (ADJ ? d.in_row + m : r16_group_row(d, m))] = make_float2(0.f, 0.f);
    }
    return;
  }
  const int n0 = blockIdx.y * RN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const float2* Wb = W + d.w_off;
  // loads: state entries (n = tid / 16 + 16 j, k = tid % 16); block: 4 consecutive
  // reduction entries of one output row (forward: row tid % 64, group
  // tid / 64, lanes along rows; adjoint: row tid / 4, group tid % 4, lanes
  // along the contiguous reduction index)
  const int ak = tid % RK, an = tid / RK;
  const int bm = ADJ ? tid / 4 : tid % RM, bg = ADJ ? tid % 4 : tid / RM;
  struct Regs {
    float2 x[NTN];
    float2 w[4];
    uint32_t ok;  // bit j: x[j] in range; bit NTN + i: w[i] in range
  };
  // Branch-free loads: addresses clamped into the block (a chunk past the
  // end reads valid, recently read entries); the zeros outside the block are
  // selected in stash.  A guarded load, or a select right after the load,
  // would make the compiler wait for it on the spot and the prefetch would
  // not overlap the matrix-core work.
  auto load = [&](Regs& g, int q0) {
    const int q = q0 + ak, qc = min(q, Q - 1);
    const int64_t xr = ADJ ? r16_group_row(d, qc) : d.in_row + qc;
    g.ok = 0;
#pragma unroll
    for (int j = 0; j < NTN; ++j) {
      const int n = n0 + an + RT * j;
      g.x[j] = in[(int64_t)min(n, nrhs - 1) * ld_in + xr];
      g.ok |= (uint32_t)(q < Q && n < nrhs) << j;
    }
    const int m = r0 + bm, mc = min(m, R - 1);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int qq = q0 + 4 * bg + i, qqc = min(qq, Q - 1);
      g.w[i] = ADJ ? Wb[(int64_t)mc * d.M + qqc] : Wb[(int64_t)qqc * d.M + mc];
      g.ok |= (uint32_t)(m < R && qq < Q) << (NTN + i);
    }
  };
  auto stash = [&](const Regs& r) {
    Regs g = r;
    const float2 z = make_float2(0.f, 0.f);
#pragma unroll
    for (int j = 0; j < NTN; ++j)
      if (!((g.ok >> j) & 1)) g.x[j] = z;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (!((g.ok >> (NTN + i)) & 1)) g.w[i] = z;
#pragma unroll
    for (int j = 0; j < NTN; ++j) {
      As[0][(an + RT * j) * RP + perm(ak)] = g.x[j].x;
      As[1][(an + RT * j) * RP + perm(ak)] = g.x[j].y;
    }
    const float s = ADJ ? -1.f : 1.f;
    const int c0 = 2 * bm;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int w = perm(4 * bg + i);
      const float wr = g.w[i].x, wi = s * g.w[i].y;
      Bs[0][c0 * RP + w] = wr;         // B(2k, 2m)     = Wr
      Bs[0][(c0 + 1) * RP + w] = wi;   // B(2k, 2m+1)   = Wi
      Bs[1][c0 * RP + w] = -wi;        // B(2k+1, 2m)   = -Wi
      Bs[1][(c0 + 1) * RP + w] = wr;   // B(2k+1, 2m+1) = Wr
    }
  };
  const int g = lane >> 4, li = lane & 15;
  const int c = g & 1, half = g >> 1;
  const int wm = wave * 32;  // real columns of this wave
  v4f acc[NTN][2];
#pragma unroll
  for (int j = 0; j < NTN; ++j) acc[j][0] = acc[j][1] = v4f{};
  // two chunks ahead in registers: cur (next to stash) and ahead
  Regs cur, ahead;
  load(cur, 0);
  load(ahead, RK);
  for (int q0 = 0; q0 < Q; q0 += RK) {
    stash(cur);
    __syncthreads();
    cur = ahead;
    load(ahead, q0 + 2 * RK);
    v4f p[NTN][2];
#pragma unroll
    for (int j = 0; j < NTN; ++j) p[j][0] = p[j][1] = v4f{};
#pragma unroll
    for (int kb = 0; kb < RK; kb += 8) {
      const int w0 = half * (RK / 2) + kb / 2;
      float4 av[NTN], bv[2];
#pragma unroll
      for (int j = 0; j < NTN; ++j) av[j] = *reinterpret_cast<const float4*>(&As[c][(RT * j + li) * RP + w0]);
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) bv[ct] = *reinterpret_cast<const float4*>(&Bs[c][(wm + 16 * ct + li) * RP + w0]);
      // consecutive instructions go to different accumulator tiles
#pragma unroll
      for (int j = 0; j < NTN; ++j)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) p[j][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[j].x, bv[ct].x, p[j][ct], 0, 0, 0);
#pragma unroll
      for (int j = 0; j < NTN; ++j)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) p[j][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[j].y, bv[ct].y, p[j][ct], 0, 0, 0);
#pragma unroll
      for (int j = 0; j < NTN; ++j)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) p[j][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[j].z, bv[ct].z, p[j][ct], 0, 0, 0);
#pragma unroll
      for (int j = 0; j < NTN; ++j)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) p[j][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[j].w, bv[ct].w, p[j][ct], 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < NTN; ++j) {
      acc[j][0] += p[j][0];
      acc[j][1] += p[j][1];
    }
    __syncthreads();
  }
  // lane holds D[4 g + i][li] of each tile: RHS 16 j + 4 g + i, real column wm + 16 ct + li
  float* o = reinterpret_cast<float*>(out);
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int col = wm + 16 * ct + li;
    const int m = r0 + (col >> 1);
    if (m >= R) continue;
    const int32_t row = ADJ ? d.in_row + m : r16_group_row(d, m);
    const float sc = scale ? scale[row] : 1.0f;
#pragma unroll
    for (int j = 0; j < NTN; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int n = n0 + RT * j + 4 * g + i;
        if (n < nrhs) o[2 * ((int64_t)n * ld_out + row) + (col & 1)] = acc[j][ct][i] * sc;
      }
  }
}

}  // namespace

Error launch_stage_r16(const DevPart& P, int s, bool adj, const BlockDesc* blk, const void* W, const void* in,
                       int64_t ld_in, void* out, int64_t ld_out, int nrhs, const float* scale, hipStream_t st) {
  if (nrhs < 1) return {MBF_ERR_INVALID_ARG, "r16 stage: nrhs < 1"};
  const int Rmax = adj ? P.max_K[s] : P.max_M[s];
  const int mtiles = std::max(1, (Rmax + RM - 1) / RM);
  const int64_t total = (int64_t)P.nblk[s] * mtiles;
  const int64_t gx = (total + kXcdR - 1) / kXcdR * kXcdR;
  const int ntn = nrhs <= RT ? 1 : 2;
  const int64_t gy = (nrhs + RT * ntn - 1) / (RT * ntn);
  if (gx > INT32_MAX || gy > 65535) return {MBF_ERR_UNSUPPORTED, "r16 stage grid too large"};
  const dim3 grid((unsigned)gx, (unsigned)gy);
  const float2* x = reinterpret_cast<const float2*>(in);
  float2* y = reinterpret_cast<float2*>(out);
  const float2* w = reinterpret_cast<const float2*>(W);
  if (adj && ntn == 1)
    hipLaunchKernelGGL((k_stage_r16<true, 1>), grid, dim3(256), 0, st, blk, w, x, ld_in, y, ld_out, nrhs, scale,
                       mtiles, total);
  else if (adj)
    hipLaunchKernelGGL((k_stage_r16<true, 2>), grid, dim3(256), 0, st, blk, w, x, ld_in, y, ld_out, nrhs, scale,
                       mtiles, total);
  else if (ntn == 1)
    hipLaunchKernelGGL((k_stage_r16<false, 1>), grid, dim3(256), 0, st, blk, w, x, ld_in, y, ld_out, nrhs, scale,
                       mtiles, total);
  else
    hipLaunchKernelGGL((k_stage_r16<false, 2>), grid, dim3(256), 0, st, blk, w, x, ld_in, y, ld_out, nrhs, scale,
                       mtiles, total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return {MBF_ERR_HIP, std::string("r16 stage launch: ") + hipGetErrorString(e)};
  return {MBF_OK, ""};
}

}  // namespace mbf
