// Stage block products for up to 16 right-hand sides on the matrix cores
// (FP32, v_mfma_f32_16x16x4_f32).
//
// With few right-hand sides a stage streams its blocks from HBM; on the
// vector ALUs the 4 real FMAs of every complex multiply-add then cost about
// as much time as the bytes.  The 16 x 16 matrix-core tile fits 16
// right-hand sides exactly, so the arithmetic moves to the matrix cores and
// the kernel is left with the block stream.
//
// Same real embedding as the wide kernels, Out^T = In^T W^T:
//   A(n, 2k+c)    = (Re, Im)_c x(n, k)                   16 RHS x 32 real k per chunk
//   B(2k+c, 2m+d) = [[Wr, Wi], [-Wi, Wr]]_{c,d}          forward (conj(W) for the adjoint)
// One instruction consumes 4 real k = 2 complex k: lane group g = lane / 16
// supplies complex k = 2 j + g / 2 (j-th instruction of a group of 8), part
// c = g % 2.  In LDS the complex index is stored even-first
// (word = (k & 1) * 8 + k / 2 within a chunk of 16), so the 4 instructions of
// a group read one 16-byte word per lane.
// Workgroup: 16 RHS x 64 complex output rows, 4 waves of 16 RHS x 32 real
// columns (2 tiles of 16 x 16).  Two-level sums as in the other FP32 kernels.
#include "stage_r16.h"

namespace mbf {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int RN = 16;   // right-hand sides per workgroup
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

template <bool ADJ>
__global__ __launch_bounds__(256) void k_stage_r16(const BlockDesc* __restrict__ blk, const float2* __restrict__ W,
                                                   const float2* __restrict__ in, int64_t ld_in,
                                                   float2* __restrict__ out, int64_t ld_out, int nrhs,
                                                   const float* __restrict__ scale, int mtiles, int64_t total) {
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
  const int n0 = blockIdx.y * RN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const float2* Wb = W + d.w_off;
  // loads: state entry (n = tid / 16, k = tid % 16); block: 4 consecutive
  // reduction entries of one output row (forward: row tid % 64, group
  // tid / 64, lanes along rows; adjoint: row tid / 4, group tid % 4, lanes
  // along the contiguous reduction index)
  const int ak = tid % RK, an = tid / RK;
  const int bm = ADJ ? tid / 4 : tid % RM, bg = ADJ ? tid % 4 : tid / RM;
  struct Regs {
    float2 x;
    float2 w[4];
  };
  auto load = [&](Regs& g, int q0) {
    const int q = q0 + ak;
    g.x = make_float2(0.f, 0.f);
    if (q < Q && n0 + an < nrhs)
      g.x = in[(int64_t)(n0 + an) * ld_in + (ADJ ? r16_group_row(d, q) : d.in_row + q)];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int qq = q0 + 4 * bg + i, m = r0 + bm;
      float2 w = make_float2(0.f, 0.f);
      if (m < R && qq < Q) w = ADJ ? Wb[(int64_t)m * d.M + qq] : Wb[(int64_t)qq * d.M + m];
      g.w[i] = w;
    }
  };
  auto stash = [&](const Regs& g) {
    As[0][an * RP + perm(ak)] = g.x.x;
    As[1][an * RP + perm(ak)] = g.x.y;
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
  v4f acc[2] = {v4f{}, v4f{}};
  // two chunks ahead in registers: cur (next to stash) and ahead
  Regs cur, ahead;
  load(cur, 0);
  if (RK < Q) load(ahead, RK);
  for (int q0 = 0; q0 < Q; q0 += RK) {
    stash(cur);
    __syncthreads();
    if (q0 + RK < Q) {
      cur = ahead;
      if (q0 + 2 * RK < Q) load(ahead, q0 + 2 * RK);
    }
    v4f p[2] = {v4f{}, v4f{}};
#pragma unroll
    for (int kb = 0; kb < RK; kb += 8) {
      const int w0 = half * (RK / 2) + kb / 2;
      const float4 av = *reinterpret_cast<const float4*>(&As[c][li * RP + w0]);
      float4 bv[2];
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) bv[ct] = *reinterpret_cast<const float4*>(&Bs[c][(wm + 16 * ct + li) * RP + w0]);
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) p[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv[ct].x, p[ct], 0, 0, 0);
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) p[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv[ct].y, p[ct], 0, 0, 0);
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) p[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, bv[ct].z, p[ct], 0, 0, 0);
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) p[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, bv[ct].w, p[ct], 0, 0, 0);
    }
    acc[0] += p[0];
    acc[1] += p[1];
    __syncthreads();
  }
  // lane holds D[4 g + i][li] of each tile: RHS 4 g + i, real column wm + 16 ct + li
  float* o = reinterpret_cast<float*>(out);
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int col = wm + 16 * ct + li;
    const int m = r0 + (col >> 1);
    if (m >= R) continue;
    const int32_t row = ADJ ? d.in_row + m : r16_group_row(d, m);
    const float sc = scale ? scale[row] : 1.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int n = n0 + 4 * g + i;
      if (n < nrhs) o[2 * ((int64_t)n * ld_out + row) + (col & 1)] = acc[ct][i] * sc;
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
  const int64_t gy = (nrhs + RN - 1) / RN;
  if (gx > INT32_MAX || gy > 65535) return {MBF_ERR_UNSUPPORTED, "r16 stage grid too large"};
  const dim3 grid((unsigned)gx, (unsigned)gy);
  const float2* x = reinterpret_cast<const float2*>(in);
  float2* y = reinterpret_cast<float2*>(out);
  const float2* w = reinterpret_cast<const float2*>(W);
  if (adj)
    hipLaunchKernelGGL(k_stage_r16<true>, grid, dim3(256), 0, st, blk, w, x, ld_in, y, ld_out, nrhs, scale, mtiles,
                       total);
  else
    hipLaunchKernelGGL(k_stage_r16<false>, grid, dim3(256), 0, st, blk, w, x, ld_in, y, ld_out, nrhs, scale, mtiles,
                       total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return {MBF_ERR_HIP, std::string("r16 stage launch: ") + hipGetErrorString(e)};
  return {MBF_OK, ""};
}

}  // namespace mbf
