// Stage block products for few right-hand sides (FP32, nrhs <= 32).
//
// With few right-hand sides a stage is bound by reading its blocks from HBM
// once (8 bytes per complex entry against 8 nrhs flops), so the kernel is
// organised around streaming W: one thread per output row of a block, 256
// rows per workgroup, the reduction in chunks of 32 entries.
//   forward  out(n, m) = sum_k W(m, k) x(n, k): thread m reads W(m, k) for
//            the chunk's k straight from HBM; for each k the 256 threads of a
//            workgroup read 256 consecutive entries of a column of W.
//   adjoint  out(n, k) = sum_m conj(W(m, k)) x(n, m): the 256 x 32 tile of W
//            (256 output columns k, 32 reduction rows m) is loaded along m
//            (contiguous) and transposed through LDS.
// The chunk of the input state (32 x NR) sits in LDS and every lane reads the
// same entry (broadcast).  Sums are two-level, as in the matrix-core kernels:
// a partial sum per chunk, added to the running sum.
#include "stage_narrow.h"

namespace mbf {

namespace {

constexpr int NT = 256;  // threads = output rows per workgroup
constexpr int KCN = 32;  // reduction chunk

__device__ __forceinline__ int32_t out_group_row(const BlockDesc& d, int32_t i) {
  int32_t base = d.orow[0] - d.ms[0];
  base = i >= d.ms[1] ? d.orow[1] - d.ms[1] : base;
  base = i >= d.ms[2] ? d.orow[2] - d.ms[2] : base;
  base = i >= d.ms[3] ? d.orow[3] - d.ms[3] : base;
  return base + i;
}

template <bool ADJ, int NR>
__global__ __launch_bounds__(NT) void k_stage_narrow(const BlockDesc* __restrict__ blk,
                                                     const float2* __restrict__ W,
                                                     const float2* __restrict__ in, int64_t ld_in,
                                                     float2* __restrict__ out, int64_t ld_out, int nrhs,
                                                     const float* __restrict__ scale, int mtiles) {
  __shared__ float2 Xs[KCN][NR];
  __shared__ float2 Ws[ADJ ? NT : 1][KCN + 1];
  const int b = blockIdx.x / mtiles, mt = blockIdx.x % mtiles;
  const BlockDesc d = blk[b];
  const int R = ADJ ? d.K : d.M;
  const int Q = ADJ ? d.M : d.K;
  const int r0 = mt * NT;
  if (r0 >= R) return;
  const int n0 = blockIdx.y * NR;
  const int tid = threadIdx.x;
  const int r = r0 + tid;
  const float2* Wb = W + d.w_off;
  float2 acc[NR];
#pragma unroll
  for (int n = 0; n < NR; ++n) acc[n] = make_float2(0.f, 0.f);
  for (int q0 = 0; q0 < Q; q0 += KCN) {
    float2 w[ADJ ? 1 : KCN];
    if (!ADJ) {  // issue the chunk's W loads first; they land while x is staged
#pragma unroll
      for (int k = 0; k < KCN; ++k) {
        float2 v = make_float2(0.f, 0.f);
        if (r < R && q0 + k < Q) v = Wb[(int64_t)(q0 + k) * d.M + r];
        w[k] = v;
      }
    } else {  // two rounds of 16 loads in flight before their LDS stores
      const int mm = tid % KCN;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        float2 t[KCN / 2];
#pragma unroll
        for (int j = 0; j < KCN / 2; ++j) {
          const int ko = tid / KCN + (h * (KCN / 2) + j) * (NT / KCN);
          float2 v = make_float2(0.f, 0.f);
          if (r0 + ko < R && q0 + mm < Q) v = Wb[(int64_t)(r0 + ko) * d.M + q0 + mm];
          t[j] = v;
        }
#pragma unroll
        for (int j = 0; j < KCN / 2; ++j) Ws[tid / KCN + (h * (KCN / 2) + j) * (NT / KCN)][mm] = t[j];
      }
    }
    for (int e = tid; e < KCN * NR; e += NT) {  // lanes along k: consecutive state rows
      const int k = e % KCN, n = e / KCN;
      const int q = q0 + k, gn = n0 + n;
      float2 v = make_float2(0.f, 0.f);
      if (q < Q && gn < nrhs) v = in[(int64_t)gn * ld_in + (ADJ ? out_group_row(d, q) : d.in_row + q)];
      Xs[k][n] = v;
    }
    __syncthreads();
    float2 p[NR];
#pragma unroll
    for (int n = 0; n < NR; ++n) p[n] = make_float2(0.f, 0.f);
#pragma unroll
    for (int k = 0; k < KCN; ++k) {
      const float2 wk = ADJ ? Ws[tid][k] : w[k];
      const float wr = wk.x, wi = ADJ ? -wk.y : wk.y;
#pragma unroll
      for (int n = 0; n < NR; ++n) {
        const float2 xv = Xs[k][n];
        p[n].x += wr * xv.x - wi * xv.y;
        p[n].y += wr * xv.y + wi * xv.x;
      }
    }
#pragma unroll
    for (int n = 0; n < NR; ++n) {
      acc[n].x += p[n].x;
      acc[n].y += p[n].y;
    }
    __syncthreads();
  }
  if (r < R) {
    const int32_t row = ADJ ? d.in_row + r : out_group_row(d, r);
    const float s = scale ? scale[row] : 1.0f;
#pragma unroll
    for (int n = 0; n < NR; ++n)
      if (n0 + n < nrhs) out[(int64_t)(n0 + n) * ld_out + row] = make_float2(acc[n].x * s, acc[n].y * s);
  }
}

template <bool ADJ>
void launch(int nr, dim3 grid, hipStream_t st, const BlockDesc* blk, const float2* W, const float2* x,
            int64_t ld_in, float2* y, int64_t ld_out, int nrhs, const float* scale, int mtiles) {
  if (nr == 8)
    hipLaunchKernelGGL((k_stage_narrow<ADJ, 8>), grid, dim3(NT), 0, st, blk, W, x, ld_in, y, ld_out, nrhs, scale,
                       mtiles);
  else if (nr == 16)
    hipLaunchKernelGGL((k_stage_narrow<ADJ, 16>), grid, dim3(NT), 0, st, blk, W, x, ld_in, y, ld_out, nrhs, scale,
                       mtiles);
  else
    hipLaunchKernelGGL((k_stage_narrow<ADJ, 32>), grid, dim3(NT), 0, st, blk, W, x, ld_in, y, ld_out, nrhs, scale,
                       mtiles);
}

}  // namespace

Error launch_stage_narrow(const DevPart& P, int s, bool adj, const BlockDesc* blk, const void* W, const void* in,
                          int64_t ld_in, void* out, int64_t ld_out, int nrhs, const float* scale, hipStream_t st) {
  if (nrhs < 1) return {MBF_ERR_INVALID_ARG, "narrow stage: nrhs < 1"};
  const int Rmax = adj ? P.max_K[s] : P.max_M[s];
  const int mtiles = std::max(1, (Rmax + NT - 1) / NT);
  const int nr = nrhs <= 8 ? 8 : nrhs <= 16 ? 16 : 32;
  const int64_t gx = (int64_t)P.nblk[s] * mtiles;
  const int64_t gy = (nrhs + nr - 1) / nr;
  if (gx > INT32_MAX || gy > 65535) return {MBF_ERR_UNSUPPORTED, "narrow stage grid too large"};
  const dim3 grid((unsigned)gx, (unsigned)gy);
  const float2* x = reinterpret_cast<const float2*>(in);
  float2* y = reinterpret_cast<float2*>(out);
  const float2* w = reinterpret_cast<const float2*>(W);
  if (adj)
    launch<true>(nr, grid, st, blk, w, x, ld_in, y, ld_out, nrhs, scale, mtiles);
  else
    launch<false>(nr, grid, st, blk, w, x, ld_in, y, ld_out, nrhs, scale, mtiles);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return {MBF_ERR_HIP, std::string("narrow stage launch: ") + hipGetErrorString(e)};
  return {MBF_OK, ""};
}

}  // namespace mbf
