// Matrix-core (MFMA) stage kernels for many right-hand sides; see stage_mfma.h.
//
// A stage block computes, for the nrhs columns of the state,
//   forward: out(n, m) = sum_k W(m, k) x(n, k)        (M x K block)
//   adjoint: out(n, k) = sum_m conj(W(m, k)) x(n, m)
// i.e. Out^T = In^T W^T: the right-hand sides run along the MFMA rows, the
// block's output rows along the MFMA columns, and the complex product is
// the real product of the embeddings
//   A(n, 2k+c)      = (Re, Im)_c x(n, k)
//   B(2k+c, 2m+d)   = [[Wr, Wi], [-Wi, Wr]]_{c,d}   (forward)
//                     [[Wr, -Wi], [Wi, Wr]]_{c,d}   (adjoint, conj(W))
// so that D(n, 2m+d) is the real (d=0) / imaginary (d=1) part of out(n, m):
// output rows are interleaved complex and store coalesced into the state.
//
// Tile: 64 or 128 right-hand sides x 64 complex output rows per workgroup
// (4 waves, each 32 or 64 right-hand sides x 64 real columns), reduction
// staged through LDS in chunks of 16 or 32 complex entries; the chunk sums
// are added to the running sums (two-level summation).  Two arithmetic modes:
//   F32    v_mfma_f32_32x32x2_f32, one complex k per instruction;
//   BF16X3 v_mfma_f32_32x32x16_bf16, eight complex k per instruction; every
//          operand is split as hi + lo (both BF16) and the product is
//          hi*hi + hi*lo + lo*hi with FP32 accumulation.
// Workgroup -> tile mapping is XCD-aware: consecutive logical tiles (the
// right-hand-side tiles of one output tile, then the output tiles of one
// block) land on the same XCD so that they share its L2.
#include "stage_mfma.h"

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

namespace mbf {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int TN = 64;   // right-hand sides per tile
constexpr int TM = 64;   // complex output rows per tile
constexpr int kXcd = 8;  // XCDs per device

// Selects instead of an indexed load keep the descriptor in registers (a
// run-time index into its arrays would place it in private memory).
__device__ __forceinline__ int32_t grp_row(const BlockDesc& d, int32_t i) {
  int32_t base = d.orow[0] - d.ms[0];
  base = i >= d.ms[1] ? d.orow[1] - d.ms[1] : base;
  base = i >= d.ms[2] ? d.orow[2] - d.ms[2] : base;
  base = i >= d.ms[3] ? d.orow[3] - d.ms[3] : base;
  return base + i;
}

__device__ __forceinline__ uint32_t f2bf_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float bf_bits2f(uint32_t h) { return __uint_as_float(h << 16); }
// (hi, lo) BF16 split of an FP32 value.
__device__ __forceinline__ void split_bf(float x, uint32_t& hi, uint32_t& lo) {
  hi = f2bf_bits(x);
  lo = f2bf_bits(x - bf_bits2f(hi));
}

struct Tile {
  int b, mt, nt;
};

// Logical tile of this workgroup, or b = -1 when it has none.
__device__ __forceinline__ Tile map_tile(int64_t total, int mtiles, int ntiles) {
  const int64_t per = (total + kXcd - 1) / kXcd;
  const int64_t L = blockIdx.x;
  const int64_t t = (L % kXcd) * per + L / kXcd;
  Tile r{-1, 0, 0};
  if (t >= total) return r;
  r.nt = (int)(t % ntiles);
  const int64_t rest = t / ntiles;
  r.mt = (int)(rest % mtiles);
  r.b = (int)(rest / mtiles);
  return r;
}

// Store the wave's NS x 2 accumulator tiles (32 x 32 real each): rows are
// right-hand sides wn + 32 ns + (MFMA row), columns real output columns
// wm + 32 cs + (lane % 32); lanes of a row write consecutive floats.
template <bool ADJ, int NS>
__device__ __forceinline__ void store_out(const BlockDesc& d, int R, int r0, int n0, const v16f (&acc)[NS][2],
                                          int wn, int wm, float2* __restrict__ out, int64_t ld_out, int nrhs,
                                          const float* __restrict__ scale) {
  const int lane = threadIdx.x & 63;
  float* o = reinterpret_cast<float*>(out);
#pragma unroll
  for (int cs = 0; cs < 2; ++cs) {
    const int col = wm + cs * 32 + (lane & 31);  // real output column
    const int m = r0 + (col >> 1);
    if (m >= R) continue;
    const int32_t row = ADJ ? d.in_row + m : grp_row(d, m);
    const float sc = scale ? scale[row] : 1.0f;
#pragma unroll
    for (int ns = 0; ns < NS; ++ns)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int n = n0 + wn + 32 * ns + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
        if (n < nrhs) o[2 * ((int64_t)n * ld_out + row) + (col & 1)] = acc[ns][cs][j] * sc;
      }
  }
}

// ------------------------------------------------------------------ loads
// Each chunk moves a TNV x KC tile of the input state (A) and a KC x TM tile
// of the block (B) into LDS, with consecutive lanes on consecutive memory
// (the reduction index for A and for the adjoint's B, the output index for
// the forward B).  With PF the registers for the next chunk are loaded while
// the matrix cores work on the current one.
template <int TNV, int KC, bool ADJ, typename WT>
struct Loader {
  static constexpr int EA = TNV * KC / 256;
  static constexpr int EB = TM * KC / 256;
  float2 a[EA];
  WT b[EB];
  __device__ __forceinline__ void load(const BlockDesc& d, const float2* __restrict__ in, int64_t ld_in,
                                       const WT* __restrict__ Wb, int R, int Q, int r0, int n0, int q0,
                                       int nrhs) {
    const int tid = threadIdx.x;
    {  // A(n, k): k = tid % KC, rows tid / KC + j * (256 / KC)
      const int k = tid % KC, n = tid / KC;
      const int q = q0 + k;
      int32_t row = 0;
      if (q < Q) row = ADJ ? grp_row(d, q) : d.in_row + q;
#pragma unroll
      for (int j = 0; j < EA; ++j) {
        const int gn = n0 + n + j * (256 / KC);
        float2 v = make_float2(0.f, 0.f);
        if (gn < nrhs && q < Q) v = in[(int64_t)gn * ld_in + row];
        a[j] = v;
      }
    }
    if (!ADJ) {  // W(m, k), m contiguous: m = tid % 64, k = tid / 64 + 4 j
      const int m = r0 + (tid & 63), kb = tid >> 6;
#pragma unroll
      for (int j = 0; j < EB; ++j) {
        const int q = q0 + kb + 4 * j;
        WT w{};
        if (m < R && q < Q) w = Wb[(int64_t)q * d.M + m];
        b[j] = w;
      }
    } else {  // W(m', k'), m' contiguous: m' = tid % KC, k' = tid / KC + j * (256 / KC)
      const int mr = q0 + tid % KC, kp = tid / KC;
#pragma unroll
      for (int j = 0; j < EB; ++j) {
        const int kout = r0 + kp + j * (256 / KC);
        WT w{};
        if (kout < R && mr < Q) w = Wb[(int64_t)kout * d.M + mr];
        b[j] = w;
      }
    }
  }
};

// ------------------------------------------------------------------ FP32
// Wave layout: 4 waves; wave w covers right-hand sides wn = (w % 2) * TNV / 2
// (NS = TNV / 64 subtiles of 32) and real columns wm = (w / 2) * 64.
template <bool ADJ, int TNV, int KC, bool PF>
__global__ __launch_bounds__(256) void k_stage_f32(const BlockDesc* __restrict__ blk,
                                                   const float2* __restrict__ W,
                                                   const float2* __restrict__ in, int64_t ld_in,
                                                   float2* __restrict__ out, int64_t ld_out, int nrhs,
                                                   const float* __restrict__ scale, int mtiles, int ntiles,
                                                   int64_t total) {
  constexpr int P = KC + 4;
  constexpr int NS = TNV / 64;
  __shared__ __attribute__((aligned(16))) float As[2][TNV][P];     // [re|im][n][k]
  __shared__ __attribute__((aligned(16))) float Bs[2][2 * TM][P];  // [c][real col][k]
  const Tile tl = map_tile(total, mtiles, ntiles);
  if (tl.b < 0) return;
  const BlockDesc d = blk[tl.b];
  const int R = ADJ ? d.K : d.M;
  const int Q = ADJ ? d.M : d.K;
  const int r0 = tl.mt * TM;
  if (r0 >= R) return;
  const int n0 = tl.nt * TNV;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wn = (wave & 1) * (TNV / 2), wm = (wave >> 1) * 64;
  const float2* Wb = W + d.w_off;
  // Two-level summation: the matrix cores sum one chunk into p, which is then
  // added to the running sums; the rounding error grows with the chunk
  // length plus the number of chunks instead of with the full reduction.
  v16f acc[NS][2];
#pragma unroll
  for (int a = 0; a < NS; ++a) acc[a][0] = acc[a][1] = v16f{};
  Loader<TNV, KC, ADJ, float2> ld;
  if (PF) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, 0, nrhs);
  for (int q0 = 0; q0 < Q; q0 += KC) {
    if (!PF) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, q0, nrhs);
    {  // registers -> LDS
      const int k = tid % KC, n = tid / KC;
#pragma unroll
      for (int j = 0; j < Loader<TNV, KC, ADJ, float2>::EA; ++j) {
        As[0][n + j * (256 / KC)][k] = ld.a[j].x;
        As[1][n + j * (256 / KC)][k] = ld.a[j].y;
      }
      if (!ADJ) {
        const int c = 2 * (tid & 63), kb = tid >> 6;
#pragma unroll
        for (int j = 0; j < Loader<TNV, KC, ADJ, float2>::EB; ++j) {
          const float2 w = ld.b[j];
          const int kk = kb + 4 * j;
          Bs[0][c][kk] = w.x;
          Bs[0][c + 1][kk] = w.y;
          Bs[1][c][kk] = -w.y;
          Bs[1][c + 1][kk] = w.x;
        }
      } else {
        const int mr = tid % KC, kp = tid / KC;
#pragma unroll
        for (int j = 0; j < Loader<TNV, KC, ADJ, float2>::EB; ++j) {
          const float2 w = ld.b[j];
          const int c = 2 * (kp + j * (256 / KC));
          Bs[0][c][mr] = w.x;
          Bs[0][c + 1][mr] = -w.y;
          Bs[1][c][mr] = w.y;
          Bs[1][c + 1][mr] = w.x;
        }
      }
    }
    __syncthreads();
    if (PF && q0 + KC < Q) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, q0 + KC, nrhs);
    const int kk = lane >> 5, li = lane & 31;
    v16f p[NS][2];
#pragma unroll
    for (int a = 0; a < NS; ++a) p[a][0] = p[a][1] = v16f{};
#pragma unroll
    for (int kb = 0; kb < KC; kb += 4) {
      float4 av[NS], bv[2];
#pragma unroll
      for (int a = 0; a < NS; ++a) av[a] = *reinterpret_cast<const float4*>(&As[kk][wn + 32 * a + li][kb]);
#pragma unroll
      for (int c = 0; c < 2; ++c) bv[c] = *reinterpret_cast<const float4*>(&Bs[kk][wm + 32 * c + li][kb]);
#pragma unroll
      for (int a = 0; a < NS; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          p[a][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].x, bv[c].x, p[a][c], 0, 0, 0);
          p[a][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].y, bv[c].y, p[a][c], 0, 0, 0);
          p[a][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].z, bv[c].z, p[a][c], 0, 0, 0);
          p[a][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].w, bv[c].w, p[a][c], 0, 0, 0);
        }
    }
#pragma unroll
    for (int a = 0; a < NS; ++a) {
      acc[a][0] += p[a][0];
      acc[a][1] += p[a][1];
    }
    __syncthreads();
  }
  store_out<ADJ, NS>(d, R, r0, n0, acc, wn, wm, out, ld_out, nrhs, scale);
}

// ------------------------------------------------------------------ BF16 x3
// LDS rows hold interleaved pairs along the complex reduction index: entry
// (row, k) is one 32-bit word = two BF16 values (real-k 2k and 2k+1).  The
// split products carry ~2^-16 relative error, so the partial sums go straight
// into the matrix-core accumulators (no compensation).
template <bool ADJ, int TNV, int KC, bool PF>
__global__ __launch_bounds__(256) void k_stage_bf16x3(const BlockDesc* __restrict__ blk,
                                                      const uint2* __restrict__ W,  // (re_hi,im_hi | re_lo,im_lo)
                                                      const float2* __restrict__ in, int64_t ld_in,
                                                      float2* __restrict__ out, int64_t ld_out, int nrhs,
                                                      const float* __restrict__ scale, int mtiles, int ntiles,
                                                      int64_t total) {
  constexpr int P = KC + 4;  // words per LDS row (16-byte aligned rows)
  constexpr int NS = TNV / 64;
  __shared__ __attribute__((aligned(16))) uint32_t Ah[TNV][P], Al[TNV][P];
  __shared__ __attribute__((aligned(16))) uint32_t Bh[2 * TM][P], Bl[2 * TM][P];
  const Tile tl = map_tile(total, mtiles, ntiles);
  if (tl.b < 0) return;
  const BlockDesc d = blk[tl.b];
  const int R = ADJ ? d.K : d.M;
  const int Q = ADJ ? d.M : d.K;
  const int r0 = tl.mt * TM;
  if (r0 >= R) return;
  const int n0 = tl.nt * TNV;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wn = (wave & 1) * (TNV / 2), wm = (wave >> 1) * 64;
  const uint2* Wb = W + d.w_off;
  v16f acc[NS][2];
#pragma unroll
  for (int a = 0; a < NS; ++a) acc[a][0] = acc[a][1] = v16f{};
  Loader<TNV, KC, ADJ, uint2> ld;
  if (PF) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, 0, nrhs);
  for (int q0 = 0; q0 < Q; q0 += KC) {
    if (!PF) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, q0, nrhs);
    {  // registers -> LDS (state split into BF16 hi/lo here)
      const int k = tid % KC, n = tid / KC;
#pragma unroll
      for (int j = 0; j < Loader<TNV, KC, ADJ, uint2>::EA; ++j) {
        uint32_t rh, rl, ih, il;
        split_bf(ld.a[j].x, rh, rl);
        split_bf(ld.a[j].y, ih, il);
        Ah[n + j * (256 / KC)][k] = rh | (ih << 16);
        Al[n + j * (256 / KC)][k] = rl | (il << 16);
      }
      if (!ADJ) {
        const int c = 2 * (tid & 63), kb = tid >> 6;
#pragma unroll
        for (int j = 0; j < Loader<TNV, KC, ADJ, uint2>::EB; ++j) {
          const uint2 w = ld.b[j];
          const int kk = kb + 4 * j;
          const uint32_t reh = w.x & 0xffffu, imh = w.x >> 16, rel = w.y & 0xffffu, iml = w.y >> 16;
          // column 2m (real part): (Wr, -Wi);  column 2m+1 (imag part): (Wi, Wr)
          Bh[c][kk] = reh | ((imh ^ 0x8000u) << 16);
          Bh[c + 1][kk] = imh | (reh << 16);
          Bl[c][kk] = rel | ((iml ^ 0x8000u) << 16);
          Bl[c + 1][kk] = iml | (rel << 16);
        }
      } else {
        const int mr = tid % KC, kp = tid / KC;
#pragma unroll
        for (int j = 0; j < Loader<TNV, KC, ADJ, uint2>::EB; ++j) {
          const uint2 w = ld.b[j];
          const int c = 2 * (kp + j * (256 / KC));
          const uint32_t reh = w.x & 0xffffu, imh = w.x >> 16, rel = w.y & 0xffffu, iml = w.y >> 16;
          // conj(W): column 2k' (real part): (Wr, Wi);  column 2k'+1 (imag part): (-Wi, Wr)
          Bh[c][mr] = reh | (imh << 16);
          Bh[c + 1][mr] = (imh ^ 0x8000u) | (reh << 16);
          Bl[c][mr] = rel | (iml << 16);
          Bl[c + 1][mr] = (iml ^ 0x8000u) | (rel << 16);
        }
      }
    }
    __syncthreads();
    if (PF && q0 + KC < Q) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, q0 + KC, nrhs);
    const int kh = lane >> 5, li = lane & 31;
#pragma unroll
    for (int kb = 0; kb < KC; kb += 8) {
      // lane holds real-k 8*kh .. 8*kh+7 of this step = complex k kb + 4*kh .. +3
      const int ko = kb + 4 * kh;
      bf16x8 ah[NS], al[NS], bh[2], bl[2];
#pragma unroll
      for (int a = 0; a < NS; ++a) {
        ah[a] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Ah[wn + 32 * a + li][ko]));
        al[a] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Al[wn + 32 * a + li][ko]));
      }
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        bh[c] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Bh[wm + 32 * c + li][ko]));
        bl[c] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Bl[wm + 32 * c + li][ko]));
      }
#pragma unroll
      for (int a = 0; a < NS; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          acc[a][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[c], acc[a][c], 0, 0, 0);
          acc[a][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[c], acc[a][c], 0, 0, 0);
          acc[a][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[c], acc[a][c], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  store_out<ADJ, NS>(d, R, r0, n0, acc, wn, wm, out, ld_out, nrhs, scale);
}

}  // namespace

bool use_mfma(const DevPart&, int, int64_t nrhs, int prec) {
  if (prec == MBF_C64_SPLIT_BF16) return true;
  if (prec == MBF_C64) return nrhs >= 32;
  return false;
}

// ------------------------------------------------------------------ autotuner
// Variant choice per (precision, direction, output-rows bucket, reduction
// bucket, RHS tiles).  Filled by autotune_stage (timing every variant on the
// stage's real shape) and optionally persisted as text lines
// "prec adj rb qb nb variant" in the file named by MBF_TUNE_FILE.
namespace {
using TuneKey = std::tuple<int, int, int, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;
bool g_tune_loaded = false;

TuneKey tune_key(int prec, bool adj, int R, int Q, int nrhs) {
  return TuneKey{prec, adj ? 1 : 0, (R + 63) / 64, (Q + 63) / 64, (nrhs + TN - 1) / TN};
}

void load_tune_file_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("MBF_TUNE_FILE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  int a, b, c, d, e, v;
  while (std::fscanf(f, "%d %d %d %d %d %d", &a, &b, &c, &d, &e, &v) == 6)
    if (v >= 0 && v < kNumVariants) g_tune[TuneKey{a, b, c, d, e}] = v;
  std::fclose(f);
}
}  // namespace

int tuned_variant(int prec, bool adj, int R, int Q, int nrhs) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  load_tune_file_locked();
  auto it = g_tune.find(tune_key(prec, adj, R, Q, nrhs));
  if (it != g_tune.end()) return it->second;
  if (const char* e = std::getenv("MBF_STAGE_VARIANT")) {
    const int v = std::atoi(e);
    if (v >= 0 && v < kNumVariants) return v;
  }
  return prec == MBF_C64 ? 0 : 3;
}

// Kernel variants (RHS tile, reduction chunk, register prefetch):
//   0 = (64, 16, off)  1 = (64, 16, on)  2 = (64, 32, off)  3 = (64, 32, on)
//   4 = (128, 16, on)  5 = (128, 32, on)
static int variant_tn(int v) { return v >= 4 ? 128 : 64; }

template <bool ADJ>
static void launch_variant(int prec, int v, dim3 grid, hipStream_t st, const BlockDesc* blk, const void* W,
                           const float2* x, int64_t ld_in, float2* y, int64_t ld_out, int nrhs, const float* scale,
                           int mtiles, int ntiles, int64_t total) {
#define MBF_LAUNCH(KER, WT, TNV, KCV, PFV)                                                                    \
  hipLaunchKernelGGL((KER<ADJ, TNV, KCV, PFV>), grid, dim3(256), 0, st, blk, reinterpret_cast<const WT*>(W), x, \
                     ld_in, y, ld_out, nrhs, scale, mtiles, ntiles, total)
  if (prec == MBF_C64) {
    switch (v) {
      case 0: MBF_LAUNCH(k_stage_f32, float2, 64, 16, false); break;
      case 1: MBF_LAUNCH(k_stage_f32, float2, 64, 16, true); break;
      case 2: MBF_LAUNCH(k_stage_f32, float2, 64, 32, false); break;
      case 3: MBF_LAUNCH(k_stage_f32, float2, 64, 32, true); break;
      case 4: MBF_LAUNCH(k_stage_f32, float2, 128, 16, true); break;
      default: MBF_LAUNCH(k_stage_f32, float2, 128, 32, true); break;
    }
  } else {
    switch (v) {
      case 0: MBF_LAUNCH(k_stage_bf16x3, uint2, 64, 16, false); break;
      case 1: MBF_LAUNCH(k_stage_bf16x3, uint2, 64, 16, true); break;
      case 2: MBF_LAUNCH(k_stage_bf16x3, uint2, 64, 32, false); break;
      case 3: MBF_LAUNCH(k_stage_bf16x3, uint2, 64, 32, true); break;
      case 4: MBF_LAUNCH(k_stage_bf16x3, uint2, 128, 16, true); break;
      default: MBF_LAUNCH(k_stage_bf16x3, uint2, 128, 32, true); break;
    }
  }
#undef MBF_LAUNCH
}

Error launch_stage_mfma(const DevPart& P, int s, int prec, bool adj, const BlockDesc* blk, const void* W,
                        const void* in, int64_t ld_in, void* out, int64_t ld_out, int nrhs, const float* scale,
                        hipStream_t st, int force_variant) {
  const int Rmax = adj ? P.max_K[s] : P.max_M[s];
  const int Qmax = adj ? P.max_M[s] : P.max_K[s];
  if (prec != MBF_C64 && prec != MBF_C64_SPLIT_BF16) return {MBF_ERR_UNSUPPORTED, "no MFMA stage kernel"};
  const int v = force_variant >= 0 ? force_variant : tuned_variant(prec, adj, Rmax, Qmax, nrhs);
  const int tn = variant_tn(v);
  const int mtiles = std::max(1, (Rmax + TM - 1) / TM);
  const int ntiles = (nrhs + tn - 1) / tn;
  const int64_t total = (int64_t)P.nblk[s] * mtiles * ntiles;
  const int64_t grid = (total + kXcd - 1) / kXcd * kXcd;
  if (grid > INT32_MAX) return {MBF_ERR_UNSUPPORTED, "stage grid too large"};
  const float2* x = reinterpret_cast<const float2*>(in);
  float2* y = reinterpret_cast<float2*>(out);
  if (adj)
    launch_variant<true>(prec, v, dim3((unsigned)grid), st, blk, W, x, ld_in, y, ld_out, nrhs, scale, mtiles, ntiles,
                         total);
  else
    launch_variant<false>(prec, v, dim3((unsigned)grid), st, blk, W, x, ld_in, y, ld_out, nrhs, scale, mtiles, ntiles,
                          total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return {MBF_ERR_HIP, std::string("stage launch: ") + hipGetErrorString(e)};
  return {MBF_OK, ""};
}

}  // namespace mbf

namespace mbf {

Error autotune_stage(const DevPart& P, int s, int prec, bool adj, const BlockDesc* blk, const void* W,
                     const void* in, int64_t ld_in, void* out, int64_t ld_out, int nrhs, hipStream_t st,
                     int* chosen, float* best_ms) {
  const int Rmax = adj ? P.max_K[s] : P.max_M[s];
  const int Qmax = adj ? P.max_M[s] : P.max_K[s];
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return {MBF_ERR_HIP, "hipEventCreate"};
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return {MBF_ERR_HIP, "hipEventCreate"};
  }
  int best = -1;
  float bt = 0.f;
  Error err{MBF_OK, ""};
  for (int v = 0; v < kNumVariants && err.st == MBF_OK; ++v) {
    err = launch_stage_mfma(P, s, prec, adj, blk, W, in, ld_in, out, ld_out, nrhs, nullptr, st, v);
    if (err.st != MBF_OK) break;
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < 2 && err.st == MBF_OK; ++r)
      err = launch_stage_mfma(P, s, prec, adj, blk, W, in, ld_in, out, ld_out, nrhs, nullptr, st, v);
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) {
      err = {MBF_ERR_HIP, "autotune timing"};
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (best < 0 || ms < bt) {
      best = v;
      bt = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err.st != MBF_OK) return err;
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    load_tune_file_locked();
    const TuneKey k = tune_key(prec, adj, Rmax, Qmax, nrhs);
    g_tune[k] = best;
    if (const char* path = std::getenv("MBF_TUNE_FILE")) {
      if (FILE* f = std::fopen(path, "a")) {
        std::fprintf(f, "%d %d %d %d %d %d\n", std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k),
                     std::get<4>(k), best);
        std::fclose(f);
      }
    }
  }
  if (chosen) *chosen = best;
  if (best_ms) *best_ms = bt / 2.f;
  return {MBF_OK, ""};
}

}  // namespace mbf
