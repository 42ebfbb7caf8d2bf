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

constexpr int kTuneRhs = 64;  // right-hand-side bucket of the tuning key
constexpr int kXcd = 8;       // XCDs per device

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

// Tile shape of a kernel variant: TNV right-hand sides x TMV complex output
// rows per workgroup of NTH threads; each wave owns RT x CT matrix-core tiles
// of 32 right-hand sides x 32 real columns; the reduction runs in chunks of
// KC complex entries, with register prefetch of the next chunk when PF.
template <int TNV_, int TMV_, int NTH_, int RT_, int CT_, int KC_, bool PF_>
struct Shape {
  static constexpr int TNV = TNV_, TMV = TMV_, NTH = NTH_, RT = RT_, CT = CT_, KC = KC_;
  static constexpr bool PF = PF_;
  static constexpr int WR = TNV / (32 * RT);      // waves along right-hand sides
  static constexpr int WC = 2 * TMV / (32 * CT);  // waves along real columns
  static_assert(WR * WC * 64 == NTH, "the waves must cover the tile");
  static constexpr int EA = TNV * KC / NTH;  // state entries per thread per chunk
  static constexpr int EB = TMV * KC / NTH;  // block entries per thread per chunk
  static_assert(EA * NTH == TNV * KC && EB * NTH == TMV * KC, "load mapping");
  static_assert(NTH % KC == 0 && NTH % TMV == 0 && KC % (NTH / TMV) == 0, "load mapping");
  static constexpr int P = KC + 4;  // LDS row pitch in words (16-byte aligned rows)
};

// Store the wave's RT x CT accumulator tiles (32 x 32 real each): rows are
// right-hand sides wn + 32 a + (MFMA row), columns real output columns
// wm + 32 c + (lane % 32); lanes of a row write consecutive floats.
template <bool ADJ, int RT, int CT>
__device__ __forceinline__ void store_out(const BlockDesc& d, int R, int r0, int n0, const v16f (&acc)[RT][CT],
                                          int wn, int wm, float2* __restrict__ out, int64_t ld_out, int nrhs,
                                          const float* __restrict__ scale) {
  const int lane = threadIdx.x & 63;
  float* o = reinterpret_cast<float*>(out);
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    const int col = wm + c * 32 + (lane & 31);  // real output column
    const int m = r0 + (col >> 1);
    if (m >= R) continue;
    const int32_t row = ADJ ? d.in_row + m : grp_row(d, m);
    const float sc = scale ? scale[row] : 1.0f;
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int n = n0 + wn + 32 * a + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
        if (n < nrhs) o[2 * ((int64_t)n * ld_out + row) + (col & 1)] = acc[a][c][j] * sc;
      }
  }
}

// ------------------------------------------------------------------ loads
// Each chunk moves a TNV x KC tile of the input state (A) and a KC x TMV
// tile of the block (B) into registers, with consecutive lanes on
// consecutive memory (the reduction index for A and for the adjoint's B, the
// output index for the forward B).  With PF the registers for the next chunk
// are loaded while the matrix cores work on the current one.
//   A:             k = tid % KC,  n = tid / KC + j (NTH / KC)
//   B (forward):   m = tid % TMV, k = tid / TMV + j (NTH / TMV)
//   B (adjoint):   m' = tid % KC, k' = tid / KC + j (NTH / KC)
template <class S, bool ADJ, typename WT>
struct Loader {
  float2 a[S::EA];
  WT b[S::EB];
  __device__ __forceinline__ void load(const BlockDesc& d, const float2* __restrict__ in, int64_t ld_in,
                                       const WT* __restrict__ Wb, int R, int Q, int r0, int n0, int q0,
                                       int nrhs) {
    constexpr int KC = S::KC, NTH = S::NTH, TMV = S::TMV;
    const int tid = threadIdx.x;
    {
      const int k = tid % KC, n = tid / KC;
      const int q = q0 + k;
      int32_t row = 0;
      if (q < Q) row = ADJ ? grp_row(d, q) : d.in_row + q;
#pragma unroll
      for (int j = 0; j < S::EA; ++j) {
        const int gn = n0 + n + j * (NTH / KC);
        float2 v = make_float2(0.f, 0.f);
        if (gn < nrhs && q < Q) v = in[(int64_t)gn * ld_in + row];
        a[j] = v;
      }
    }
    if (!ADJ) {
      const int m = r0 + tid % TMV, kb = tid / TMV;
#pragma unroll
      for (int j = 0; j < S::EB; ++j) {
        const int q = q0 + kb + j * (NTH / TMV);
        WT w{};
        if (m < R && q < Q) w = Wb[(int64_t)q * d.M + m];
        b[j] = w;
      }
    } else {
      const int mr = q0 + tid % KC, kp = tid / KC;
#pragma unroll
      for (int j = 0; j < S::EB; ++j) {
        const int kout = r0 + kp + j * (NTH / KC);
        WT w{};
        if (kout < R && mr < Q) w = Wb[(int64_t)kout * d.M + mr];
        b[j] = w;
      }
    }
  }
};

// ------------------------------------------------------------------ FP32
// Wave w covers right-hand sides wn = (w % WR) * 32 RT and real columns
// wm = (w / WR) * 32 CT.
template <bool ADJ, class S>
__global__ __launch_bounds__(S::NTH) void k_stage_f32(const BlockDesc* __restrict__ blk,
                                                      const float2* __restrict__ W,
                                                      const float2* __restrict__ in, int64_t ld_in,
                                                      float2* __restrict__ out, int64_t ld_out, int nrhs,
                                                      const float* __restrict__ scale, int mtiles, int ntiles,
                                                      int64_t total) {
  constexpr int KC = S::KC, NTH = S::NTH, TMV = S::TMV, P = S::P, RT = S::RT, CT = S::CT;
  __shared__ __attribute__((aligned(16))) float As[2][S::TNV][P];  // [re|im][n][k]
  __shared__ __attribute__((aligned(16))) float Bs[2][2 * TMV][P];  // [c][real col][k]
  const Tile tl = map_tile(total, mtiles, ntiles);
  if (tl.b < 0) return;
  const BlockDesc d = blk[tl.b];
  const int R = ADJ ? d.K : d.M;
  const int Q = ADJ ? d.M : d.K;
  const int r0 = tl.mt * TMV;
  if (r0 >= R) return;
  const int n0 = tl.nt * S::TNV;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wn = (wave % S::WR) * 32 * RT, wm = (wave / S::WR) * 32 * CT;
  const float2* Wb = W + d.w_off;
  // Two-level summation: the matrix cores sum one chunk into p, which is then
  // added to the running sums; the rounding error grows with the chunk
  // length plus the number of chunks instead of with the full reduction.
  v16f acc[RT][CT];
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[a][c] = v16f{};
  Loader<S, ADJ, float2> ld;
  if (S::PF) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, 0, nrhs);
  for (int q0 = 0; q0 < Q; q0 += KC) {
    if (!S::PF) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, q0, nrhs);
    {  // registers -> LDS
      const int k = tid % KC, n = tid / KC;
#pragma unroll
      for (int j = 0; j < S::EA; ++j) {
        As[0][n + j * (NTH / KC)][k] = ld.a[j].x;
        As[1][n + j * (NTH / KC)][k] = ld.a[j].y;
      }
      if (!ADJ) {
        const int c = 2 * (tid % TMV), kb = tid / TMV;
#pragma unroll
        for (int j = 0; j < S::EB; ++j) {
          const float2 w = ld.b[j];
          const int kk = kb + j * (NTH / TMV);
          Bs[0][c][kk] = w.x;
          Bs[0][c + 1][kk] = w.y;
          Bs[1][c][kk] = -w.y;
          Bs[1][c + 1][kk] = w.x;
        }
      } else {
        const int mr = tid % KC, kp = tid / KC;
#pragma unroll
        for (int j = 0; j < S::EB; ++j) {
          const float2 w = ld.b[j];
          const int c = 2 * (kp + j * (NTH / KC));
          Bs[0][c][mr] = w.x;
          Bs[0][c + 1][mr] = -w.y;
          Bs[1][c][mr] = w.y;
          Bs[1][c + 1][mr] = w.x;
        }
      }
    }
    __syncthreads();
    if (S::PF && q0 + KC < Q) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, q0 + KC, nrhs);
    const int kk = lane >> 5, li = lane & 31;
    v16f p[RT][CT];
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int c = 0; c < CT; ++c) p[a][c] = v16f{};
#pragma unroll
    for (int kb = 0; kb < KC; kb += 4) {
      float4 av[RT], bv[CT];
#pragma unroll
      for (int a = 0; a < RT; ++a) av[a] = *reinterpret_cast<const float4*>(&As[kk][wn + 32 * a + li][kb]);
#pragma unroll
      for (int c = 0; c < CT; ++c) bv[c] = *reinterpret_cast<const float4*>(&Bs[kk][wm + 32 * c + li][kb]);
#pragma unroll
      for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int c = 0; c < CT; ++c) {
          p[a][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].x, bv[c].x, p[a][c], 0, 0, 0);
          p[a][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].y, bv[c].y, p[a][c], 0, 0, 0);
          p[a][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].z, bv[c].z, p[a][c], 0, 0, 0);
          p[a][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].w, bv[c].w, p[a][c], 0, 0, 0);
        }
    }
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[a][c] += p[a][c];
    __syncthreads();
  }
  store_out<ADJ, RT, CT>(d, R, r0, n0, acc, wn, wm, out, ld_out, nrhs, scale);
}

// ------------------------------------------------------------------ BF16 x3
// LDS rows hold interleaved pairs along the complex reduction index: entry
// (row, k) is one 32-bit word = two BF16 values (real-k 2k and 2k+1).  The
// split products carry ~2^-16 relative error, so the partial sums go straight
// into the matrix-core accumulators (no compensation).
template <bool ADJ, class S>
__global__ __launch_bounds__(S::NTH) void k_stage_bf16x3(const BlockDesc* __restrict__ blk,
                                                         const uint2* __restrict__ W,  // (re_hi,im_hi | re_lo,im_lo)
                                                         const float2* __restrict__ in, int64_t ld_in,
                                                         float2* __restrict__ out, int64_t ld_out, int nrhs,
                                                         const float* __restrict__ scale, int mtiles, int ntiles,
                                                         int64_t total) {
  constexpr int KC = S::KC, NTH = S::NTH, TMV = S::TMV, P = S::P, RT = S::RT, CT = S::CT;
  __shared__ __attribute__((aligned(16))) uint32_t Ah[S::TNV][P], Al[S::TNV][P];
  __shared__ __attribute__((aligned(16))) uint32_t Bh[2 * TMV][P], Bl[2 * TMV][P];
  const Tile tl = map_tile(total, mtiles, ntiles);
  if (tl.b < 0) return;
  const BlockDesc d = blk[tl.b];
  const int R = ADJ ? d.K : d.M;
  const int Q = ADJ ? d.M : d.K;
  const int r0 = tl.mt * TMV;
  if (r0 >= R) return;
  const int n0 = tl.nt * S::TNV;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wn = (wave % S::WR) * 32 * RT, wm = (wave / S::WR) * 32 * CT;
  const uint2* Wb = W + d.w_off;
  v16f acc[RT][CT];
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[a][c] = v16f{};
  Loader<S, ADJ, uint2> ld;
  if (S::PF) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, 0, nrhs);
  for (int q0 = 0; q0 < Q; q0 += KC) {
    if (!S::PF) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, q0, nrhs);
    {  // registers -> LDS (state split into BF16 hi/lo here)
      const int k = tid % KC, n = tid / KC;
#pragma unroll
      for (int j = 0; j < S::EA; ++j) {
        uint32_t rh, rl, ih, il;
        split_bf(ld.a[j].x, rh, rl);
        split_bf(ld.a[j].y, ih, il);
        Ah[n + j * (NTH / KC)][k] = rh | (ih << 16);
        Al[n + j * (NTH / KC)][k] = rl | (il << 16);
      }
      if (!ADJ) {
        const int c = 2 * (tid % TMV), kb = tid / TMV;
#pragma unroll
        for (int j = 0; j < S::EB; ++j) {
          const uint2 w = ld.b[j];
          const int kk = kb + j * (NTH / TMV);
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
        for (int j = 0; j < S::EB; ++j) {
          const uint2 w = ld.b[j];
          const int c = 2 * (kp + j * (NTH / KC));
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
    if (S::PF && q0 + KC < Q) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, q0 + KC, nrhs);
    const int kh = lane >> 5, li = lane & 31;
#pragma unroll
    for (int kb = 0; kb < KC; kb += 8) {
      // lane holds real-k 8*kh .. 8*kh+7 of this step = complex k kb + 4*kh .. +3
      const int ko = kb + 4 * kh;
      bf16x8 ah[RT], al[RT], bh[CT], bl[CT];
#pragma unroll
      for (int a = 0; a < RT; ++a) {
        ah[a] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Ah[wn + 32 * a + li][ko]));
        al[a] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Al[wn + 32 * a + li][ko]));
      }
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        bh[c] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Bh[wm + 32 * c + li][ko]));
        bl[c] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Bl[wm + 32 * c + li][ko]));
      }
#pragma unroll
      for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int c = 0; c < CT; ++c) {
          acc[a][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[c], acc[a][c], 0, 0, 0);
          acc[a][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[c], acc[a][c], 0, 0, 0);
          acc[a][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[c], acc[a][c], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  store_out<ADJ, RT, CT>(d, R, r0, n0, acc, wn, wm, out, ld_out, nrhs, scale);
}

// BF16 x3 with two LDS buffers: the registers of chunk i+1 are written to
// one buffer while the matrix cores read chunk i from the other, so one
// barrier per chunk separates the phases and the waves of a workgroup overlap
// their LDS writes with the other waves' matrix-core work.  Rows carry no
// padding; the 16-byte groups of a row are XOR-swizzled with bits 1..2 of
// the row index, which keeps 8 consecutive rows of a 16-byte read on
// distinct banks.
template <bool ADJ, class S>
__global__ __launch_bounds__(S::NTH) void k_stage_bf16x3_db(const BlockDesc* __restrict__ blk,
                                                            const uint2* __restrict__ W,
                                                            const float2* __restrict__ in, int64_t ld_in,
                                                            float2* __restrict__ out, int64_t ld_out, int nrhs,
                                                            const float* __restrict__ scale, int mtiles,
                                                            int ntiles, int64_t total) {
  constexpr int KC = S::KC, NTH = S::NTH, TMV = S::TMV, TNV = S::TNV, RT = S::RT, CT = S::CT;
  static_assert(KC == 16, "swizzle assumes four 16-byte groups per row");
  __shared__ __attribute__((aligned(16))) uint32_t Ah[2][TNV * KC], Al[2][TNV * KC];
  __shared__ __attribute__((aligned(16))) uint32_t Bh[2][2 * TMV * KC], Bl[2][2 * TMV * KC];
  auto sw = [](int r, int k) { return r * KC + ((((k >> 2) ^ (r >> 1)) & 3) << 2) + (k & 3); };
  const Tile tl = map_tile(total, mtiles, ntiles);
  if (tl.b < 0) return;
  const BlockDesc d = blk[tl.b];
  const int R = ADJ ? d.K : d.M;
  const int Q = ADJ ? d.M : d.K;
  const int r0 = tl.mt * TMV;
  if (r0 >= R) return;
  const int n0 = tl.nt * TNV;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wn = (wave % S::WR) * 32 * RT, wm = (wave / S::WR) * 32 * CT;
  const uint2* Wb = W + d.w_off;
  v16f acc[RT][CT];
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[a][c] = v16f{};
  Loader<S, ADJ, uint2> ld;
  auto stash = [&](int buf) {  // registers -> LDS buffer (state split into BF16 hi/lo)
    const int k = tid % KC, n = tid / KC;
#pragma unroll
    for (int j = 0; j < S::EA; ++j) {
      uint32_t rh, rl, ih, il;
      split_bf(ld.a[j].x, rh, rl);
      split_bf(ld.a[j].y, ih, il);
      const int e = sw(n + j * (NTH / KC), k);
      Ah[buf][e] = rh | (ih << 16);
      Al[buf][e] = rl | (il << 16);
    }
    if (!ADJ) {
      const int c = 2 * (tid % TMV), kb = tid / TMV;
#pragma unroll
      for (int j = 0; j < S::EB; ++j) {
        const uint2 w = ld.b[j];
        const int kk = kb + j * (NTH / TMV);
        const uint32_t reh = w.x & 0xffffu, imh = w.x >> 16, rel = w.y & 0xffffu, iml = w.y >> 16;
        Bh[buf][sw(c, kk)] = reh | ((imh ^ 0x8000u) << 16);
        Bh[buf][sw(c + 1, kk)] = imh | (reh << 16);
        Bl[buf][sw(c, kk)] = rel | ((iml ^ 0x8000u) << 16);
        Bl[buf][sw(c + 1, kk)] = iml | (rel << 16);
      }
    } else {
      const int mr = tid % KC, kp = tid / KC;
#pragma unroll
      for (int j = 0; j < S::EB; ++j) {
        const uint2 w = ld.b[j];
        const int c = 2 * (kp + j * (NTH / KC));
        const uint32_t reh = w.x & 0xffffu, imh = w.x >> 16, rel = w.y & 0xffffu, iml = w.y >> 16;
        Bh[buf][sw(c, mr)] = reh | (imh << 16);
        Bh[buf][sw(c + 1, mr)] = (imh ^ 0x8000u) | (reh << 16);
        Bl[buf][sw(c, mr)] = rel | (iml << 16);
        Bl[buf][sw(c + 1, mr)] = (iml ^ 0x8000u) | (rel << 16);
      }
    }
  };
  ld.load(d, in, ld_in, Wb, R, Q, r0, n0, 0, nrhs);
  stash(0);
  if (KC < Q) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, KC, nrhs);
  __syncthreads();
  const int kh = lane >> 5, li = lane & 31;
  for (int q0 = 0, cur = 0; q0 < Q; q0 += KC, cur ^= 1) {
    // Buffer cur^1 was last read before the previous barrier: refill it.
    if (q0 + KC < Q) {
      stash(cur ^ 1);
      if (q0 + 2 * KC < Q) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, q0 + 2 * KC, nrhs);
    }
#pragma unroll
    for (int kb = 0; kb < KC; kb += 8) {
      const int ko = kb + 4 * kh;
      bf16x8 ah[RT], al[RT], bh[CT], bl[CT];
#pragma unroll
      for (int a = 0; a < RT; ++a) {
        const int e = sw(wn + 32 * a + li, ko);
        ah[a] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Ah[cur][e]));
        al[a] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Al[cur][e]));
      }
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const int e = sw(wm + 32 * c + li, ko);
        bh[c] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Bh[cur][e]));
        bl[c] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Bl[cur][e]));
      }
#pragma unroll
      for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int c = 0; c < CT; ++c) {
          acc[a][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[c], acc[a][c], 0, 0, 0);
          acc[a][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[c], acc[a][c], 0, 0, 0);
          acc[a][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[c], acc[a][c], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  store_out<ADJ, RT, CT>(d, R, r0, n0, acc, wn, wm, out, ld_out, nrhs, scale);
}

// Kernel variants: Shape<TNV, TMV, NTH, RT, CT, KC, PF>.
using V0 = Shape<64, 64, 256, 1, 2, 16, false>;
using V1 = Shape<64, 64, 256, 1, 2, 16, true>;
using V2 = Shape<64, 64, 256, 1, 2, 32, false>;
using V3 = Shape<64, 64, 256, 1, 2, 32, true>;
using V4 = Shape<128, 64, 256, 2, 2, 16, true>;
using V5 = Shape<128, 64, 256, 2, 2, 32, true>;
// FP32 with 8 waves (two accumulator sets per tile bound the wave tile).
using F6 = Shape<256, 64, 512, 2, 2, 16, true>;
using F7 = Shape<128, 128, 512, 2, 2, 16, true>;
// BF16 x3 with wide wave tiles (one accumulator set per tile).
using B6 = Shape<256, 128, 512, 2, 4, 16, true>;
using B7 = Shape<128, 128, 256, 2, 4, 16, true>;
// Double-buffered BF16 x3 (k_stage_bf16x3_db).
using B8 = Shape<256, 128, 512, 2, 4, 16, true>;
using B9 = Shape<128, 64, 256, 2, 2, 16, true>;

struct VariantDims {
  int tnv, tmv, nth;
};
template <class S>
constexpr VariantDims dims_of() {
  return {S::TNV, S::TMV, S::NTH};
}

VariantDims variant_dims(int prec, int v) {
  switch (v) {
    case 0: return dims_of<V0>();
    case 1: return dims_of<V1>();
    case 2: return dims_of<V2>();
    case 3: return dims_of<V3>();
    case 4: return dims_of<V4>();
    case 5: return dims_of<V5>();
    case 6: return prec == MBF_C64 ? dims_of<F6>() : dims_of<B6>();
    case 7: return prec == MBF_C64 ? dims_of<F7>() : dims_of<B7>();
    case 8: return prec == MBF_C64 ? dims_of<F7>() : dims_of<B8>();
    default: return prec == MBF_C64 ? dims_of<F7>() : dims_of<B9>();
  }
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
  return TuneKey{prec, adj ? 1 : 0, (R + 63) / 64, (Q + 63) / 64, (nrhs + kTuneRhs - 1) / kTuneRhs};
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
    if (v >= 0 && v < num_variants(a)) g_tune[TuneKey{a, b, c, d, e}] = v;
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
    if (v >= 0 && v < num_variants(prec)) return v;
  }
  return prec == MBF_C64 ? 0 : 3;
}

template <bool ADJ>
static void launch_variant(int prec, int v, dim3 grid, hipStream_t st, const BlockDesc* blk, const void* W,
                           const float2* x, int64_t ld_in, float2* y, int64_t ld_out, int nrhs, const float* scale,
                           int mtiles, int ntiles, int64_t total) {
#define MBF_LAUNCH(KER, WT, S)                                                                            \
  hipLaunchKernelGGL((KER<ADJ, S>), grid, dim3(S::NTH), 0, st, blk, reinterpret_cast<const WT*>(W), x, ld_in, \
                     y, ld_out, nrhs, scale, mtiles, ntiles, total)
  if (prec == MBF_C64) {
    switch (v) {
      case 0: MBF_LAUNCH(k_stage_f32, float2, V0); break;
      case 1: MBF_LAUNCH(k_stage_f32, float2, V1); break;
      case 2: MBF_LAUNCH(k_stage_f32, float2, V2); break;
      case 3: MBF_LAUNCH(k_stage_f32, float2, V3); break;
      case 4: MBF_LAUNCH(k_stage_f32, float2, V4); break;
      case 5: MBF_LAUNCH(k_stage_f32, float2, V5); break;
      case 6: MBF_LAUNCH(k_stage_f32, float2, F6); break;
      default: MBF_LAUNCH(k_stage_f32, float2, F7); break;
    }
  } else {
    switch (v) {
      case 0: MBF_LAUNCH(k_stage_bf16x3, uint2, V0); break;
      case 1: MBF_LAUNCH(k_stage_bf16x3, uint2, V1); break;
      case 2: MBF_LAUNCH(k_stage_bf16x3, uint2, V2); break;
      case 3: MBF_LAUNCH(k_stage_bf16x3, uint2, V3); break;
      case 4: MBF_LAUNCH(k_stage_bf16x3, uint2, V4); break;
      case 5: MBF_LAUNCH(k_stage_bf16x3, uint2, V5); break;
      case 6: MBF_LAUNCH(k_stage_bf16x3, uint2, B6); break;
      case 7: MBF_LAUNCH(k_stage_bf16x3, uint2, B7); break;
      case 8: MBF_LAUNCH(k_stage_bf16x3_db, uint2, B8); break;
      default: MBF_LAUNCH(k_stage_bf16x3_db, uint2, B9); break;
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
  const VariantDims vd = variant_dims(prec, v);
  const int mtiles = std::max(1, (Rmax + vd.tmv - 1) / vd.tmv);
  const int ntiles = (nrhs + vd.tnv - 1) / vd.tnv;
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
  for (int v = 0; v < num_variants(prec) && err.st == MBF_OK; ++v) {
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
